// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include "common.hpp"

namespace prism {

// transition constants: frame interval and per-step noise variances in the
// tangent order (dt, dtheta, dv, dw)
struct TransC {
    double dt;
    double du;   // factor of the control in the velocity update: dt, or dt^2 (the printed form)
    double q[15];   // (q[12..14]: the bias random walk of the 15-D state)
    double g[3];    // gravity (15-D state: the linear control is a body-frame specific force)
};

struct MapUpdC {
    float trunc32;          // decision: z <= D + trunc in single precision
    double trunc, lam_u;    // values
};

// ---------------------------------------------------------------------------
// batched steps over many filters (serving)
// ---------------------------------------------------------------------------
// Everything a kernel needs to run one filter's part of a batched step.  One
// copy lives in each filter's state buffer (device), written from the
// handle's host copy whenever it changes.
struct AgentDesc {
    GridC g;
    CamC c;
    GridD gd;
    CamD cd;
    WeightsC w;
    WeightsC w_irls;      // the weights of a Gauss-Newton iteration (w when the L1 mode is off)
    TransC tc;
    MapUpdC mp;
    MapAux aux;
    double ema;
    double lap_h;         // factor of H in the Laplace covariance (f H + Lp)^-1: 2, or 1
    double min_inliers;   // contributing pixels below which a step raises PRISM_FLAG_LOW_INLIERS
    float normal_disc;
    int dtype, n_gn, nseg, upd_groups;
    int obj_blocks;   // workgroups (reduction partials) of one objective evaluation: tracking (P2) or
                      // render-through (P1)
    void* map;
    const unsigned* bits;   // free-space bits for the renderer (NULL when tau != 0)
    prism_filter_state* S;
    prism_filter_bias_state* X;   // the 15-D state's bias part (NULL for the 12-D state)
    float *a_depth, *a_rgb, *a_normals;
    uint8_t *a_mask, *a_nmask;
    double* partials;
    Rel32* rel;   // relative pose of the current iterate to the anchor (predict / GN write it)
    prism_frame slots[4];
};

constexpr int kMaxBatch = 32;

// kernel argument of a batched launch: workgroups [start[a], start[a+1]) of
// the grid run filter a's part, reading its descriptor d[a] and input slot
// slot[a]
struct BatchArgs {
    const AgentDesc* d[kMaxBatch];
    int start[kMaxBatch + 1];
    unsigned char slot[kMaxBatch];
    int n;
    int irls;   // objective launches: 1 in Gauss-Newton iterations (rows weighted by w_irls), else 0
};

// filter of workgroup blk (the start table is uniform: a scalar search)
__device__ __forceinline__ int batch_agent(const BatchArgs& b, int blk) {
    int a = 0;
    while (a + 1 < b.n && b.start[a + 1] <= blk) ++a;
    return a;
}

// sources of the frames a batched step stages into the slots
struct StageSrc {
    const void* depth[kMaxBatch];
    const void* rgb[kMaxBatch];
    const void* u[kMaxBatch];
};

// Batched launchers: one launch per stage for all filters of the batch.
hipError_t launch_stage_batch(const BatchArgs& b, const StageSrc& src, hipStream_t st);
hipError_t launch_predict_batch(const BatchArgs& b, hipStream_t st);
hipError_t launch_track_p2_batch(const BatchArgs& b, hipStream_t st);
hipError_t launch_gn_step_batch(const BatchArgs& b, hipStream_t st);
hipError_t launch_laplace_combine_batch(const BatchArgs& b, hipStream_t st);
hipError_t launch_first_frame_batch(const BatchArgs& b, hipStream_t st);
hipError_t launch_cull_batch(const BatchArgs& b, hipStream_t st);
// recompute the dilated free-space bits of one map / of every map of a batch
hipError_t launch_dilate(const GridC& g, const MapAux& aux, hipStream_t st);
hipError_t launch_dilate_batch(const BatchArgs& b, hipStream_t st);
hipError_t launch_map_update_batch(const BatchArgs& b, int dtype, bool pool, int max_nseg, hipStream_t st);
hipError_t launch_render_batch(const BatchArgs& b, int dtype, bool pool, int max_lds_words, hipStream_t st);
// the render-through (P1) objective of every filter of the batch at its iterate
hipError_t launch_render_jac_batch(const BatchArgs& b, int dtype, bool pool, int max_lds_words, hipStream_t st);
hipError_t launch_normals_batch(const BatchArgs& b, hipStream_t st);
int stage_blocks(const CamC& c);

int render_blocks(const CamC& c);   // render, render_jacobian
int vjp_blocks(const CamC& c);      // render_vjp
int track_blocks(const CamC& c);

// bits: the map's free-space bits, or NULL to evaluate every sample (they are
// only passed when tau == 0, where skipping a brick whose occupancies are all
// <= 0 cannot change a decision)
hipError_t launch_render(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, int dtype, const void* map,
                         const unsigned* bits, const prism_pose* poses, int n_frames, float* depth, float* rgb,
                         uint8_t* mask, int32_t* hit_k, hipStream_t st);
// counts/ngroups/n_updated (nullable): also total the preceding map update's
// per-workgroup counts into *n_updated
hipError_t launch_normals(const CamC& c, int n_frames, const float* depth, const uint8_t* mask, float disc,
                          float* normals, uint8_t* nmask, const int* counts, int ngroups, int64_t* n_updated,
                          int64_t* n_updated_total, hipStream_t st);
hipError_t launch_render_jac(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, int dtype,
                             const void* map, const unsigned* bits, const prism_pose* poses, int n_frames,
                             const float* obs_depth,
                             const float* obs_rgb, const WeightsC& w, float* depth, float* rgb, uint8_t* mask,
                             float* J, float* resid, uint8_t* rowmask, double* partials, hipStream_t st);
hipError_t launch_render_vjp(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, const float* map,
                             const prism_pose* poses, int n_frames, const int32_t* hit_k, const float* g_depth,
                             const float* g_rgb, float* grad_mean, double* partials, hipStream_t st);
hipError_t launch_track_p2(const CamC& c, const CamD& cd, const prism_pose* pose, const prism_pose* pose_prev,
                           const float* obs_depth, const float* obs_rgb, const float* a_depth,
                           const float* a_rgb, const uint8_t* a_mask, const float* a_normals,
                           const uint8_t* a_nmask, const WeightsC& w, float* J, float* resid,
                           uint8_t* rowmask, double* partials, const Rel32* rel, hipStream_t st);
hipError_t launch_finalize(const double* partials, int nblocks, int n_frames, int nvals, double* out,
                           int stride, hipStream_t st);

hipError_t launch_map_init(const GridC& g, int dtype, void* map, float occ0, float rgb0, float var0,
                           const MapAux& aux, hipStream_t st);
hipError_t launch_brick_max(const GridC& g, int dtype, const void* map, const MapAux& aux, hipStream_t st);
hipError_t launch_from_dense(const GridC& g, int dtype, void* map, const float* mean4, const float* var4,
                             const MapAux& aux, hipStream_t st);
hipError_t launch_to_dense(const GridC& g, int dtype, const void* map, float* mean4, float* var4,
                           const MapAux& aux, hipStream_t st);
hipError_t launch_planes(int n, int channels, const float* src, float* dst, int to_dense, hipStream_t st);
// n_updated (nullable): total of updated voxels, by an extra one-workgroup
// kernel; t_begin / t_end (nullable): events recorded around the update kernel
hipError_t launch_map_update(const GridC& g, const CamC& c, const GridD& gd, int dtype, void* map,
                             const prism_pose* pose, const float* depth, const float* rgb, double trunc, double lam_u,
                             const MapAux& aux, int64_t* n_updated, hipStream_t st, hipEvent_t t_begin = nullptr,
                             hipEvent_t t_end = nullptr);
// workgroups (and per-workgroup counts) of one update launch, alone or
// within a batched launch
int map_update_groups(const GridC& g);
int map_update_groups_batch(const GridC& g);

// descent mapping (gradient pass, step on marked bricks, cost total)
// list: [0] number of bricks, then the bricks, in the order first touched
hipError_t launch_gd_grad(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, const float* map,
                          const unsigned* bits, const prism_pose* pose, const float* obs_depth, const float* obs_rgb,
                          const WeightsC& w, double* grad, unsigned* marks, int* list, double* partials,
                          hipStream_t st);
hipError_t launch_gd_update(const GridC& g, float* map, const MapAux& aux, float* save, double* grad,
                            const int* list, unsigned* saved, double lr_occ, double lr_rgb, double* partials,
                            hipStream_t st);
hipError_t launch_gd_cost(const double* pd, int nd, const double* pp, int np, double* cost, hipStream_t st);
hipError_t launch_gd_clear(unsigned* words, int n, hipStream_t st);
int gd_update_groups(const GridC& g);

// frame staging: depth [npix] f32, rgb [3 npix] f32 and (if u) 6 f64 copied
// into a serving slot in one kernel
hipError_t launch_stage(const void* depth, const void* rgb, const void* u, float* d_out, float* c_out, double* u_out,
                        long long npix, hipStream_t st);

// Adam (first moment off) on sampled pixels of the P2 objective
struct AdamC {
    double lr[6];              // step size per component (translation x3, rotation x3)
    double beta2, eps, scale;  // scale: image pixels / pixels per step
    int n_steps, n_pix;
};
hipError_t launch_pose_adam(prism_filter_state* S, const CamC& c, const CamD& cd, const float* obs_depth,
                            const float* obs_rgb, const float* a_depth, const float* a_rgb, const uint8_t* a_mask,
                            const float* a_normals, const uint8_t* a_nmask, const WeightsC& w, const int32_t* pixels,
                            const AdamC& ad, hipStream_t st);

// predictive rollouts: sampled trajectories (n_samples x k poses) and the
// closed-form predicted moments (nullable mean [k][13], cov [k][144]; for the
// 15-D state, X non-NULL, mean [k][16] and cov [k][225])
hipError_t launch_rollout(const prism_filter_state* S, const prism_filter_bias_state* X, const double* u, int k,
                          int n_samples, const double* noise,
                          const TransC& tc, prism_pose* poses, double* mean, double* cov, int32_t* flags,
                          hipStream_t st);
hipError_t launch_predict(prism_filter_state* S, prism_filter_bias_state* X, const double* u, const TransC& tc,
                          Rel32* rel, hipStream_t st);
hipError_t launch_gn_step(prism_filter_state* S, const double* partials, int nblocks, Rel32* rel, hipStream_t st);
hipError_t launch_laplace_combine(prism_filter_state* S, prism_filter_bias_state* X, const double* partials,
                                  int nblocks, double ema, double min_inliers, double lap_h, hipStream_t st);
// the left, world-frame retraction t <- t + dt, R <- Exp(dtheta) R of n poses
hipError_t launch_pose_retract(const prism_pose* poses, const double* delta, int n, prism_pose* out, hipStream_t st);
hipError_t launch_first_frame(prism_filter_state* S, hipStream_t st);

}  // namespace prism
