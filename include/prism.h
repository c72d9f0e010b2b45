/*
 * prism.h -- C ABI of the MI355X (gfx950) PRISM filter hot path.
 *
 * Paper: A. Mirchev, B. Kayalibay, A. Agha, P. van der Smagt, D. Cremers,
 * J. Bayer, "PRISM: Probabilistic Real-Time Inference in Spatial World
 * Models", CoRL 2022 (arXiv 2212.02988).
 *
 * The library computes, on one GPU, the data-parallel steps of the paper's
 * approximate marginal filters:
 *   - the ray-marching RGB-D emission from the voxel map        (App. B)
 *   - its 6-DoF pose Jacobian reduced to normal equations       (Sec. 4.3.2)
 *   - the prediction-to-observation tracking objective          (App. E.3)
 *   - Gauss-Newton MAP pose, Laplace covariance, linear-Gaussian
 *     propagation / split / combination of the state belief     (App. E.1-E.3)
 *   - the closed-form per-voxel Gaussian map update             (App. D)
 *   - the adjoint of the emission w.r.t. voxel means and pose
 *
 * Conventions shared by every call
 * --------------------------------
 * World frame right-handed.  A pose is 7 doubles (t[3], q[4] = w,x,y,z),
 * camera -> world: X_w = R(q) X_c + t (q need not be normalised; it is
 * normalised on use).  Camera frame: x right, y down, z forward.  Pixel
 * (u, v) has centre (u + 1/2, v + 1/2) and looks along
 * ((u + 1/2 - cx)/fx, (v + 1/2 - cy)/fy, 1): rendered and observed depths are
 * z-depths.  Sample k of a ray (k = 0..K-1) is at depth
 * d_near + k (d_far - d_near)/(K - 1).  A pose perturbation delta =
 * (dt, dtheta) acts as t <- t + dt, R <- Exp(dtheta) R (world frame); all
 * Jacobians and covariances are in that tangent.
 *
 * The voxel map holds per voxel and channel (occupancy = -SDF, R, G, B) a
 * Gaussian mean and variance.  Voxel (i, j, k) has its centre at
 * origin + voxel * (i + 1/2, j + 1/2, k + 1/2).  Trilinear interpolation
 * uses the 8 surrounding centres; corners outside the grid take the values
 * occ_out / rgb_out (the paper's first map belief, App. G).
 *
 * Memory: the library never allocates device memory.  Every pointer named
 * "device" must point to device memory the caller owns and keeps alive until
 * the call's work on `stream` has completed.  Calls are asynchronous on
 * `stream` (NULL = the default stream); outputs are valid once the stream is
 * synchronised.  Numeric conditions (no valid pixel, a non positive-definite
 * system) never fail a call: they are reported in device-side flags.
 *
 * Errors: every call returns a prism_status.  Non-zero values leave outputs
 * untouched and set a thread-local message readable with prism_last_error().
 */
#ifndef PRISM_H
#define PRISM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t prism_status;
#define PRISM_OK 0
#define PRISM_INVALID_ARGUMENT 1 /* null pointer, bad size, misaligned buffer */
#define PRISM_UNSUPPORTED 2      /* dtype / shape outside the supported set */
#define PRISM_HIP_ERROR 3        /* a HIP runtime call failed (message has the code) */
#define PRISM_BUSY 4             /* every input slot of the handle holds a step still running */
#define PRISM_CAPTURE_ERROR 5    /* a HIP graph could not be recorded or instantiated, or the call
                                    cannot run on a stream that is being captured */

/* Map storage types. */
#define PRISM_F32 0
#define PRISM_BF16 1

/* Device-side flags (prism_filter_state.flags). */
#define PRISM_FLAG_NO_VALID_PIXELS 1 /* an objective evaluation had no contributing pixel */
#define PRISM_FLAG_CHOL_FALLBACK 2   /* a normal matrix was not positive definite: the
                                        pose kept the prior mean and covariance */
#define PRISM_FLAG_PRIOR_NOT_PD 4    /* set with CHOL_FALLBACK when the predicted pose
                                        covariance itself was not positive definite: the
                                        whole state kept the predicted mean and joint
                                        covariance, the Laplace average is unchanged */
#define PRISM_FLAG_LOW_INLIERS 8     /* the objective at the final iterate had fewer
                                        contributing pixels than min_inlier_frac of the
                                        image: the step ran, but the pose is weakly
                                        constrained by the frame */

/* Objectives for the pose update. */
#define PRISM_OBJ_P2 0 /* prediction-to-observation surrogate against the previous
                          render (App. E.3), the paper's objective */
#define PRISM_OBJ_P1 1 /* render-through likelihood of the current map (Sec. 4.3.2) */

typedef struct {
    int32_t n;        /* voxels per axis; multiple of 8, 8 <= n <= 1024 */
    int32_t dtype;    /* PRISM_F32 or PRISM_BF16 (storage of means and variances) */
    double voxel;     /* voxel edge length (m), > 0 */
    double origin[3]; /* grid min corner (m) */
    double occ_out;   /* occupancy of corners outside the grid (paper: -0.001) */
    double rgb_out;   /* colour of corners outside the grid (paper: 0) */
    int64_t capacity; /* 0: dense map.  > 0: brick-pool map with room for this many
                         8^3 bricks, 1 <= capacity <= (n/8)^3 (see "Brick-pool maps") */
} prism_grid;

typedef struct {
    int32_t width, height; /* pixels, 1..8192 each */
    double fx, fy, cx, cy; /* pinhole intrinsics (pixels) */
    double d_near, d_far;  /* first and last sample depth (m), 0 <= d_near < d_far */
    int32_t n_samples;     /* K samples per ray, 2..4096 */
    int32_t pad_;
    double tau; /* hit threshold on occupancy (paper: 0) */
} prism_camera;

typedef struct {
    double t[3];
    double q[4]; /* w, x, y, z */
} prism_pose;

typedef struct {
    double w_depth;    /* weight of a depth / point-to-plane row, 1/b_geo^2 */
    double w_rgb;      /* weight of each colour row, 1/b_rgb^2 */
    double gate_depth; /* a depth row is dropped if |r| > gate_depth (m) */
    double gate_rgb;   /* the colour rows are dropped if |r_r|+|r_g|+|r_b| > gate_rgb */
} prism_weights;

typedef struct {
    double trunc;      /* truncation distance (m), > 0 */
    double lam_update; /* update precision 1/sigma_u^2, > 0 */
} prism_map_params;

/* Normal equations of one frame: 29 doubles
 *   [0..20]  upper triangle of H = sum_rows w J^T J, row-major (a <= b)
 *   [21..26] g = sum_rows w J^T r
 *   [27]     cost sum_rows w r^2
 *   [28]     number of pixels that contributed at least one row
 * Rows are the depth (or point-to-plane) row and the three colour rows of a
 * pixel, each kept or dropped by the gates of prism_weights. */
#define PRISM_NEQ 29

/* Last error message of the calling thread ("" if none). */
const char *prism_last_error(void);

/* Library version string. */
const char *prism_version(void);

/* sizeof() of a public struct given its name ("prism_grid", "prism_camera",
 * "prism_pose", "prism_weights", "prism_map_params", "prism_filter_cfg",
 * "prism_filter_state", "prism_filter_bias_state", "prism_frame",
 * "prism_adam_params"); 0 for an unknown
 * name.  Lets
 * bindings verify their struct mirrors. */
size_t prism_sizeof(const char *type_name);

/* ------------------------------------------------------------------------ */
/* Voxel map                                                                */
/* ------------------------------------------------------------------------ */
/* The map is one opaque device buffer of prism_map_bytes() bytes: eight
 * planes (mean occupancy, mean R, G, B, then the four variances) of n^3
 * values of the grid's dtype, each plane in 8x8x8-brick order, followed by a
 * brick summary (one value per 8^3 brick, <= 0 exactly when every occupancy
 * mean of the brick is <= 0, the largest occupancy mean when that is > 0; the
 * renderer uses it to skip free space when tau == 0) and a small scratch area used by
 * prism_map_update.  Every call of this library that writes the map keeps the
 * summary current; after writing the planes directly (e.g. a gradient step on
 * the means), call prism_map_refresh before rendering.  Calls that write the
 * same map must not overlap.  Use prism_map_from_dense / prism_map_to_dense
 * to exchange the planes with the dense layout [4][n][n][n] (channel, z, y,
 * x; x fastest). */

/* Brick-pool maps (grid.capacity > 0; the memory-efficient representation
 * the paper points to in Sec. 6 and App. I): only bricks that have received
 * an update hold storage.  A dense table maps each 8^3 brick of the grid to a
 * slot of a pool of `capacity` bricks (8 planes each, same storage type), or
 * to none; a voxel of a brick without a slot reads as the grid's outside
 * values (occ_out, rgb_out) with the variance given to prism_map_init, which
 * is also how a dense map's untouched voxels read when it was initialised
 * with occ0 = occ_out and rgb0 = rgb_out.  prism_map_update gives a brick a
 * slot (filled with those values) the first time one of its voxels is
 * updated; when the pool is full the brick's update is dropped and counted
 * (prism_map_pool_usage).  With enough capacity every result equals the dense
 * map's bit for bit.  Rendering, the P1 Jacobian, tracking, the filter and
 * the serving calls accept both kinds; the adjoint and descent mapping need a
 * dense FP32 map. */

/* Bytes of a map of this grid (App. D map belief: mean and variance per
 * voxel and channel).  Fails on an unsupported grid. */
prism_status prism_map_bytes(const prism_grid *grid, size_t *bytes);

/* Sets every voxel to (occ0, rgb0, rgb0, rgb0) with variance var0 in all
 * four channels (App. B/G first map belief: occupancy -0.001, colour 0,
 * broad variance).  map: device, prism_map_bytes() bytes, 256-byte aligned.
 * A brick-pool map empties its pool; it requires occ0 == occ_out and
 * rgb0 == rgb_out (as floats) and keeps var0 for bricks given a slot later. */
prism_status prism_map_init(const prism_grid *grid, void *map, float occ0, float rgb0, float var0,
                            hipStream_t stream);

/* Brick-pool maps: usage[0] = bricks holding a slot, usage[1] = brick
 * updates dropped because the pool was full, both since prism_map_init.
 * usage: device int32 [2], written asynchronously. */
prism_status prism_map_pool_usage(const prism_grid *grid, const void *map, int32_t *usage,
                                  hipStream_t stream);

/* Dense FP32 [4][n][n][n] means and variances (device) -> map.  BF16 maps
 * round to nearest-even.  Either of mean4 / var4 may be NULL to leave that
 * half untouched.  Dense maps only. */
prism_status prism_map_from_dense(const prism_grid *grid, void *map, const float *mean4,
                                  const float *var4, hipStream_t stream);

/* Recomputes the brick summary from the mean planes (after direct writes). */
prism_status prism_map_refresh(const prism_grid *grid, void *map, hipStream_t stream);

/* map -> dense FP32 [4][n][n][n] (device); either output may be NULL. */
prism_status prism_map_to_dense(const prism_grid *grid, const void *map, float *mean4, float *var4,
                                hipStream_t stream);

/* FP32 [c][n^3] brick-ordered planes <-> dense [c][n][n][n] (device), for
 * gradients of the map means (see prism_render_vjp). */
prism_status prism_bricks_to_dense(int32_t n, int32_t channels, const float *bricks, float *dense,
                                   hipStream_t stream);
prism_status prism_dense_to_bricks(int32_t n, int32_t channels, const float *dense, float *bricks,
                                   hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Emission (App. B)                                                        */
/* ------------------------------------------------------------------------ */
/* Renders n_frames RGB-D frames from the map means.  Per pixel ray: the
 * occupancy at the K samples by trilinear interpolation; the first sample k*
 * whose occupancy exceeds tau; alpha = (tau - f(k*-1)) / (f(k*) - f(k*-1));
 * depth = alpha d(k*) + (1 - alpha) d(k*-1) and colour the same blend of the
 * two samples' interpolated colours (App. B, depth-interpolation equation;
 * colour "analogously").  A ray without a crossing, or whose first sample is
 * already occupied (k* = 0), is invalid: depth 0, rgb 0, mask 0.
 *
 * poses:   device, n_frames prism_pose.
 * depth:   device [n_frames][H][W] float.      rgb: [n_frames][H][W][3] float.
 * mask:    device [n_frames][H][W] uint8 (1 = valid).
 * hit_k:   nullable, device [n_frames][H][W] int32: k*, or -1 without crossing.
 * normals: nullable, device [n_frames][H][W][3] float, camera frame, with
 * nmask:   (required iff normals) [n_frames][H][W] uint8: normal of the
 *          rendered depth image by central differences of the back-projected
 *          points, oriented towards the camera; 0 on the border, next to an
 *          invalid pixel or where a neighbour's depth differs by more than
 *          normal_disc metres (App. E.3 anchor normals; App. G discontinuous
 *          depth ignored). */
prism_status prism_render(const prism_grid *grid, const void *map, const prism_camera *cam,
                          const prism_pose *poses, int32_t n_frames, float *depth, float *rgb,
                          uint8_t *mask, int32_t *hit_k, float *normals, uint8_t *nmask,
                          double normal_disc, hipStream_t stream);

/* The paper's ray sampling (App. B: ray points at depth offsets eps, 2 eps,
 * 3 eps, ...; App. G: eps = 0.4 voxel, rays up to the maximum camera
 * depth) as a camera's sampling: sets cam->d_near = eps, cam->n_samples =
 * floor(max_depth / eps) and cam->d_far = n_samples eps, so that sample k
 * lies at depth (k + 1) eps (to rounding).  Other fields are left as they
 * are.  Host only, no GPU work.  PRISM_INVALID_ARGUMENT for a NULL camera or
 * a voxel or max_depth that is not finite and > 0; PRISM_UNSUPPORTED when
 * the count falls outside 2..4096 (cam then unchanged). */
prism_status prism_camera_paper_sampling(prism_camera *cam, double voxel, double max_depth);

/* Workspace bytes needed by prism_render_jacobian / prism_track_p2 /
 * prism_render_vjp for n_frames frames of this camera. */
prism_status prism_reduce_workspace_bytes(const prism_camera *cam, int32_t n_frames, size_t *bytes);

/* Render-through (P1) pose Jacobian and normal equations (Sec. 4.3.2 MAP
 * objective with the emission likelihood): for every valid ray, the 4x6
 * derivative of (depth, r, g, b) w.r.t. delta with k* held fixed; residuals
 * r = rendered - observed; rows gated and weighted by `w`; per frame the
 * 29-double normal equations (see PRISM_NEQ).  A pixel contributes only if
 * its ray is valid and its observed depth is finite and > 0.
 *
 * obs_depth: device [n][H][W] float;  obs_rgb: device [n][H][W][3] float.
 * depth/rgb/mask: nullable outputs as in prism_render.
 * J:      nullable, device [n][H][W][4][6] float (0 for pixels that do not
 *         contribute).  resid: nullable [n][H][W][4] float.
 * rowmask: nullable [n][H][W] uint8, bit0 depth row kept, bit1 colour rows kept.
 * neq:    device [n][29] double.
 * workspace: device, >= prism_reduce_workspace_bytes(cam, n) bytes. */
prism_status prism_render_jacobian(const prism_grid *grid, const void *map,
                                   const prism_camera *cam, const prism_pose *poses,
                                   int32_t n_frames, const float *obs_depth, const float *obs_rgb,
                                   const prism_weights *w, float *depth, float *rgb, uint8_t *mask,
                                   float *J, float *resid, uint8_t *rowmask, double *neq,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream);

/* prism_render_jacobian for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and results, bit for
 * bit, minus workspace/workspace_bytes: the per-workgroup partial sums go to
 * a fixed array inside the library, one copy per GPU, of
 * prism_render_jacobian_noalloc_max_bytes() bytes (8 MiB), held until the
 * process ends.  A call needs n_frames * ceil(W/8) * ceil(H/8) * 232 bytes of
 * it (320x240: 30 frames at most; 640x480: 7) and fails with
 * PRISM_INVALID_ARGUMENT, queuing nothing, beyond that.  Allocates nothing:
 * no hipMalloc, hipFree or allocating library call.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (on different
 * streams, or from different threads) race and give undefined results; calls
 * in order on one stream are safe. */
size_t prism_render_jacobian_noalloc_max_bytes(void);
prism_status prism_render_jacobian_noalloc(const prism_grid *grid, const void *map,
                                           const prism_camera *cam, const prism_pose *poses,
                                           int32_t n_frames, const float *obs_depth,
                                           const float *obs_rgb, const prism_weights *w, float *depth,
                                           float *rgb, uint8_t *mask, float *J, float *resid,
                                           uint8_t *rowmask, double *neq, hipStream_t stream);

/* The pose perturbation all Jacobians are taken in (a left retraction in the
 * world frame): out[i] = (t_i + dt_i, Exp(dtheta_i) R_i) for delta[i] =
 * (dt_i, dtheta_i).  poses, out: device, n prism_pose (may alias); delta:
 * device double [n][6].  The differentiable renderer (RenderFn) renders at
 * these poses. */
prism_status prism_pose_retract(const prism_pose *poses, const double *delta, int32_t n, prism_pose *out,
                                hipStream_t stream);

/* Prediction-to-observation objective (App. E.3, P2) for one frame: each
 * observed pixel with valid depth D is back-projected (D r_c), moved by the
 * pose iterate `pose` and brought into the camera of `pose_prev` (the pose the
 * anchor frame was rendered at).  Geometric row: point-to-plane residual
 * n.(p - Y) with the nearest anchor pixel's back-projected point p and normal
 * n (requires a valid anchor pixel and normal).  Colour rows: anchor colour
 * bilinearly interpolated at the projection minus the observed colour
 * (requires the 4 taps valid).  Derivatives w.r.t. delta of `pose`; gating,
 * weights and outputs as in prism_render_jacobian (n_frames = 1).
 * anchor_*: device buffers as produced by prism_render (+ normals). */
prism_status prism_track_p2(const prism_camera *cam, const prism_pose *pose,
                            const prism_pose *pose_prev, const float *obs_depth,
                            const float *obs_rgb, const float *anchor_depth,
                            const float *anchor_rgb, const uint8_t *anchor_mask,
                            const float *anchor_normals, const uint8_t *anchor_nmask,
                            const prism_weights *w, float *J, float *resid, uint8_t *rowmask,
                            double *neq, void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/* Adjoint of prism_render w.r.t. the map means and the pose (k* of each ray
 * held fixed, as given in hit_k from the forward render of the same map and
 * poses).  Given upstream gradients of depth and rgb:
 *   grad_mean += dL/dmean, FP32 [4][n^3] in brick order (the first four planes
 *                of an FP32 map; prism_bricks_to_dense converts);
 *   grad_pose  = dL/ddelta per frame, device [n_frames][6] double.
 * The map must be FP32.  Scatter into grad_mean uses atomic adds (order of
 * additions, hence the last bits, may vary between runs). */
prism_status prism_render_vjp(const prism_grid *grid, const void *map, const prism_camera *cam,
                              const prism_pose *poses, int32_t n_frames, const int32_t *hit_k,
                              const float *g_depth, const float *g_rgb, float *grad_mean,
                              double *grad_pose, void *workspace, size_t workspace_bytes,
                              hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Map update (App. D)                                                      */
/* ------------------------------------------------------------------------ */
/* Closed-form update of the map belief with one RGB-D frame at `pose`: every
 * voxel whose centre has camera depth z > 0, projects into the image at pixel
 * (floor(u), floor(v)) with observed depth D finite and > 0, and z <= D +
 * trunc, is multiplied per channel by the update Gaussian
 * N(f, 1/lam_update), f = (max(z - D, -trunc), observed rgb), in the
 * precision form of App. D, in double precision in this order and rounded
 * once to the map's storage type:
 *   lambda = 1/var,  var' = 1/(lambda + lam_update),
 *   mean' = var' (lambda mean + lam_update f).
 * Other voxels are left bitwise unchanged.
 * pose: device.  obs_depth [H][W], obs_rgb [H][W][3]: device float.
 * n_updated: nullable, device int64: receives the number of updated voxels. */
prism_status prism_map_update(const prism_grid *grid, void *map, const prism_camera *cam,
                              const prism_pose *pose, const float *obs_depth,
                              const float *obs_rgb, const prism_map_params *p,
                              int64_t *n_updated, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Map inference by gradient descent (Sec. 4.3.1 alternative, Sec. 5.3)     */
/* ------------------------------------------------------------------------ */
/* The map-filter target of Sec. 4.3.1 (emission likelihood of one frame at
 * the nominal pose times the previous map belief) minimised directly by
 * gradient descent through the renderer, the alternative the paper compares
 * the closed-form update against.  Objective, up to constants:
 *   E(mean) = sum over kept rows w r^2 + 1/2 sum (mean - mean0)^2 / var
 * with the rows, weights and gates of prism_render_jacobian (r = rendered -
 * observed) and (mean0, var) the map on entry.  Each of n_iters steps renders
 * at the current means, forms dE/dmean through the adjoint of the emission
 * (first crossing held) and takes mean <- mean - lr dE/dmean, lr = lr_occ for
 * occupancy and lr_rgb for colour.  Only bricks some ray touched move; the
 * variances stay as they were (descent estimates none); the brick summary is
 * kept current.  FP32 maps only.
 *
 * map:       device, updated in place (the previous belief on entry).
 * pose:      device.  obs_depth [H][W], obs_rgb [H][W][3]: device float.
 * cost:      nullable, device double [n_iters]: E at the means before each step.
 * workspace: device, 256-byte aligned, >= prism_map_gd_workspace_bytes().
 *            Its gradient accumulators must be zero on entry: zero-fill the
 *            workspace once; every call that returns PRISM_OK leaves them
 *            zero again.  Calls sharing a workspace must not overlap. */
prism_status prism_map_gd_workspace_bytes(const prism_grid *grid, const prism_camera *cam,
                                          size_t *bytes);
prism_status prism_map_gd(const prism_grid *grid, void *map, const prism_camera *cam,
                          const prism_pose *pose, const float *obs_depth, const float *obs_rgb,
                          const prism_weights *w, double lr_occ, double lr_rgb, int32_t n_iters,
                          double *cost, void *workspace, size_t workspace_bytes,
                          hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Filter (Sec. 4.3; App. C, E)                                             */
/* ------------------------------------------------------------------------ */
/* The paper's literal forms a filter can select (prism_filter_cfg.modes,
 * any combination; 0 keeps the readings the library takes by default, where
 * the printed form is ambiguous or inconsistent):
 *   PRISM_MODE_TRANSITION_DT2  the control enters the velocities as u dt^2,
 *       as App. E.1 prints it (default u dt, an acceleration integrated over
 *       the frame interval).  Predict steps and prism_rollout alike.
 *   PRISM_MODE_LAPLACE_FACTOR1 Laplace covariance (H_o + Lp)^-1, the
 *       posterior covariance under a Gaussian likelihood of precision w,
 *       instead of Sec. 5.1's (2 H_o + Lp)^-1 (H_o = sum w J^T J over the
 *       kept rows at the final iterate, Lp the prior pose precision).
 *   PRISM_MODE_IRLS_L1 the Gauss-Newton iterations minimise the L1 data
 *       terms of App. E.3, sum |r| / b with b = 1/sqrt(w) per row, plus the
 *       prior, by iteratively reweighted least squares: in each iteration a
 *       kept row weighs 1 / (2 b max(|r|, irls_floor b)) at the iterate's
 *       residual r instead of w.  The gates are unchanged, and the Laplace
 *       covariance still squares the rows' Jacobian with weights w (App. E.3
 *       takes the curvature of the squared form).  prism_pose_update_adam
 *       returns PRISM_UNSUPPORTED for filters with this mode.
 *   PRISM_MODE_ACCEL_BIAS a 15-D state: pose, velocities and an accelerometer
 *       bias b (body frame; the paper's state is 12-D, App. E, and this
 *       extension serves inputs from a biased IMU).  The linear part of each
 *       frame's control is then the accelerometer's body-frame specific force
 *       f (its mean over the frame interval), the acceleration R (f - b) + g
 *       with the state's own rotation R and cfg->gravity; b follows a random
 *       walk of cfg->sigma_bias per step.  Prediction, split and combination
 *       run over the 15x15 covariance (tangent dt, dtheta, dv, dw, db) with a
 *       9-D velocity-and-bias conditional; the pose objective is unchanged.
 *       The bias, the full covariance and the conditional are in the filter's
 *       prism_filter_bias_state (prism_filter_bias_state_ptr); the state's
 *       P holds the leading 12x12 block.  Set the belief with
 *       prism_filter_reset_bias.  prism_rollout draws and predicts the 15-D
 *       state (its noise rows and moments are 15-D). */
#define PRISM_MODE_TRANSITION_DT2 1
#define PRISM_MODE_LAPLACE_FACTOR1 2
#define PRISM_MODE_IRLS_L1 4
#define PRISM_MODE_ACCEL_BIAS 8

typedef struct {
    prism_grid grid;
    prism_camera cam;
    double dt;                          /* frame interval (s) */
    double sigma_vel_t, sigma_vel_r;    /* transition scales per step (App. G table) */
    double sigma_pose_t, sigma_pose_r;
    prism_weights w;                    /* residual weights and gates (App. G) */
    double ema;                         /* EMA coefficient of Laplace covariances (0.8) */
    int32_t n_gn;                       /* Gauss-Newton iterations per step, 0..64 */
    int32_t objective;                  /* PRISM_OBJ_P2 or PRISM_OBJ_P1 */
    prism_map_params map;               /* update truncation and precision */
    double normal_disc;                 /* anchor-normal discontinuity threshold (m) */
    double min_inlier_frac;             /* PRISM_FLAG_LOW_INLIERS below this fraction of the
                                           image's pixels contributing, [0, 1] (0: never) */
    int32_t modes;                      /* PRISM_MODE_* bits (0: the default readings) */
    int32_t pad_;
    double irls_floor;                  /* PRISM_MODE_IRLS_L1: residual floor as a fraction of each
                                           row's scale b, finite and > 0; unused otherwise */
    double sigma_bias;                  /* PRISM_MODE_ACCEL_BIAS: bias random walk per step (m/s^2),
                                           >= 0; unused otherwise */
    double gravity[3];                  /* PRISM_MODE_ACCEL_BIAS: gravity in the world frame (m/s^2) */
} prism_filter_cfg;

/* Device-resident filter state (first bytes of the state buffer), FP64.
 * Covariances are row-major over the tangent (dt, dtheta, dv, dw). */
typedef struct {
    prism_pose pose;        /* posterior mean pose */
    double v[3], w[3];      /* posterior mean velocity (world, linear / angular) */
    double P[144];          /* 12x12 state covariance */
    double Sbar[36];        /* EMA of the Laplace pose covariances */
    prism_pose anchor;      /* pose the anchor frame was rendered at */
    prism_pose prior;       /* predicted pose mean of the current step */
    prism_pose iter;        /* Gauss-Newton iterate */
    double vel_prior[6];    /* predicted velocity mean */
    double Lp[36];          /* prior pose precision */
    double D[36];           /* velocity-conditional gain: E[dv | dpose] = D dpose */
    double Sv[36];          /* velocity-conditional covariance */
    double S_lap[36];       /* last Laplace covariance */
    double neq[29];         /* normal equations at the final iterate */
    double u[6];            /* control of the last step */
    int64_t step;           /* frames consumed */
    int64_t n_updated;      /* voxels updated by the last map update */
    int32_t flags;          /* PRISM_FLAG_* of the last step */
    int32_t has_sbar;
    int64_t n_updated_total; /* voxels updated by all map updates of the filter's steps */
} prism_filter_state;

/* The accelerometer-bias part of a PRISM_MODE_ACCEL_BIAS filter's state
 * (device, FP64; in the state buffer after prism_filter_state).
 * Covariances are row-major over the tangent (dt, dtheta, dv, dw, db). */
typedef struct {
    double b[3];          /* posterior mean bias */
    double P[225];        /* 15x15 state covariance */
    double D[54];         /* 9x6 gain of (dv, dw, db) on the pose offset */
    double Sv[81];        /* 9x9 covariance of (dv, dw, db) given the pose */
    double rest_prior[9]; /* predicted (v, w, b) */
} prism_filter_bias_state;

typedef struct prism_filter prism_filter;

/* One frame for a filter step.  All pointers device. */
typedef struct {
    const float *depth; /* [H][W] observed z-depth (<= 0 or non-finite: invalid) */
    const float *rgb;   /* [H][W][3] observed colour */
    const double *u;    /* [6] control between the previous and this frame:
                           linear then angular acceleration, world frame;
                           ignored for a filter's first frame */
} prism_frame;

/* Bytes of the state buffer of a filter (state struct, anchor frame, reduction
 * workspace), excluding the map. */
prism_status prism_filter_bytes(const prism_filter_cfg *cfg, size_t *bytes);

/* Creates a handle that borrows state_mem (prism_filter_bytes, 256-byte
 * aligned) and map_mem (prism_map_bytes of cfg->grid).  The handle owns only
 * host memory; prism_filter_destroy never frees the borrowed buffers. */
prism_status prism_filter_create(const prism_filter_cfg *cfg, void *state_mem, void *map_mem,
                                 prism_filter **out);
prism_status prism_filter_destroy(prism_filter *f);

/* Sets the state belief: x0 = (t[3], q[4], v[3], w[3]) and P0 [12x12], both
 * host; resets the step counter (the next frame is the first, Sec. 4.1: x_1
 * given).  Does not touch the map. */
prism_status prism_filter_reset(prism_filter *f, const double *x0, const double *P0,
                                hipStream_t stream);

/* prism_filter_reset for PRISM_MODE_ACCEL_BIAS filters: x0 = (t[3], q[4],
 * v[3], w[3], b[3]) and P0 [15x15] (tangent dt, dtheta, dv, dw, db), both
 * host.  PRISM_UNSUPPORTED for filters without the mode (and
 * prism_filter_reset is refused for filters with it). */
prism_status prism_filter_reset_bias(prism_filter *f, const double *x0, const double *P0,
                                     hipStream_t stream);

/* Device address of a PRISM_MODE_ACCEL_BIAS filter's bias state (read it
 * after the stream's work completes); PRISM_UNSUPPORTED without the mode. */
prism_status prism_filter_bias_state_ptr(const prism_filter *f, prism_filter_bias_state **out);

/* State filter only (Sec. 4.3.2): predict and split the state belief with
 * the frame's control, n_gn Gauss-Newton steps of the configured objective
 * from the predicted pose, Laplace covariance at the final iterate (EMA'd),
 * and combination with the velocity conditional (cfg->modes selects the
 * paper's literal transition, Laplace factor and L1 objective).  Not valid
 * for the first frame. */
prism_status prism_pose_update(prism_filter *f, const prism_frame *frame, hipStream_t stream);

/* The paper's own pose optimiser (App. G): Adam with its momentum disabled,
 * separate step sizes for translation and rotation, a fixed number of steps,
 * each on pixels sampled uniformly from the frame. */
typedef struct {
    int32_t n_steps;  /* optimisation steps (paper: 1000), 1..1000000 */
    int32_t n_pixels; /* pixels per step (paper: 200), 1..65536 */
    double lr_t;      /* step size of the translation components (paper: 0.001) */
    double lr_r;      /* step size of the rotation components (paper: 0.00036) */
    double beta2;     /* second-moment decay, [0, 1) (Adam's default 0.999) */
    double eps;       /* denominator floor, > 0 (Adam's default 1e-8) */
} prism_adam_params;

/* prism_pose_update with the Gauss-Newton iterations replaced by the
 * paper's optimiser on the P2 objective (Sec. 4.3.2 MAP objective, App. E.3
 * surrogate, App. G optimiser).  From the predicted pose, step k evaluates
 * the rows of the pixels pixels[k][0..n_pixels) (row-major indices v*W+u into
 * the frame, drawn by the caller; an index outside the image is a pixel
 * without rows, repeats count repeatedly) and forms the gradient of the MAP
 * objective with the data term scaled by W*H/n_pixels (an unbiased estimate
 * of the full-frame sum): g = scale * sum 2 w r J + Lp e.  The step keeps a
 * second moment v <- beta2 v + (1-beta2) g^2 per component, bias-corrects it,
 * and moves the pose by -lr g / (sqrt(vhat) + eps) (left retraction, as the
 * Gauss-Newton step).  The Laplace covariance then comes from the dense
 * normal equations at the final pose, as in prism_pose_update.  The whole
 * optimisation is one kernel launch (one workgroup).  Filters configured for
 * the P1 objective or PRISM_MODE_IRLS_L1 return PRISM_UNSUPPORTED.
 * pixels: device int32 [n_steps][n_pixels]. */
prism_status prism_pose_update_adam(prism_filter *f, const prism_frame *frame,
                                    const prism_adam_params *p, const int32_t *pixels,
                                    hipStream_t stream);

/* One filter step (as prism_filter_step for one handle) whose state filter
 * is prism_pose_update_adam; a filter's first frame only updates the map and
 * renders the anchor (p and pixels are still checked). */
prism_status prism_filter_step_adam(prism_filter *f, const prism_frame *frame,
                                    const prism_adam_params *p, const int32_t *pixels,
                                    hipStream_t stream);

/* Predictive rollout (App. J, prediction and control): from the handle's
 * current state belief N(x, P) and map means, predict k steps ahead under
 * the candidate controls u[0..k) with the generative transition (App. B):
 * n_samples sampled trajectories, their poses and (optionally) the frames
 * rendered from the map means at every sampled pose, plus the closed-form
 * linearised moments of the predicted state (the uncertainty envelope).
 * u:     device double [k][6] (linear then angular acceleration, world).
 * noise: device double [n_samples][k+1][12] standard normal draws (the
 *        caller's): row 0 draws the start state x (+) L z (P = L L^T, tangent
 *        order t, theta, v, w, left retraction for the pose), row j+1 the
 *        process noise of step j, n = sqrt(diag Q) z, entering as
 *        v' = v + u_v dt + n_v, w' = w + u_w dt + n_w, t' = t + v' dt + n_t,
 *        (u dt^2 in place of u dt under PRISM_MODE_TRANSITION_DT2),
 *        R' = Exp(n_theta) Exp(w' dt) R.
 *        PRISM_MODE_ACCEL_BIAS filters: rows of 15 draws (the bias last;
 *        start state b + L z, process noise n_b walking the bias), u_v is
 *        the body-frame specific force and the acceleration R (u_v - b) + g
 *        uses the draw's own rotation and bias.
 * poses: device [n_samples][k] (required when n_samples > 0).
 * mean:  nullable device [k][13] (t, q, v, w); cov: nullable [k][144]: the
 *        linearised prediction (App. E.2) after each control.  With
 *        PRISM_MODE_ACCEL_BIAS: mean [k][16] (t, q, v, w, b), cov [k][225].
 * depth/rgb/mask: nullable together, [n_samples*k][H][W] (rgb [..][3]), as
 *        prism_render at poses (sample-major); needs n_samples*k <= 65535.
 * flags: nullable device int32: PRISM_FLAG_CHOL_FALLBACK when P is not
 *        positive definite (the samples then start at the mean), else 0. */
prism_status prism_rollout(prism_filter *f, const double *u, int32_t k, int32_t n_samples,
                           const double *noise, prism_pose *poses, double *mean, double *cov,
                           float *depth, float *rgb, uint8_t *mask, int32_t *flags,
                           hipStream_t stream);

/* One full filter step for each of n handles (Sec. 4.3): the state filter
 * as in prism_pose_update (skipped for a filter's first frame), then the map
 * update at the posterior mean pose (App. C nominal state), then the anchor
 * frame rendered from the updated map at that pose for the next step.
 * frames: host array of n descriptors. */
prism_status prism_filter_step(prism_filter *const *fs, int32_t n, const prism_frame *frames,
                               hipStream_t stream);

/* Same result as prism_filter_step, bit for bit, for serving loops that
 * replay steps: after a filter's first frame each step is launched as one
 * HIP graph that the handle records the first time it sees a frame with
 * these buffer addresses (depth, rgb, u) and replays afterwards, so callers
 * keep a few fixed input slots per stream and copy each frame into one.  A
 * handle keeps up to 4 graphs; recording a fifth evicts the least recently
 * used one once its last launch has finished.  stream must be a non-default
 * stream that is not being captured; a graph launched on a stream other than
 * its previous launch's first waits (on the host) for that launch.  The
 * graphs hold the addresses of the handle's state and map buffers, which
 * must stay where they are; prism_filter_destroy waits for each graph's last
 * launch, then frees them. */
prism_status prism_filter_step_graph(prism_filter *const *fs, int32_t n, const prism_frame *frames,
                                     hipStream_t stream);

/* ---- serving: per-handle input slots, submission and completion ---------- */

/* Registers n_slots (1..4) input slots: caller-owned device buffers, each a
 * depth [H][W] f32, rgb [H][W][3] f32 and control [6] f64 (16-byte aligned),
 * that prism_filter_submit copies frames into.  Resets the submission and
 * completion counters; must not be called while submitted steps run. */
prism_status prism_filter_set_slots(prism_filter *f, int32_t n_slots, const prism_frame *slots);

#define PRISM_SUBMIT_FROM_HOST 1 /* src buffers are host memory (pinned for an asynchronous copy) */
#define PRISM_SUBMIT_EAGER 2     /* launch the step's kernels one by one instead of a graph */
#define PRISM_SUBMIT_GRAPH 4     /* prism_filter_step_batch: replay the batch's stages from a HIP
                                    graph recorded for its members, their slots and which of them
                                    are on their first frame */

/* Queues one filter step for the frame src (u may be NULL only for the
 * handle's first frame) without waiting: the frame is copied into the next
 * slot (round robin; one staging kernel for device sources, asynchronous
 * copies for host sources), then the step runs as in prism_filter_step_graph
 * on that slot, and an event marks its end.  *seq (nullable) receives the
 * step's 0-based submission number.  Returns PRISM_BUSY, and queues nothing,
 * when the slot's previous step has not finished.  All submissions of a
 * handle must use one non-default stream; the copy out of src is
 * asynchronous, so src must stay unchanged until the step has completed. */
prism_status prism_filter_submit(prism_filter *f, const prism_frame *src, int32_t flags, hipStream_t stream,
                                 int64_t *seq);

/* Continuous batching: one filter step for each of n distinct handles (frame
 * src[i] for fs[i]) in a single batch, with the same effect on each handle,
 * bit for bit, as prism_filter_submit.  Each stage of the step (frame
 * staging, predict, tracking, Gauss-Newton, Laplace/combine, cull, map
 * update, anchor render, normals) is one kernel launch for the whole batch,
 * workgroups assigned to handles by ragged block ranges, so handles of
 * different image and map sizes, storage types and objectives (P2 and P1)
 * share launches.  Handles must have input slots registered; each takes its
 * next slot.  Returns PRISM_BUSY, and queues nothing, when any handle has
 * every slot in flight.  flags: PRISM_SUBMIT_FROM_HOST as for
 * prism_filter_submit; PRISM_SUBMIT_GRAPH launches every stage after the
 * frame staging from one HIP graph, recorded the first time the batch's
 * members (in this order), their slots and their first-frame states occur
 * and replayed afterwards (up to 64 graphs per process, least recently used
 * evicted once its last launch has finished; a handle's graphs are released
 * by prism_filter_destroy).  Same results, bit for bit.  stream must not be
 * being captured (PRISM_CAPTURE_ERROR). */
prism_status prism_filter_step_batch(prism_filter *const *fs, int32_t n, const prism_frame *src, int32_t flags,
                                     hipStream_t stream);

/* Stage timer (profiling aid): prism_stage_timer_arm(cap) makes every later
 * prism_filter_step_batch record an event pair around each stage's launch,
 * up to cap launches per stage (cap 0 disarms); prism_stage_timer_read
 * waits for them, disarms, and returns per stage (index PRISM_STAGE_*) the
 * summed launch time in ms and the number of launches timed.  Process-wide;
 * events are created on arm and kept for reuse. */
#define PRISM_STAGE_STAGING 0
#define PRISM_STAGE_PREDICT 1
#define PRISM_STAGE_TRACK 2
#define PRISM_STAGE_GN 3
#define PRISM_STAGE_LAPLACE 4
#define PRISM_STAGE_CULL 5
#define PRISM_STAGE_MAP_UPDATE 6
#define PRISM_STAGE_RENDER 7
#define PRISM_STAGE_NORMALS 8
#define PRISM_STAGE_FIRST_FRAME 9
#define PRISM_N_STAGES 10
prism_status prism_stage_timer_arm(int32_t cap);
prism_status prism_stage_timer_read(double *ms /* [PRISM_N_STAGES] */, int64_t *launches /* [PRISM_N_STAGES] */);

/* Non-blocking: *completed = number of submitted steps that have finished
 * (steps finish in submission order). */
prism_status prism_filter_poll(prism_filter *f, int64_t *completed);

/* prism_filter_poll for n handles: completed[i] for fs[i] (host array). */
prism_status prism_filter_poll_batch(prism_filter *const *fs, int32_t n, int64_t *completed);

/* ---- checkpoints: the belief (q_t(M), q_t(x)) in and out (Sec. 4.2-4.3) ---- */

/* Bytes of a checkpoint of a filter of this configuration: a 512-byte header,
 * the state buffer's belief part (state struct and bias state, anchor frame,
 * relative pose) and the whole map buffer. */
prism_status prism_filter_save_bytes(const prism_filter_cfg *cfg, size_t *bytes);

/* Copies the filter's current belief (map and state, after every step queued
 * before on `stream`) into dst, device or host memory (pinned host memory for
 * an asynchronous copy) of at least prism_filter_save_bytes() bytes, 16-byte
 * aligned.  Asynchronous on `stream`; dst is complete once the stream is.  The
 * header (grid, camera, step counter) is copied from a buffer the handle
 * owns, which the next save of the same handle reuses only after this copy
 * has finished. */
prism_status prism_filter_save(prism_filter *f, void *dst, size_t dst_bytes, hipStream_t stream);

/* Restores a checkpoint into f (the same handle or another one made with the
 * same grid, camera and state size (12-D, or 15-D under PRISM_MODE_ACCEL_BIAS);
 * the other configuration values may differ): map and
 * state are overwritten, the next step continues from the saved belief,
 * bit for bit as the saved filter would have.  Reads the header first, so
 * the call waits for `stream` (PRISM_CAPTURE_ERROR while it is being
 * captured) and fails with PRISM_INVALID_ARGUMENT, changing nothing, on a
 * bad magic, version, size, grid, camera or state size.  No step of f may be
 * in flight. */
prism_status prism_filter_load(prism_filter *f, const void *src, size_t src_bytes, hipStream_t stream);

/* Device pointer to the filter's prism_filter_state (inside state_mem). */
prism_status prism_filter_state_ptr(const prism_filter *f, prism_filter_state **state);

/* Device pointers to the anchor frame buffers (inside state_mem). */
prism_status prism_filter_anchor(const prism_filter *f, float **depth, float **rgb, uint8_t **mask,
                                 float **normals, uint8_t **nmask);

#ifdef __cplusplus
}
#endif

#endif /* PRISM_H */
