// Prediction-to-observation tracking objective (App. E.3): point-to-plane
// against the nearest anchor pixel and photometric error against the
// bilinearly interpolated anchor colour, with the fused reduction of the
// gated, weighted normal equations.  One observed pixel per lane, pixels in
// row-major order so observation reads are coalesced; anchor reads are
// gathers around the reprojected location.  (Two or four pixels per lane,
// paying the 29-sum reduction once for them, measured slower: the running
// sums stay live across a pixel's work, which takes 100-170 VGPRs and halves
// the waves per SIMD.)
#include "common.hpp"
#include "launch.hpp"
#include "se3.hpp"

namespace prism {

// The rows of observed pixel p (row-major index): geometric row 0
// (point-to-plane against the nearest anchor pixel) and colour rows 1-3
// (bilinear anchor colour minus the observation), residuals in double
// precision, Jacobians w.r.t. the pose perturbation in single precision.
// rm: bit 0 the geometric row passed its gate, bit 1 the colour rows.
// D and orgb: the pixel's observed depth and colour (loaded by the caller).
__device__ __forceinline__ void p2_pixel(const CamC& c, const CamD& cd, const Rel32& rel, int p, float D,
                                         const float orgb[3], const float* __restrict__ a_depth,
                                         const float* __restrict__ a_rgb, const uint8_t* __restrict__ a_mask,
                                         const float* __restrict__ a_normals, const uint8_t* __restrict__ a_nmask,
                                         const WeightsC& wt, float J[4][6], double r[4], int& rm) {
    const int u = p % c.W, v = p / c.W;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        r[a] = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) J[a][m] = 0.0f;
    }
    rm = 0;
    if (!depth_ok(D)) return;
    float rx = ((float)u + 0.5f - c.cx) * c.ifx;
    float ry = ((float)v + 0.5f - c.cy) * c.ify;
    float X[3] = {D * rx, D * ry, D};
    float Y[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Y[a] = ((rel.R[a][0] * X[0] + rel.R[a][1] * X[1]) + rel.R[a][2] * X[2]) + rel.t[a];
    bool geo = false, pho = false;
    int giu = 0, giv = 0, bix = 0, biy = 0;
    float uu = 0.0f, vv = 0.0f;
    if (Y[2] > 0.0f) {
        uu = c.fx * (Y[0] / Y[2]) + c.cx;
        vv = c.fy * (Y[1] / Y[2]) + c.cy;
        if (uu >= 0.0f && uu < (float)c.W && vv >= 0.0f && vv < (float)c.H) {
            giu = (int)uu;
            giv = (int)vv;
            geo = true;
        }
        float bx = uu - 0.5f, by = vv - 0.5f;
        if (bx >= 0.0f && bx < (float)(c.W - 1) && by >= 0.0f && by < (float)(c.H - 1)) {
            bix = (int)bx;
            biy = (int)by;
            pho = true;
        }
    }
    if (geo) {
        int q = giv * c.W + giu;
        geo = a_mask[q] && a_nmask[q];
    }
    int q00 = biy * c.W + bix;
    if (pho) pho = a_mask[q00] && a_mask[q00 + 1] && a_mask[q00 + c.W] && a_mask[q00 + c.W + 1];
    if (!(geo || pho)) return;
    {
    // the value path may fuse multiplies and adds: the pixel decisions above
    // stay in the fixed single-precision recipe; the residual gates below
    // compare double-precision values, which differ from the oracle's by
    // rounding either way
#pragma clang fp contract(fast)
    // values in double precision: back-projected point, moved into the
    // anchor camera; Jacobians in single precision
    const Pose64& Pc = rel.cur;
    const Pose64& Pp = rel.prev;
    double rc[3], Xd[3], RXd[3], dW[3], Yd[3];
    pixel_dir64(cd, u, v, rc);
#pragma unroll
    for (int a = 0; a < 3; ++a) Xd[a] = (double)D * rc[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) RXd[a] = Pc.R[a][0] * Xd[0] + Pc.R[a][1] * Xd[1] + Pc.R[a][2] * Xd[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) dW[a] = RXd[a] + Pc.t[a] - Pp.t[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) Yd[a] = Pp.R[0][a] * dW[0] + Pp.R[1][a] * dW[1] + Pp.R[2][a] * dW[2];
    // dY/ddelta = Rp^T [I | -[R X]x]
    float RX[3] = {(float)RXd[0], (float)RXd[1], (float)RXd[2]};
    float dY[3][6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float e0 = (float)Pp.R[0][a], e1 = (float)Pp.R[1][a], e2 = (float)Pp.R[2][a];
        dY[a][0] = e0;
        dY[a][1] = e1;
        dY[a][2] = e2;
        dY[a][3] = fmaf(RX[1], e2, -RX[2] * e1);
        dY[a][4] = fmaf(RX[2], e0, -RX[0] * e2);
        dY[a][5] = fmaf(RX[0], e1, -RX[1] * e0);
    }
    if (geo) {
        int q = giv * c.W + giu;
        double ra[3];
        pixel_dir64(cd, giu, giv, ra);
        double da = (double)a_depth[q];
        double n0 = a_normals[3 * q], n1 = a_normals[3 * q + 1], n2 = a_normals[3 * q + 2];
        double rg = n0 * (da * ra[0] - Yd[0]) + n1 * (da * ra[1] - Yd[1]) + n2 * (da * ra[2] - Yd[2]);
        r[0] = rg;
        float fn0 = (float)n0, fn1 = (float)n1, fn2 = (float)n2;
#pragma unroll
        for (int m = 0; m < 6; ++m) J[0][m] = -fmaf(fn2, dY[2][m], fmaf(fn1, dY[1][m], fn0 * dY[0][m]));
        if (fabs(rg) <= wt.gate_depth) rm |= 1;
    }
    if (pho) {
        const double izd = 1.0 / Yd[2];
        double ud = cd.fx * Yd[0] * izd + cd.cx;
        double vd = cd.fy * Yd[1] * izd + cd.cy;
        double ax = (ud - 0.5) - (double)bix, ay = (vd - 0.5) - (double)biy;
        float Y2 = (float)Yd[2];
        float iz = 1.0f / Y2;
        float du_[3] = {c.fx * iz, 0.0f, -c.fx * (float)Yd[0] * iz * iz};
        float dv_[3] = {0.0f, c.fy * iz, -c.fy * (float)Yd[1] * iz * iz};
        float dum[6], dvm[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            dum[m] = fmaf(du_[2], dY[2][m], du_[0] * dY[0][m]);
            dvm[m] = fmaf(dv_[2], dY[2][m], dv_[1] * dY[1][m]);
        }
        double l1 = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            double I00 = a_rgb[3 * q00 + ch], I10 = a_rgb[3 * (q00 + 1) + ch];
            double I01 = a_rgb[3 * (q00 + c.W) + ch], I11 = a_rgb[3 * (q00 + c.W + 1) + ch];
            // bilinear value and its image gradient as linear blends (fused
            // multiply-adds; the same interpolant as the hat-weight sum, to
            // rounding): rows blended along x, then the rows along y
            const double d0 = I10 - I00, d1 = I11 - I01;
            const double t0 = __builtin_fma(ax, d0, I00), t1 = __builtin_fma(ax, d1, I01);
            double Ii = __builtin_fma(ay, t1 - t0, t0);
            float gu = (float)__builtin_fma(ay, d1 - d0, d0);
            float gv = (float)(t1 - t0);
            double rp = Ii - (double)orgb[ch];
            r[1 + ch] = rp;
            l1 += fabs(rp);
#pragma unroll
            for (int m = 0; m < 6; ++m) J[1 + ch][m] = fmaf(gv, dvm[m], gu * dum[m]);
        }
        if (l1 <= wt.gate_rgb) rm |= 2;
    }
    }
}

// one workgroup (blk: its index within this frame's grid) of the tracking
// objective; partials receives the workgroup's 29 sums at row blk
__device__ __forceinline__ void track_p2_block(int blk, const CamC& c, const CamD& cd,
                                               const prism_pose* __restrict__ pose,
                                               const prism_pose* __restrict__ pose_prev,
                                               const float* __restrict__ obs_depth,
                                               const float* __restrict__ obs_rgb,
                                               const float* __restrict__ a_depth,
                                               const float* __restrict__ a_rgb,
                                               const uint8_t* __restrict__ a_mask,
                                               const float* __restrict__ a_normals,
                                               const uint8_t* __restrict__ a_nmask, const WeightsC& wt,
                                               float* __restrict__ Jout, float* __restrict__ resid,
                                               uint8_t* __restrict__ rowmask, double* __restrict__ partials,
                                               const Rel32* __restrict__ grel) {
    __shared__ Rel32 srel;
    __shared__ double lds[kRedLds];
    // the filter's relative pose when it keeps one (copied word by word),
    // else formed here by thread 0
    constexpr int kRelWords = (int)(sizeof(Rel32) / 4);
    static_assert(sizeof(Rel32) % 4 == 0 && kRelWords <= 256, "Rel32 is copied by one word per thread");
    if (grel) {
        if (threadIdx.x < kRelWords)
            reinterpret_cast<unsigned*>(&srel)[threadIdx.x] = reinterpret_cast<const unsigned*>(grel)[threadIdx.x];
    } else if (threadIdx.x == 0) {
        rel_of(pose, pose_prev, srel);
    }
    __syncthreads();
    const Rel32& rel = srel;
    // this pixel's rows summed in single precision (at most 4 rows of
    // single-precision Jacobians), reduced over the workgroup by
    // block_reduce29f (single precision within 32 lanes, then double)
    float pacc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) pacc[q] = 0.0f;
    int p = blk * blockDim.x + threadIdx.x;
    if (p < c.W * c.H) {
        float J[4][6];
        double r[4];
        int rm;
        const float orgb[3] = {obs_rgb[3 * p], obs_rgb[3 * p + 1], obs_rgb[3 * p + 2]};
        p2_pixel(c, cd, rel, p, obs_depth[p], orgb, a_depth, a_rgb, a_mask, a_normals, a_nmask, wt, J, r, rm);
        if (rm & 1) neq_add32(pacc, J[0], (float)r[0], row_weight(wt, false, r[0]));
        if (rm & 2)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) neq_add32(pacc, J[1 + ch], (float)r[1 + ch], row_weight(wt, true, r[1 + ch]));
        if (rm) pacc[28] = 1.0f;
        if (Jout) {
            float4* jo = reinterpret_cast<float4*>(Jout + 24 * (long long)p);
#pragma unroll
            for (int q = 0; q < 6; ++q)
                jo[q] = make_float4(J[(4 * q) / 6][(4 * q) % 6], J[(4 * q + 1) / 6][(4 * q + 1) % 6],
                                    J[(4 * q + 2) / 6][(4 * q + 2) % 6], J[(4 * q + 3) / 6][(4 * q + 3) % 6]);
        }
        if (resid)
            reinterpret_cast<float4*>(resid)[p] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
        if (rowmask) rowmask[p] = (uint8_t)rm;
    }
    block_reduce29f(pacc, lds, partials + (long long)blk * PRISM_NEQ);
}

__global__ __launch_bounds__(256) void k_track_p2(CamC c, CamD cd, const prism_pose* __restrict__ pose,
                                                  const prism_pose* __restrict__ pose_prev,
                                                  const float* __restrict__ obs_depth,
                                                  const float* __restrict__ obs_rgb,
                                                  const float* __restrict__ a_depth,
                                                  const float* __restrict__ a_rgb,
                                                  const uint8_t* __restrict__ a_mask,
                                                  const float* __restrict__ a_normals,
                                                  const uint8_t* __restrict__ a_nmask, WeightsC wt,
                                                  float* __restrict__ Jout, float* __restrict__ resid,
                                                  uint8_t* __restrict__ rowmask,
                                                  double* __restrict__ partials, const Rel32* __restrict__ rel) {
    track_p2_block(blockIdx.x, c, cd, pose, pose_prev, obs_depth, obs_rgb, a_depth, a_rgb, a_mask, a_normals, a_nmask,
                   wt, Jout, resid, rowmask, partials, rel);
}

// batched: every filter tracks its slot's frame from its current iterate
// against its anchor
__global__ __launch_bounds__(256) void k_track_p2_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    const prism_frame& fr = D.slots[b.slot[a]];
    track_p2_block(blockIdx.x - b.start[a], D.c, D.cd, &D.S->iter, &D.S->anchor, (const float*)fr.depth,
                   (const float*)fr.rgb, D.a_depth, D.a_rgb, D.a_mask, D.a_normals, D.a_nmask, b.irls ? D.w_irls : D.w,
                   nullptr, nullptr, nullptr, D.partials, D.rel);
}

// ---------------------------------------------------------------------------
// the paper's pose optimiser: Adam without momentum on sampled pixels
// ---------------------------------------------------------------------------
// One workgroup runs the whole optimisation: at each step the 256 threads
// evaluate the objective's rows on that step's sampled pixels (row-major
// indices; an index outside the image is a pixel without rows; repeated
// indices count repeatedly) at the current iterate, the gradient
//   g = scale * sum 2 w r J + Lp e,   e = pose error of the iterate w.r.t. the prior,
// is reduced in a fixed order, and the step is taken: second moment
// v <- b2 v + (1 - b2) g^2 (first moment off: the step follows g itself),
// bias-corrected vhat = v / (1 - b2^k), delta = -lr g / (sqrt(vhat) + eps),
// iterate <- retract(iterate, delta).  scale = image pixels / sampled pixels
// makes each step's data term an unbiased estimate of the full-image sum.
// The serial part of a step is kept short: the prior term Lp e is formed by
// the last thread while the others evaluate pixels, the six components'
// moments by six lanes, and the iterate is carried as a rotation matrix
// (converted back to a quaternion once, at the end).
// Skipped when the prediction already fell back (improper prior).

// Exp of a rotation vector; the series of sin(th)/th and (1 - cos(th))/th^2
// to th^8 is exact in double precision below th = 0.01
__device__ inline void so3_exp_step(const double w[3], double E[9]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    if (th2 >= 1e-4) {
        so3_exp(w, E, nullptr);
        return;
    }
    const double A = 1.0 - th2 / 6.0 * (1.0 - th2 / 20.0 * (1.0 - th2 / 42.0 * (1.0 - th2 / 72.0)));
    const double B = 0.5 * (1.0 - th2 / 12.0 * (1.0 - th2 / 30.0 * (1.0 - th2 / 56.0 * (1.0 - th2 / 90.0))));
    double K[9], K2[9];
    skew(w, K);
    mat3mul(K, K, K2);
    for (int i = 0; i < 9; ++i) E[i] = A * K[i] + B * K2[i];
    E[0] += 1.0;
    E[4] += 1.0;
    E[8] += 1.0;
}

__global__ __launch_bounds__(256) void k_pose_adam(prism_filter_state* __restrict__ S, CamC c, CamD cd,
                                                   const float* __restrict__ obs_depth,
                                                   const float* __restrict__ obs_rgb,
                                                   const float* __restrict__ a_depth,
                                                   const float* __restrict__ a_rgb,
                                                   const uint8_t* __restrict__ a_mask,
                                                   const float* __restrict__ a_normals,
                                                   const uint8_t* __restrict__ a_nmask, WeightsC wt,
                                                   const int32_t* __restrict__ pixels, AdamC ad) {
    __shared__ Rel32 srel;   // cur: the iterate (double R, t); prev: the anchor pose
    __shared__ double red[4][6];
    __shared__ double lpe[6];
    __shared__ double Rp[9], tp[3];
    __shared__ double Lp[36];
    __shared__ int skip;
    if (threadIdx.x == 0) {
        const prism_pose it = S->iter, pr = S->prior, an = S->anchor;
        skip = (S->flags & PRISM_FLAG_CHOL_FALLBACK) != 0;
        rel_of(&it, &an, srel);
        quat_to_R9(pr.q, Rp);
        for (int i = 0; i < 3; ++i) tp[i] = pr.t[i];
    }
    if (threadIdx.x < 36) Lp[threadIdx.x] = S->Lp[threadIdx.x];
    __syncthreads();
    if (skip) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int npix = c.W * c.H;
    double v2 = 0.0, b2k = 1.0;   // lanes 0..5 of wave 0: second moment of their component
    // the observation at a thread's first sampled pixel does not depend on
    // the pose: it is loaded one step ahead
    auto fetch = [&](int step, int& p, float& D, float rgb[3]) {
        p = -1;
        if ((int)threadIdx.x < ad.n_pix) {
            p = pixels[(long long)step * ad.n_pix + threadIdx.x];
            if ((unsigned)p < (unsigned)npix) {
                D = obs_depth[p];
                rgb[0] = obs_rgb[3 * p];
                rgb[1] = obs_rgb[3 * p + 1];
                rgb[2] = obs_rgb[3 * p + 2];
            } else {
                p = -1;
            }
        }
    };
    int pn;
    float Dn = 0.0f, cn[3] = {0.0f, 0.0f, 0.0f};
    fetch(0, pn, Dn, cn);
    for (int step = 0; step < ad.n_steps; ++step) {
        double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const int p0 = pn;
        const float D0 = Dn, c0[3] = {cn[0], cn[1], cn[2]};
        if (step + 1 < ad.n_steps) fetch(step + 1, pn, Dn, cn);
        for (int j = threadIdx.x; j < ad.n_pix; j += 256) {
            int p;
            float D, orgb[3];
            if (j == (int)threadIdx.x) {
                p = p0;
                D = D0;
                orgb[0] = c0[0];
                orgb[1] = c0[1];
                orgb[2] = c0[2];
                if (p < 0) continue;
            } else {
                p = pixels[(long long)step * ad.n_pix + j];
                if ((unsigned)p >= (unsigned)npix) continue;
                D = obs_depth[p];
                orgb[0] = obs_rgb[3 * p];
                orgb[1] = obs_rgb[3 * p + 1];
                orgb[2] = obs_rgb[3 * p + 2];
            }
            float J[4][6];
            double r[4];
            int rm;
            p2_pixel(c, cd, srel, p, D, orgb, a_depth, a_rgb, a_mask, a_normals, a_nmask, wt, J, r, rm);
            if (rm & 1)
#pragma unroll
                for (int m = 0; m < 6; ++m) g[m] += wt.w_depth * r[0] * (double)J[0][m];
            if (rm & 2)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch)
#pragma unroll
                    for (int m = 0; m < 6; ++m) g[m] += wt.w_rgb * r[1 + ch] * (double)J[1 + ch][m];
        }
        if (threadIdx.x == 255) {
            // prior term at the current iterate: e = (t - tp, Log(R Rp^T))
            double M[9], e[6];
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k)
                    M[i * 3 + k] = srel.cur.R[i][0] * Rp[k * 3] + srel.cur.R[i][1] * Rp[k * 3 + 1] +
                                   srel.cur.R[i][2] * Rp[k * 3 + 2];
            for (int i = 0; i < 3; ++i) e[i] = srel.cur.t[i] - tp[i];
            so3_log(M, e + 3);
            for (int i = 0; i < 6; ++i) {
                double s = 0.0;
                for (int k = 0; k < 6; ++k) s += Lp[i * 6 + k] * e[k];
                lpe[i] = s;
            }
        }
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) g[m] += __shfl_xor(g[m], off, 64);
        if (lane == 0)
#pragma unroll
            for (int m = 0; m < 6; ++m) red[wv][m] = g[m];
        __syncthreads();
        if (wv == 0) {
            double di = 0.0;
            if (lane < 6) {
                const double gi = 2.0 * ad.scale * ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) +
                                  lpe[lane];
                b2k *= ad.beta2;
                v2 = ad.beta2 * v2 + (1.0 - ad.beta2) * gi * gi;
                const double vhat = v2 / (1.0 - b2k);
                di = -ad.lr[lane] * gi / (sqrt(vhat) + ad.eps);
            }
            double d[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) d[m] = __shfl(di, m, 64);
            if (lane == 0) {
                double E[9], R[9], R2[9];
                so3_exp_step(d + 3, E);
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) R[i * 3 + k] = srel.cur.R[i][k];
                mat3mul(E, R, R2);
                const Pose64& Q = srel.prev;
                double t[3], dd[3];
                for (int i = 0; i < 3; ++i) {
                    t[i] = srel.cur.t[i] + d[i];
                    dd[i] = t[i] - Q.t[i];
                }
                for (int a = 0; a < 3; ++a) {
                    for (int b = 0; b < 3; ++b)
                        srel.R[a][b] = (float)((Q.R[0][a] * R2[b] + Q.R[1][a] * R2[3 + b]) + Q.R[2][a] * R2[6 + b]);
                    srel.t[a] = (float)((Q.R[0][a] * dd[0] + Q.R[1][a] * dd[1]) + Q.R[2][a] * dd[2]);
                }
                for (int i = 0; i < 3; ++i) {
                    srel.cur.t[i] = t[i];
                    for (int k = 0; k < 3; ++k) srel.cur.R[i][k] = R2[i * 3 + k];
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double R[9];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) R[i * 3 + k] = srel.cur.R[i][k];
        prism_pose it;
        for (int i = 0; i < 3; ++i) it.t[i] = srel.cur.t[i];
        R9_to_quat(R, it.q);
        S->iter = it;
    }
}

hipError_t launch_pose_adam(prism_filter_state* S, const CamC& c, const CamD& cd, const float* obs_depth,
                            const float* obs_rgb, const float* a_depth, const float* a_rgb, const uint8_t* a_mask,
                            const float* a_normals, const uint8_t* a_nmask, const WeightsC& w, const int32_t* pixels,
                            const AdamC& ad, hipStream_t st) {
    k_pose_adam<<<1, 256, 0, st>>>(S, c, cd, obs_depth, obs_rgb, a_depth, a_rgb, a_mask, a_normals, a_nmask, w, pixels,
                                   ad);
    return hipGetLastError();
}

int track_blocks(const CamC& c) { return (c.W * c.H + 255) / 256; }

hipError_t launch_track_p2_batch(const BatchArgs& b, hipStream_t st) {
    k_track_p2_batch<<<b.start[b.n], 256, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_track_p2(const CamC& c, const CamD& cd, const prism_pose* pose, const prism_pose* pose_prev,
                           const float* obs_depth, const float* obs_rgb, const float* a_depth,
                           const float* a_rgb, const uint8_t* a_mask, const float* a_normals,
                           const uint8_t* a_nmask, const WeightsC& w, float* J, float* resid,
                           uint8_t* rowmask, double* partials, const Rel32* rel, hipStream_t st) {
    k_track_p2<<<track_blocks(c), 256, 0, st>>>(c, cd, pose, pose_prev, obs_depth, obs_rgb, a_depth, a_rgb,
                                                a_mask, a_normals, a_nmask, w, J, resid, rowmask, partials, rel);
    return hipGetLastError();
}

}  // namespace prism
