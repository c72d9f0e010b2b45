// Prediction-to-observation tracking objective (App. E.3): point-to-plane
// against the nearest anchor pixel and photometric error against the
// bilinearly interpolated anchor colour, with the fused reduction of the
// gated, weighted normal equations.  One observed pixel per lane, pixels in
// row-major order so observation reads are coalesced; anchor reads are
// gathers around the reprojected location.
#include "common.hpp"
#include "launch.hpp"

namespace prism {

struct Rel32 {
    float R[3][3], t[3];   // current camera -> anchor camera (association recipe)
    Pose64 cur, prev;      // both poses in double precision (values)
};

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
                                               uint8_t* __restrict__ rowmask, double* __restrict__ partials) {
    __shared__ Rel32 srel;
    __shared__ double lds[kRedLds];
    if (threadIdx.x == 0) {
        Pose64 P = load_pose64(pose), Q = load_pose64(pose_prev);
        double d[3] = {P.t[0] - Q.t[0], P.t[1] - Q.t[1], P.t[2] - Q.t[2]};
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b)
                srel.R[a][b] = (float)((Q.R[0][a] * P.R[0][b] + Q.R[1][a] * P.R[1][b]) + Q.R[2][a] * P.R[2][b]);
            srel.t[a] = (float)((Q.R[0][a] * d[0] + Q.R[1][a] * d[1]) + Q.R[2][a] * d[2]);
        }
        srel.cur = P;
        srel.prev = Q;
    }
    __syncthreads();
    const Rel32& rel = srel;
    // this pixel's rows summed in single precision (at most 4 rows of
    // single-precision Jacobians), widened once for the double-precision
    // reduction over pixels
    float pacc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) pacc[q] = 0.0f;
    int p = blk * blockDim.x + threadIdx.x;
    if (p < c.W * c.H) {
        int u = p % c.W, v = p / c.W;
        float J[4][6];
        double r[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int m = 0; m < 6; ++m) J[a][m] = 0.0f;
        uint8_t rm = 0;
        float D = obs_depth[p];
        if (depth_ok(D)) {
            float rx = ((float)u + 0.5f - c.cx) * c.ifx;
            float ry = ((float)v + 0.5f - c.cy) * c.ify;
            float X[3] = {D * rx, D * ry, D};
            float Y[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                Y[a] = ((rel.R[a][0] * X[0] + rel.R[a][1] * X[1]) + rel.R[a][2] * X[2]) + rel.t[a];
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
            if (geo || pho) {
                // values in double precision: back-projected point, moved into
                // the anchor camera; Jacobians in single precision
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
                    dY[a][3] = RX[1] * e2 - RX[2] * e1;
                    dY[a][4] = RX[2] * e0 - RX[0] * e2;
                    dY[a][5] = RX[0] * e1 - RX[1] * e0;
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
                    for (int m = 0; m < 6; ++m) J[0][m] = -(fn0 * dY[0][m] + fn1 * dY[1][m] + fn2 * dY[2][m]);
                    if (fabs(rg) <= wt.gate_depth) {
                        neq_add32(pacc, J[0], (float)rg, (float)wt.w_depth);
                        rm |= 1;
                    }
                }
                if (pho) {
                    double ud = cd.fx * Yd[0] / Yd[2] + cd.cx;
                    double vd = cd.fy * Yd[1] / Yd[2] + cd.cy;
                    double ax = (ud - 0.5) - (double)bix, ay = (vd - 0.5) - (double)biy;
                    float Y2 = (float)Yd[2];
                    float iz = 1.0f / Y2;
                    float du_[3] = {c.fx * iz, 0.0f, -c.fx * (float)Yd[0] * iz * iz};
                    float dv_[3] = {0.0f, c.fy * iz, -c.fy * (float)Yd[1] * iz * iz};
                    float dum[6], dvm[6];
#pragma unroll
                    for (int m = 0; m < 6; ++m) {
                        dum[m] = du_[0] * dY[0][m] + du_[2] * dY[2][m];
                        dvm[m] = dv_[1] * dY[1][m] + dv_[2] * dY[2][m];
                    }
                    double l1 = 0.0;
                    double rp[3];
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        double I00 = a_rgb[3 * q00 + ch], I10 = a_rgb[3 * (q00 + 1) + ch];
                        double I01 = a_rgb[3 * (q00 + c.W) + ch], I11 = a_rgb[3 * (q00 + c.W + 1) + ch];
                        double Ii = (1 - ax) * (1 - ay) * I00 + ax * (1 - ay) * I10 + (1 - ax) * ay * I01 + ax * ay * I11;
                        float gu = (float)((1 - ay) * (I10 - I00) + ay * (I11 - I01));
                        float gv = (float)((1 - ax) * (I01 - I00) + ax * (I11 - I10));
                        rp[ch] = Ii - (double)obs_rgb[3 * p + ch];
                        r[1 + ch] = rp[ch];
                        l1 += fabs(rp[ch]);
#pragma unroll
                        for (int m = 0; m < 6; ++m) J[1 + ch][m] = gu * dum[m] + gv * dvm[m];
                    }
                    if (l1 <= wt.gate_rgb) {
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) neq_add32(pacc, J[1 + ch], (float)rp[ch], (float)wt.w_rgb);
                        rm |= 2;
                    }
                }
                if (rm) pacc[28] = 1.0f;
            }
        }
        if (Jout) {
            float4* jo = reinterpret_cast<float4*>(Jout + 24 * (long long)p);
#pragma unroll
            for (int q = 0; q < 6; ++q)
                jo[q] = make_float4(J[(4 * q) / 6][(4 * q) % 6], J[(4 * q + 1) / 6][(4 * q + 1) % 6],
                                    J[(4 * q + 2) / 6][(4 * q + 2) % 6], J[(4 * q + 3) / 6][(4 * q + 3) % 6]);
        }
        if (resid)
            reinterpret_cast<float4*>(resid)[p] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
        if (rowmask) rowmask[p] = rm;
    }
    double acc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) acc[q] = (double)pacc[q];
    block_reduce29(acc, lds, partials + (long long)blk * PRISM_NEQ);
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
                                                  double* __restrict__ partials) {
    track_p2_block(blockIdx.x, c, cd, pose, pose_prev, obs_depth, obs_rgb, a_depth, a_rgb, a_mask, a_normals, a_nmask,
                   wt, Jout, resid, rowmask, partials);
}

// batched: every filter tracks its slot's frame from its current iterate
// against its anchor
__global__ __launch_bounds__(256) void k_track_p2_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    const prism_frame& fr = D.slots[b.slot[a]];
    track_p2_block(blockIdx.x - b.start[a], D.c, D.cd, &D.S->iter, &D.S->anchor, (const float*)fr.depth,
                   (const float*)fr.rgb, D.a_depth, D.a_rgb, D.a_mask, D.a_normals, D.a_nmask, D.w, nullptr, nullptr,
                   nullptr, D.partials);
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
                           uint8_t* rowmask, double* partials, hipStream_t st) {
    k_track_p2<<<track_blocks(c), 256, 0, st>>>(c, cd, pose, pose_prev, obs_depth, obs_rgb, a_depth, a_rgb,
                                                a_mask, a_normals, a_nmask, w, J, resid, rowmask, partials);
    return hipGetLastError();
}

}  // namespace prism
