// Ray-marching emission (App. B), its pose Jacobian with the fused normal-
// equation reduction, anchor normals, and the adjoint w.r.t. map means.
//
// Work split: one ray per lane, an 8x8 pixel tile per wave, 4 waves (16x16
// pixels) per workgroup, blockIdx.y = frame.  The sample loop evaluates
// kUnroll samples per trip so that 8*kUnroll independent gathers are in
// flight per lane before the first-crossing test; samples past the hit are
// evaluated but never used.
#include "common.hpp"
#include "launch.hpp"

namespace prism {

constexpr int kUnroll = 4;

struct RayHit {
    int k;          // k* or -1
    float f0, f1;   // occupancy at k*-1, k*
    Cell c0, c1;    // cells of samples k*-1, k*
};

template <typename T>
__device__ __forceinline__ float occ_at(const GridC& g, const T* occ, const Cell& c) {
    float v[8];
    corners(g, occ, c, g.occ_out, v);
    return trilerp(v, c.w);
}

// first sample whose occupancy exceeds tau (strictly), with the bracketing cells
template <typename T>
__device__ __forceinline__ RayHit march(const GridC& g, const CamC& c, const Pose32& P,
                                        const float dir[3], const T* occ) {
    RayHit h;
    h.k = -1;
    h.f0 = h.f1 = 0.0f;
    Cell prev = {};
    float fprev = 0.0f;
    for (int k0 = 0; k0 < c.K; k0 += kUnroll) {
        float f[kUnroll];
        Cell cl[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            int k = min(k0 + j, c.K - 1);
            cl[j] = sample_cell(g, c, P, dir, k);
            f[j] = occ_at(g, occ, cl[j]);
        }
        bool done = false;
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            if (!done && k0 + j < c.K) {
                if (f[j] > c.tau) {
                    h.k = k0 + j;
                    h.f1 = f[j];
                    h.c1 = cl[j];
                    h.f0 = fprev;
                    h.c0 = prev;
                    done = true;
                } else {
                    fprev = f[j];
                    prev = cl[j];
                }
            }
        }
        if (done) break;
    }
    return h;
}

struct Shade {
    float alpha, d0, d1;       // single-precision copies for the Jacobian
    float c0[3], c1[3];
    float w0[3], w1[3];        // interpolation weights from the double-precision points
    double depth, rgb[3];      // double-precision values at the hit
    double f0, f1;
};

// trilinear value of one plane in double precision: cell from the decision
// recipe, weights from the double-precision grid coordinate, sum over the 8
// corners of the product of 1-D hat weights (z, y, x order)
template <typename T>
__device__ __forceinline__ double tri64(const GridC& g, const T* plane, const double gc[3], const int cell[3],
                                        double outv) {
    double w0 = gc[0] - (double)cell[0], w1 = gc[1] - (double)cell[1], w2 = gc[2] - (double)cell[2];
    double s = 0.0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                double hx = cx ? w0 : 1.0 - w0;
                double hy = cy ? w1 : 1.0 - w1;
                double hz = cz ? w2 : 1.0 - w2;
                int i = cell[0] + cx, j = cell[1] + cy, k = cell[2] + cz;
                bool in = (unsigned)i < (unsigned)g.n && (unsigned)j < (unsigned)g.n && (unsigned)k < (unsigned)g.n;
                double V = in ? (double)ld(plane, vidx(g, i, j, k)) : outv;
                s += hx * hy * hz * V;
            }
    return s;
}

// double-precision sample point k of the ray with direction dir (world)
__device__ __forceinline__ void grid_coord64(const GridD& gd, const CamD& cd, const Pose64& P, const double dir[3],
                                             int k, double gc[3]) {
    double dk = cd.dn + (double)k * cd.step;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = P.t[a] + dk * dir[a];
        gc[a] = (p - gd.o[a]) / gd.s - 0.5;
    }
}

template <typename T>
__device__ __forceinline__ Shade shade(const GridC& g, const GridD& gd, const CamD& cd, const Pose64& P, int u,
                                       int v, const T* map, const RayHit& h) {
    Shade s;
    double rc[3], dir[3], gc0[3], gc1[3];
    pixel_dir64(cd, u, v, rc);
#pragma unroll
    for (int a = 0; a < 3; ++a) dir[a] = P.R[a][0] * rc[0] + P.R[a][1] * rc[1] + P.R[a][2] * rc[2];
    grid_coord64(gd, cd, P, dir, h.k - 1, gc0);
    grid_coord64(gd, cd, P, dir, h.k, gc1);
    double d0 = cd.dn + (double)(h.k - 1) * cd.step;
    double d1 = cd.dn + (double)h.k * cd.step;
    s.f0 = tri64(g, map, gc0, h.c0.i, gd.occ_out);
    s.f1 = tri64(g, map, gc1, h.c1.i, gd.occ_out);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.w0[a] = (float)(gc0[a] - (double)h.c0.i[a]);
        s.w1[a] = (float)(gc1[a] - (double)h.c1.i[a]);
    }
    double al = (cd.tau - s.f0) / (s.f1 - s.f0);
    s.depth = al * d1 + (1.0 - al) * d0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const T* pl = map + (long long)(1 + ch) * g.nvox;
        double c0 = tri64(g, pl, gc0, h.c0.i, gd.rgb_out);
        double c1 = tri64(g, pl, gc1, h.c1.i, gd.rgb_out);
        s.rgb[ch] = al * c1 + (1.0 - al) * c0;
        s.c0[ch] = (float)c0;
        s.c1[ch] = (float)c1;
    }
    s.alpha = (float)al;
    s.d0 = (float)d0;
    s.d1 = (float)d1;
    return s;
}

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// d(depth, r, g, b)/d(delta) of a valid ray (k* held fixed)
template <typename T>
__device__ __forceinline__ void ray_jacobian(const GridC& g, const T* map, const RayHit& h,
                                             const Shade& s, const float dir[3], float J[4][6]) {
    float a0[3], a1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) { a0[i] = s.d0 * dir[i]; a1[i] = s.d1 * dir[i]; }
    float v[8], gr0[3], gr1[3], cr[3];
    corners(g, map, h.c0, g.occ_out, v);
    trigrad(v, s.w0, gr0);
    corners(g, map, h.c1, g.occ_out, v);
    trigrad(v, s.w1, gr1);
    float rf0[6], rf1[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) { gr0[i] *= g.inv_s; gr1[i] *= g.inv_s; rf0[i] = gr0[i]; rf1[i] = gr1[i]; }
    cross3(a0, gr0, cr);
#pragma unroll
    for (int i = 0; i < 3; ++i) rf0[3 + i] = cr[i];
    cross3(a1, gr1, cr);
#pragma unroll
    for (int i = 0; i < 3; ++i) rf1[3 + i] = cr[i];
    float inv_den = (float)(1.0 / (s.f1 - s.f0));
    float al = s.alpha;
    float dal[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) dal[m] = -((1.0f - al) * rf0[m] + al * rf1[m]) * inv_den;
#pragma unroll
    for (int m = 0; m < 6; ++m) J[0][m] = (s.d1 - s.d0) * dal[m];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const T* pl = map + (long long)(1 + ch) * g.nvox;
        float G0[3], G1[3], g0[6], g1[6];
        corners(g, pl, h.c0, g.rgb_out, v);
        trigrad(v, s.w0, G0);
        corners(g, pl, h.c1, g.rgb_out, v);
        trigrad(v, s.w1, G1);
#pragma unroll
        for (int i = 0; i < 3; ++i) { G0[i] *= g.inv_s; G1[i] *= g.inv_s; g0[i] = G0[i]; g1[i] = G1[i]; }
        cross3(a0, G0, cr);
#pragma unroll
        for (int i = 0; i < 3; ++i) g0[3 + i] = cr[i];
        cross3(a1, G1, cr);
#pragma unroll
        for (int i = 0; i < 3; ++i) g1[3 + i] = cr[i];
        float dc = s.c1[ch] - s.c0[ch];
#pragma unroll
        for (int m = 0; m < 6; ++m) J[1 + ch][m] = dc * dal[m] + al * g1[m] + (1.0f - al) * g0[m];
    }
}

__device__ __forceinline__ void tile_pixel(const CamC& c, int& u, int& v) {
    int tiles_x = (c.W + 15) >> 4;
    int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    u = (bx << 4) + ((wv & 1) << 3) + (l & 7);
    v = (by << 4) + ((wv >> 1) << 3) + (l >> 3);
}

struct BlockPose {
    Pose64 d;
    Pose32 f;
};

__device__ __forceinline__ const BlockPose& block_pose(const prism_pose* poses, BlockPose* sp) {
    if (threadIdx.x == 0) {
        sp->d = load_pose64(poses + blockIdx.y);
        sp->f = to32(sp->d);
    }
    __syncthreads();
    return *sp;
}

// ---------------------------------------------------------------------------
// render
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_render(GridC g, CamC c, GridD gd, CamD cd, const T* __restrict__ map,
                                                const prism_pose* __restrict__ poses,
                                                float* __restrict__ depth, float* __restrict__ rgb,
                                                uint8_t* __restrict__ mask, int32_t* __restrict__ hit_k) {
    __shared__ BlockPose sp;
    const BlockPose& P = block_pose(poses, &sp);
    int u, v;
    tile_pixel(c, u, v);
    if (u >= c.W || v >= c.H) return;
    float dir[3];
    ray_dir32(c, P.f, u, v, dir);
    RayHit h = march(g, c, P.f, dir, map);
    long long pix = (long long)blockIdx.y * c.W * c.H + (long long)v * c.W + u;
    if (hit_k) hit_k[pix] = h.k;
    if (h.k >= 1) {
        Shade s = shade(g, gd, cd, P.d, u, v, map, h);
        depth[pix] = (float)s.depth;
        rgb[3 * pix] = (float)s.rgb[0];
        rgb[3 * pix + 1] = (float)s.rgb[1];
        rgb[3 * pix + 2] = (float)s.rgb[2];
        mask[pix] = 1;
    } else {
        depth[pix] = 0.0f;
        rgb[3 * pix] = rgb[3 * pix + 1] = rgb[3 * pix + 2] = 0.0f;
        mask[pix] = 0;
    }
}

// ---------------------------------------------------------------------------
// normals of a rendered depth image
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_normals(CamC c, int n_frames, const float* __restrict__ depth,
                                                 const uint8_t* __restrict__ mask, float disc,
                                                 float* __restrict__ normals, uint8_t* __restrict__ nmask) {
    long long npix = (long long)c.W * c.H;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= npix * n_frames) return;
    long long f = gid / npix;
    int p = (int)(gid - f * npix);
    int u = p % c.W, v = p / c.W;
    const float* D = depth + f * npix;
    const uint8_t* M = mask + f * npix;
    float* N = normals + 3 * gid;
    N[0] = N[1] = N[2] = 0.0f;
    nmask[gid] = 0;
    if (u == 0 || v == 0 || u == c.W - 1 || v == c.H - 1 || !M[p]) return;
    if (!M[p - 1] || !M[p + 1] || !M[p - c.W] || !M[p + c.W]) return;
    float d = D[p], dl = D[p - 1], dr = D[p + 1], du = D[p - c.W], dd = D[p + c.W];
    if (fabsf(dl - d) > disc || fabsf(dr - d) > disc || fabsf(du - d) > disc || fabsf(dd - d) > disc)
        return;
    float xl = ((float)(u - 1) + 0.5f - c.cx) * c.ifx, xr = ((float)(u + 1) + 0.5f - c.cx) * c.ifx;
    float x0 = ((float)u + 0.5f - c.cx) * c.ifx;
    float yu = ((float)(v - 1) + 0.5f - c.cy) * c.ify, yd = ((float)(v + 1) + 0.5f - c.cy) * c.ify;
    float y0 = ((float)v + 0.5f - c.cy) * c.ify;
    float a[3] = {dr * xr - dl * xl, dr * y0 - dl * y0, dr - dl};
    float b[3] = {dd * x0 - du * x0, dd * yd - du * yu, dd - du};
    float n[3];
    cross3(a, b, n);
    float len = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(len > 0.0f)) return;
    float sgn = (n[0] * x0 + n[1] * y0 + n[2]) * d < 0.0f ? 1.0f : -1.0f;
    float il = sgn / len;
    N[0] = n[0] * il;
    N[1] = n[1] * il;
    N[2] = n[2] * il;
    nmask[gid] = 1;
}

// ---------------------------------------------------------------------------
// render + P1 Jacobian + gated weighted normal equations
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_render_jac(GridC g, CamC c, GridD gd, CamD cd, const T* __restrict__ map,
                                                    const prism_pose* __restrict__ poses,
                                                    const float* __restrict__ obs_depth,
                                                    const float* __restrict__ obs_rgb, WeightsC wt,
                                                    float* __restrict__ depth, float* __restrict__ rgb,
                                                    uint8_t* __restrict__ mask, float* __restrict__ Jout,
                                                    float* __restrict__ resid, uint8_t* __restrict__ rowmask,
                                                    double* __restrict__ partials) {
    __shared__ BlockPose sp;
    __shared__ double lds[PRISM_NEQ * 16];
    const BlockPose& P = block_pose(poses, &sp);
    int u, v;
    tile_pixel(c, u, v);
    double acc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) acc[q] = 0.0;
    if (u < c.W && v < c.H) {
        float dir[3];
        ray_dir32(c, P.f, u, v, dir);
        RayHit h = march(g, c, P.f, dir, map);
        long long pix = (long long)blockIdx.y * c.W * c.H + (long long)v * c.W + u;
        float J[4][6];
        double r[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int m = 0; m < 6; ++m) J[a][m] = 0.0f;
        uint8_t rm = 0;
        bool valid = h.k >= 1;
        Shade s;
        if (valid) {
            s = shade(g, gd, cd, P.d, u, v, map, h);
            float D = obs_depth[pix];
            if (depth_ok(D)) {
                ray_jacobian(g, map, h, s, dir, J);
                r[0] = s.depth - (double)D;
                double l1 = 0.0;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    r[1 + ch] = s.rgb[ch] - (double)obs_rgb[3 * pix + ch];
                    l1 += fabs(r[1 + ch]);
                }
                if (fabs(r[0]) <= wt.gate_depth) {
                    neq_add(acc, J[0], r[0], wt.w_depth);
                    rm |= 1;
                }
                if (l1 <= wt.gate_rgb) {
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) neq_add(acc, J[1 + ch], r[1 + ch], wt.w_rgb);
                    rm |= 2;
                }
                if (rm) acc[28] = 1.0;
            }
            if (!rm) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int m = 0; m < 6; ++m) J[a][m] = 0.0f;
            }
        }
        if (depth) depth[pix] = valid ? (float)s.depth : 0.0f;
        if (rgb) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) rgb[3 * pix + ch] = valid ? (float)s.rgb[ch] : 0.0f;
        }
        if (mask) mask[pix] = valid ? 1 : 0;
        if (Jout) {
            float4* jo = reinterpret_cast<float4*>(Jout + 24 * pix);
#pragma unroll
            for (int q = 0; q < 6; ++q)
                jo[q] = make_float4(J[(4 * q) / 6][(4 * q) % 6], J[(4 * q + 1) / 6][(4 * q + 1) % 6],
                                    J[(4 * q + 2) / 6][(4 * q + 2) % 6], J[(4 * q + 3) / 6][(4 * q + 3) % 6]);
        }
        if (resid)
            reinterpret_cast<float4*>(resid)[pix] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
        if (rowmask) rowmask[pix] = rm;
    }
    block_reduce29(acc, lds, partials + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * PRISM_NEQ);
}

// ---------------------------------------------------------------------------
// adjoint of render w.r.t. map means (atomic scatter) and pose
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_render_vjp(GridC g, CamC c, GridD gd, CamD cd, const float* __restrict__ map,
                                                    const prism_pose* __restrict__ poses,
                                                    const int32_t* __restrict__ hit_k,
                                                    const float* __restrict__ g_depth,
                                                    const float* __restrict__ g_rgb,
                                                    float* __restrict__ grad_mean,
                                                    double* __restrict__ partials) {
    __shared__ BlockPose sp;
    __shared__ double lds[PRISM_NEQ * 16];
    const BlockPose& P = block_pose(poses, &sp);
    int u, v;
    tile_pixel(c, u, v);
    double acc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) acc[q] = 0.0;
    if (u < c.W && v < c.H) {
        long long pix = (long long)blockIdx.y * c.W * c.H + (long long)v * c.W + u;
        int k = hit_k[pix];
        if (k >= 1 && k < c.K) {
            float dir[3];
            ray_dir32(c, P.f, u, v, dir);
            RayHit h;
            h.k = k;
            h.c0 = sample_cell(g, c, P.f, dir, k - 1);
            h.c1 = sample_cell(g, c, P.f, dir, k);
            h.f0 = occ_at(g, map, h.c0);
            h.f1 = occ_at(g, map, h.c1);
            if (h.f1 > c.tau && !(h.f0 > c.tau)) {
                Shade s = shade(g, gd, cd, P.d, u, v, map, h);
                float gd = g_depth[pix];
                float gc[3] = {g_rgb[3 * pix], g_rgb[3 * pix + 1], g_rgb[3 * pix + 2]};
                float J[4][6];
                ray_jacobian(g, map, h, s, dir, J);
#pragma unroll
                for (int m = 0; m < 6; ++m)
                    acc[m] = (double)(gd * J[0][m] + gc[0] * J[1][m] + gc[1] * J[2][m] + gc[2] * J[3][m]);
                float al = s.alpha;
                float ga = gd * (s.d1 - s.d0) + gc[0] * (s.c1[0] - s.c0[0]) + gc[1] * (s.c1[1] - s.c0[1]) +
                           gc[2] * (s.c1[2] - s.c0[2]);
                float inv_den = (float)(1.0 / (s.f1 - s.f0));
                float gf[2] = {-ga * (1.0f - al) * inv_den, -ga * al * inv_den};
                float cw[2] = {1.0f - al, al};
#pragma unroll
                for (int sm = 0; sm < 2; ++sm) {
                    const Cell& cl = sm ? h.c1 : h.c0;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
                        int i = cl.i[0] + dx, j = cl.i[1] + dy, kk = cl.i[2] + dz;
                        if ((unsigned)i >= (unsigned)g.n || (unsigned)j >= (unsigned)g.n ||
                            (unsigned)kk >= (unsigned)g.n)
                            continue;
                        const float* cw3 = sm ? s.w1 : s.w0;
                        float hw = (dx ? cw3[0] : 1.0f - cw3[0]) * (dy ? cw3[1] : 1.0f - cw3[1]) *
                                   (dz ? cw3[2] : 1.0f - cw3[2]);
                        long long id = vidx(g, i, j, kk);
                        atomicAdd(grad_mean + id, gf[sm] * hw);
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch)
                            atomicAdd(grad_mean + (long long)(1 + ch) * g.nvox + id, gc[ch] * cw[sm] * hw);
                    }
                }
            }
        }
    }
    block_reduce29(acc, lds, partials + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * PRISM_NEQ);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int render_blocks(const CamC& c) { return ((c.W + 15) >> 4) * ((c.H + 15) >> 4); }

hipError_t launch_render(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, int dtype, const void* map,
                         const prism_pose* poses, int n_frames, float* depth, float* rgb, uint8_t* mask,
                         int32_t* hit_k, hipStream_t st) {
    dim3 grid(render_blocks(c), n_frames);
    if (dtype == PRISM_BF16)
        k_render<uint16_t><<<grid, 256, 0, st>>>(g, c, gd, cd, (const uint16_t*)map, poses, depth, rgb, mask, hit_k);
    else
        k_render<float><<<grid, 256, 0, st>>>(g, c, gd, cd, (const float*)map, poses, depth, rgb, mask, hit_k);
    return hipGetLastError();
}

hipError_t launch_normals(const CamC& c, int n_frames, const float* depth, const uint8_t* mask, float disc,
                          float* normals, uint8_t* nmask, hipStream_t st) {
    long long n = (long long)c.W * c.H * n_frames;
    k_normals<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(c, n_frames, depth, mask, disc, normals, nmask);
    return hipGetLastError();
}

hipError_t launch_render_jac(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, int dtype,
                             const void* map, const prism_pose* poses, int n_frames, const float* obs_depth,
                             const float* obs_rgb, const WeightsC& w, float* depth, float* rgb, uint8_t* mask,
                             float* J, float* resid, uint8_t* rowmask, double* partials, hipStream_t st) {
    dim3 grid(render_blocks(c), n_frames);
    if (dtype == PRISM_BF16)
        k_render_jac<uint16_t><<<grid, 256, 0, st>>>(g, c, gd, cd, (const uint16_t*)map, poses, obs_depth, obs_rgb,
                                                     w, depth, rgb, mask, J, resid, rowmask, partials);
    else
        k_render_jac<float><<<grid, 256, 0, st>>>(g, c, gd, cd, (const float*)map, poses, obs_depth, obs_rgb, w,
                                                  depth, rgb, mask, J, resid, rowmask, partials);
    return hipGetLastError();
}

hipError_t launch_render_vjp(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, const float* map,
                             const prism_pose* poses, int n_frames, const int32_t* hit_k, const float* g_depth,
                             const float* g_rgb, float* grad_mean, double* partials, hipStream_t st) {
    dim3 grid(render_blocks(c), n_frames);
    k_render_vjp<<<grid, 256, 0, st>>>(g, c, gd, cd, map, poses, hit_k, g_depth, g_rgb, grad_mean, partials);
    return hipGetLastError();
}

}  // namespace prism
