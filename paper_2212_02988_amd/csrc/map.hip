// Voxel-map storage kernels and the closed-form map update (App. D).
//
// Storage: 8 planes (mean occ, R, G, B, var occ, R, G, B) of n^3 values in
// 8x8x8-brick order, brick-major, x fastest inside a brick.  The map update
// runs one workgroup per brick: the brick's voxel-centre box is first tested
// against the view frustum (conservatively, with margins far above single-
// precision rounding), then each lane decides its voxels with the single-
// precision recipe and updates only those, so HBM traffic is the updated
// voxels' 8 planes read and written once.
#include "common.hpp"
#include "launch.hpp"

namespace prism {

template <typename T>
__global__ __launch_bounds__(256) void k_map_init(long long nvox, T* __restrict__ map, float occ0, float rgb0,
                                                  float var0) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nvox) return;
    st(map, i, occ0);
    st(map, nvox + i, rgb0);
    st(map, 2 * nvox + i, rgb0);
    st(map, 3 * nvox + i, rgb0);
#pragma unroll
    for (int c = 4; c < 8; ++c) st(map, c * nvox + i, var0);
}

// dense index (k*n + j)*n + i  <->  brick index
__device__ __forceinline__ long long dense_of_brick(int n, int nb, long long b_idx) {
    long long b = b_idx >> 9;
    int l = (int)(b_idx & 511);
    int bx = (int)(b % nb), by = (int)((b / nb) % nb), bz = (int)(b / ((long long)nb * nb));
    int i = (bx << 3) | (l & 7), j = (by << 3) | ((l >> 3) & 7), k = (bz << 3) | (l >> 6);
    return ((long long)k * n + j) * n + i;
}

template <typename T>
__global__ __launch_bounds__(256) void k_from_dense(int n, int nb, T* __restrict__ map,
                                                    const float* __restrict__ mean4,
                                                    const float* __restrict__ var4) {
    long long nvox = (long long)n * n * n;
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nvox) return;
    long long d = dense_of_brick(n, nb, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (mean4) st(map, c * nvox + b, mean4[c * nvox + d]);
        if (var4) st(map, (4 + c) * nvox + b, var4[c * nvox + d]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_to_dense(int n, int nb, const T* __restrict__ map,
                                                  float* __restrict__ mean4, float* __restrict__ var4) {
    long long nvox = (long long)n * n * n;
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nvox) return;
    long long d = dense_of_brick(n, nb, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (mean4) mean4[c * nvox + d] = ld(map, c * nvox + b);
        if (var4) var4[c * nvox + d] = ld(map, (4 + c) * nvox + b);
    }
}

__global__ __launch_bounds__(256) void k_planes(int n, int nb, int channels, const float* __restrict__ src,
                                                float* __restrict__ dst, int to_dense) {
    long long nvox = (long long)n * n * n;
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nvox) return;
    long long d = dense_of_brick(n, nb, b);
    for (int c = 0; c < channels; ++c) {
        if (to_dense)
            dst[c * nvox + d] = src[c * nvox + b];
        else
            dst[c * nvox + b] = src[c * nvox + d];
    }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

struct MapUpdC {
    float trunc32;          // decision: z <= D + trunc in single precision
    double trunc, lam_u;    // values
};

// Conservative brick cull: true if no voxel centre of the brick can pass the
// per-voxel test.  Each test is a convex region (intersection of half-spaces)
// checked on the 8 corners of the brick's voxel-centre box.
__device__ inline bool brick_culled(const GridC& g, const CamC& c, const Pose32& P, int bx, int by, int bz) {
    const float mz = 1e-3f, mp = 0.5f;
    bool all_behind = true, all_l = true, all_r = true, all_t = true, all_b = true;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float x[3] = {g.o[0] + g.s * ((float)((bx << 3) + ((q & 1) ? 7 : 0)) + 0.5f),
                      g.o[1] + g.s * ((float)((by << 3) + ((q & 2) ? 7 : 0)) + 0.5f),
                      g.o[2] + g.s * ((float)((bz << 3) + ((q & 4) ? 7 : 0)) + 0.5f)};
        float d[3] = {x[0] - P.t[0], x[1] - P.t[1], x[2] - P.t[2]};
        float X = P.R[0][0] * d[0] + P.R[1][0] * d[1] + P.R[2][0] * d[2];
        float Y = P.R[0][1] * d[0] + P.R[1][1] * d[1] + P.R[2][1] * d[2];
        float Z = P.R[0][2] * d[0] + P.R[1][2] * d[1] + P.R[2][2] * d[2];
        bool front = Z > mz;
        all_behind &= Z < -mz;
        all_l &= front && (c.fx * X + (c.cx + mp) * Z < 0.0f);
        all_r &= front && (c.fx * X + (c.cx - (float)c.W - mp) * Z > 0.0f);
        all_t &= front && (c.fy * Y + (c.cy + mp) * Z < 0.0f);
        all_b &= front && (c.fy * Y + (c.cy - (float)c.H - mp) * Z > 0.0f);
    }
    return all_behind || all_l || all_r || all_t || all_b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_map_update(GridC g, CamC c, GridD gd, T* __restrict__ map,
                                                    const prism_pose* __restrict__ pose,
                                                    const float* __restrict__ depth,
                                                    const float* __restrict__ rgb, MapUpdC mp,
                                                    int64_t* __restrict__ n_updated) {
    __shared__ Pose32 sp;
    __shared__ Pose64 sp64;
    __shared__ int s_cnt;
    if (threadIdx.x == 0) {
        sp64 = load_pose64(pose);
        sp = to32(sp64);
        s_cnt = 0;
    }
    __syncthreads();
    const Pose32 P = sp;
    long long b = blockIdx.x;
    int bx = (int)(b % g.nb), by = (int)((b / g.nb) % g.nb), bz = (int)(b / ((long long)g.nb * g.nb));
    if (brick_culled(g, c, P, bx, by, bz)) return;   // uniform over the block
    int cnt = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int l = threadIdx.x + h * 256;
        int i = (bx << 3) | (l & 7), j = (by << 3) | ((l >> 3) & 7), k = (bz << 3) | (l >> 6);
        float x[3] = {g.o[0] + g.s * ((float)i + 0.5f), g.o[1] + g.s * ((float)j + 0.5f),
                      g.o[2] + g.s * ((float)k + 0.5f)};
        float d[3] = {x[0] - P.t[0], x[1] - P.t[1], x[2] - P.t[2]};
        float X[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) X[a] = (P.R[0][a] * d[0] + P.R[1][a] * d[1]) + P.R[2][a] * d[2];
        if (!(X[2] > 0.0f)) continue;
        float uu = c.fx * (X[0] / X[2]) + c.cx;
        float vv = c.fy * (X[1] / X[2]) + c.cy;
        if (!(uu >= 0.0f && uu < (float)c.W && vv >= 0.0f && vv < (float)c.H)) continue;
        int pix = (int)vv * c.W + (int)uu;
        float D = depth[pix];
        if (!(depth_ok(D) && X[2] <= D + mp.trunc32)) continue;
        // values in double precision: camera depth of the voxel centre,
        // truncated negative SDF, Gaussian product in precision form
        const Pose64& Q = sp64;
        double dd0 = (gd.o[0] + gd.s * ((double)i + 0.5)) - Q.t[0];
        double dd1 = (gd.o[1] + gd.s * ((double)j + 0.5)) - Q.t[1];
        double dd2 = (gd.o[2] + gd.s * ((double)k + 0.5)) - Q.t[2];
        double z = Q.R[0][2] * dd0 + Q.R[1][2] * dd1 + Q.R[2][2] * dd2;
        double f[4];
        f[0] = z - (double)D;
        if (f[0] < -mp.trunc) f[0] = -mp.trunc;
        f[1] = (double)rgb[3 * pix];
        f[2] = (double)rgb[3 * pix + 1];
        f[3] = (double)rgb[3 * pix + 2];
        long long id = (b << 9) | l;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            double mu = (double)ld(map, ch * g.nvox + id);
            double var = (double)ld(map, (4 + ch) * g.nvox + id);
            double lam = 1.0 / var;
            double lam2 = lam + mp.lam_u;
            st(map, ch * g.nvox + id, (float)((lam * mu + mp.lam_u * f[ch]) / lam2));
            st(map, (4 + ch) * g.nvox + id, (float)(1.0 / lam2));
        }
        ++cnt;
    }
    if (n_updated) {
        // wave sum then one LDS atomic per wave, one global atomic per block
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
        if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&s_cnt, cnt);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomicAdd((unsigned long long*)n_updated, (unsigned long long)s_cnt);
    }
}

static unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_map_init(const GridC& g, int dtype, void* map, float occ0, float rgb0, float var0,
                           hipStream_t st) {
    if (dtype == PRISM_BF16)
        k_map_init<uint16_t><<<blocks_for(g.nvox), 256, 0, st>>>(g.nvox, (uint16_t*)map, occ0, rgb0, var0);
    else
        k_map_init<float><<<blocks_for(g.nvox), 256, 0, st>>>(g.nvox, (float*)map, occ0, rgb0, var0);
    return hipGetLastError();
}

hipError_t launch_from_dense(const GridC& g, int dtype, void* map, const float* mean4, const float* var4,
                             hipStream_t st) {
    if (dtype == PRISM_BF16)
        k_from_dense<uint16_t><<<blocks_for(g.nvox), 256, 0, st>>>(g.n, g.nb, (uint16_t*)map, mean4, var4);
    else
        k_from_dense<float><<<blocks_for(g.nvox), 256, 0, st>>>(g.n, g.nb, (float*)map, mean4, var4);
    return hipGetLastError();
}

hipError_t launch_to_dense(const GridC& g, int dtype, const void* map, float* mean4, float* var4,
                           hipStream_t st) {
    if (dtype == PRISM_BF16)
        k_to_dense<uint16_t><<<blocks_for(g.nvox), 256, 0, st>>>(g.n, g.nb, (const uint16_t*)map, mean4, var4);
    else
        k_to_dense<float><<<blocks_for(g.nvox), 256, 0, st>>>(g.n, g.nb, (const float*)map, mean4, var4);
    return hipGetLastError();
}

hipError_t launch_planes(int n, int channels, const float* src, float* dst, int to_dense, hipStream_t st) {
    long long nvox = (long long)n * n * n;
    k_planes<<<blocks_for(nvox), 256, 0, st>>>(n, n / 8, channels, src, dst, to_dense);
    return hipGetLastError();
}

hipError_t launch_map_update(const GridC& g, const CamC& c, const GridD& gd, int dtype, void* map,
                             const prism_pose* pose, const float* depth, const float* rgb, double trunc, double lam_u,
                             int64_t* n_updated, hipStream_t st) {
    if (n_updated) {
        k_zero_i64<<<1, 1, 0, st>>>(n_updated);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    MapUpdC mp{(float)trunc, trunc, lam_u};
    unsigned nbricks = (unsigned)((long long)g.nb * g.nb * g.nb);
    if (dtype == PRISM_BF16)
        k_map_update<uint16_t><<<nbricks, 256, 0, st>>>(g, c, gd, (uint16_t*)map, pose, depth, rgb, mp, n_updated);
    else
        k_map_update<float><<<nbricks, 256, 0, st>>>(g, c, gd, (float*)map, pose, depth, rgb, mp, n_updated);
    return hipGetLastError();
}

}  // namespace prism
