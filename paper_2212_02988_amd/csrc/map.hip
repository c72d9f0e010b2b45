// Voxel-map storage kernels and the closed-form map update (App. D).
//
// Storage: 8 planes (mean occ, R, G, B, var occ, R, G, B) of n^3 values in
// 8x8x8-brick order, brick-major, x fastest inside a brick, followed by the
// brick summary (one value per brick whose sign is exact: <= 0 exactly when
// every occupancy mean of the brick is <= 0, and then not necessarily the
// largest; the largest occupancy mean when that is > 0), a bit per brick
// telling whether the summary is <= 0 (the renderer keeps these bits in LDS
// to skip free space) and per-workgroup update counts.
//
// The map update runs in three kernels and uses no global atomics.
//   cull:   one thread per brick tests the brick's voxel-centre box against
//           the view frustum (conservatively, with margins far above
//           single-precision rounding); each workgroup compacts its survivors
//           into its own 256-entry segment of a brick list (ballot + prefix
//           sums) and stores the segment length.  Block 0 also stores the
//           pose in both precisions for the next kernel.
//   update: a fixed grid of workgroups scans the segment lengths in LDS and
//           walks the compacted list, one brick per wavefront at a time: each
//           lane decides its eight voxels (one column of the brick) with the
//           single-precision recipe and updates only those, so HBM traffic is
//           the updated voxels' 8 planes read and written once; the brick
//           summary is refreshed in the same pass (its free-space bit toggled
//           when its sign changes), reading the occupancy of voxels left alone
//           only in bricks that held a voxel above 0, and each workgroup stores
//           its update count.
//   The count of updated voxels is the sum of the per-workgroup counts, taken
//   by a one-wavefront kernel or by the next kernel of a filter step.
#include "common.hpp"
#include "launch.hpp"

namespace prism {

// value as it reads back after a store of type T
template <typename T>
__device__ __forceinline__ float stored(float v);
template <>
__device__ __forceinline__ float stored<float>(float v) { return v; }
template <>
__device__ __forceinline__ float stored<uint16_t>(float v) { return __uint_as_float(((uint32_t)f2bf(v)) << 16); }

template <typename T>
__global__ __launch_bounds__(256) void k_map_init(long long nvox, T* __restrict__ map, float occ0, float rgb0,
                                                  float var0, MapAux aux, int nbricks) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbricks) aux.bmax[i] = stored<T>(occ0);
    if (i >= nvox) return;
    st(map, i, occ0);
    st(map, nvox + i, rgb0);
    st(map, 2 * nvox + i, rgb0);
    st(map, 3 * nvox + i, rgb0);
#pragma unroll
    for (int c = 4; c < 8; ++c) st(map, c * nvox + i, var0);
}

// brick-pool map: every brick without a slot, bricks summarised by the
// value their voxels read as, pool counters cleared, var0 kept
__global__ __launch_bounds__(256) void k_pool_init(int nbricks, float pocc, float var0, MapAux aux) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) {
        aux.pool[0] = 0;
        aux.pool[1] = 0;
        *aux.var0 = var0;
    }
    if (b >= nbricks) return;
    aux.table[b] = -1;
    aux.bmax[b] = pocc;
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

// brick-pool map -> dense planes; voxels of bricks without a slot take the
// values they read as (and var0)
template <typename T>
__global__ __launch_bounds__(256) void k_pool_to_dense(GridC g, const T* __restrict__ map, MapAux aux,
                                                       float* __restrict__ mean4, float* __restrict__ var4) {
    const long long nvox = (long long)g.n * g.n * g.n;
    long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nvox) return;
    const long long d = dense_of_brick(g.n, g.nb, b);
    const int slot = g.table[b >> 9];
    const long long e = ((long long)slot << 9) | (b & 511);
    const float v0 = *aux.var0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float prior = c == 0 ? g.pocc : g.prgb;
        if (mean4) mean4[c * nvox + d] = slot >= 0 ? ld(map, c * g.nvox + e) : prior;
        if (var4) var4[c * nvox + d] = slot >= 0 ? ld(map, (4 + c) * g.nvox + e) : stored<T>(v0);
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

// maximum over a 256-thread block (lds: 4 floats); every thread gets it
__device__ __forceinline__ float block_max(float m, float* lds) {
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = m;
    __syncthreads();
    float r = lds[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, lds[w]);
    return r;
}

// brick summary of every brick (after writes that bypass the map update)
template <typename T>
__global__ __launch_bounds__(256) void k_brick_max(GridC g, const T* __restrict__ map, MapAux aux) {
    __shared__ float lds[4];
    long long slot = blockIdx.x;
    if (g.table) {
        slot = g.table[blockIdx.x];
        if (slot < 0) {
            if (threadIdx.x == 0) aux.bmax[blockIdx.x] = g.pocc;
            return;
        }
    }
    long long base = slot << 9;
    float m = fmaxf(ld(map, base + threadIdx.x), ld(map, base + threadIdx.x + 256));
    m = block_max(m, lds);
    if (threadIdx.x == 0) aux.bmax[blockIdx.x] = m;
}

// packs the free-space bits (brick maximum <= 0) from the brick summary
__global__ __launch_bounds__(256) void k_pack_bits(int nbricks, MapAux aux) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    int nwords = (nbricks + 31) >> 5;
    if (w >= nwords) return;
    unsigned word = 0;
    if ((w << 5) + 32 <= nbricks) {
        // 32 contiguous floats: eight 16-byte loads issued together
        const float4* p4 = reinterpret_cast<const float4*>(aux.bmax + (w << 5));
        float4 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = p4[i];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            word |= (v[i].x <= 0.0f ? 1u : 0u) << (4 * i);
            word |= (v[i].y <= 0.0f ? 1u : 0u) << (4 * i + 1);
            word |= (v[i].z <= 0.0f ? 1u : 0u) << (4 * i + 2);
            word |= (v[i].w <= 0.0f ? 1u : 0u) << (4 * i + 3);
        }
    } else {
        for (int i = 0; (w << 5) + i < nbricks; ++i)
            if (aux.bmax[(w << 5) + i] <= 0.0f) word |= 1u << i;
    }
    aux.bits[w] = word;
}

// The dilated free-space bits (second bitmap after the plain one): word w
// is the AND of the 32-bit windows of the plain bits that start at bricks
// 32 w + {0, 1} + {0, nb} + {0, nb^2}; words past the bitmap read as 0.  A
// cell that spans bricks lies inside the 2x2x2 block of its base corner's
// brick, so this one bit proves such a cell free (a cell within one brick
// uses the plain bit).  Recomputed after every change of the plain bits.
__device__ __forceinline__ unsigned bits_window(const unsigned* __restrict__ bits, int nwords, int bit) {
    const int w = bit >> 5, sh = bit & 31;
    const unsigned lo = w < nwords ? bits[w] : 0u, hi = w + 1 < nwords ? bits[w + 1] : 0u;
    return sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
}

__device__ __forceinline__ void dilate_block(int blk, int nb, unsigned* __restrict__ bits) {
    const int nwords = free_words(nb);
    const int w = blk * (int)blockDim.x + (int)threadIdx.x;
    if (w >= nwords) return;
    const int b = w << 5, sy = nb, sz = nb * nb;
    unsigned d = bits[w];
    d &= bits_window(bits, nwords, b + 1);
    d &= bits_window(bits, nwords, b + sy);
    d &= bits_window(bits, nwords, b + sy + 1);
    d &= bits_window(bits, nwords, b + sz);
    d &= bits_window(bits, nwords, b + sz + 1);
    d &= bits_window(bits, nwords, b + sz + sy);
    d &= bits_window(bits, nwords, b + sz + sy + 1);
    bits[nwords + w] = d;
}

__global__ __launch_bounds__(256) void k_dilate_bits(int nb, unsigned* __restrict__ bits) {
    dilate_block(blockIdx.x, nb, bits);
}

// the same, with workgroup 0 also totalling the update's per-workgroup
// voxel counts (the whole workgroup, before any thread leaves)
__global__ __launch_bounds__(256) void k_dilate_bits_sum(int nb, unsigned* __restrict__ bits,
                                                         const int* __restrict__ counts, int ngroups,
                                                         int64_t* __restrict__ n_updated) {
    __shared__ long long part[4];
    if (blockIdx.x == 0) sum_counts_block(counts, ngroups, n_updated, part);
    dilate_block(blockIdx.x, nb, bits);
}

// Conservative brick cull: true if no voxel centre of the brick can pass the
// per-voxel test.  Each test is a convex region (behind the camera, or beyond
// one side plane of the frustum) checked on the 8 corners of the brick's
// voxel-centre box.
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

struct PosePair {
    Pose32 f;
    Pose64 d;
};

// workgroup blk of the cull (bricks blk*256 .. blk*256+255)
__device__ __forceinline__ void cull_block(int blk, const GridC& g, const CamC& c, const prism_pose* __restrict__ pose,
                                           const MapAux& aux) {
    __shared__ PosePair sp;
    __shared__ int wcount[4];
    if (threadIdx.x == 0) {
        sp.d = load_pose64(pose);
        sp.f = to32(sp.d);
        if (blk == 0) *reinterpret_cast<PosePair*>(aux.pose) = sp;
    }
    __syncthreads();
    int nbricks = g.nb * g.nb * g.nb;
    int b = blk * blockDim.x + threadIdx.x;
    bool keep = false;
    if (b < nbricks) {
        int bx = b % g.nb, by = (b / g.nb) % g.nb, bz = b / (g.nb * g.nb);
        keep = !brick_culled(g, c, sp.f, bx, by, bz);
    }
    // compaction inside the workgroup: rank = survivors before this thread
    unsigned long long m = __ballot(keep);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wv; ++w) base += wcount[w];
    if (keep) aux.list[blk * 256 + base + rank] = b;
    if (threadIdx.x == 0) aux.segcnt[blk] = wcount[0] + wcount[1] + wcount[2] + wcount[3];
}

__global__ __launch_bounds__(256) void k_cull(GridC g, CamC c, const prism_pose* __restrict__ pose, MapAux aux) {
    cull_block(blockIdx.x, g, c, pose, aux);
}



// plane p of a map as a global-space pointer (uniform, so it lives in
// scalar registers), and element loads / stores through it
template <typename T>
__device__ __forceinline__ gptr<T> plane_g(const T* map, const GridC& g, int p) {
    return as_global(map + (long long)p * g.nvox);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* plane_w(T* map, const GridC& g, int p) {
    return (__attribute__((address_space(1))) T*)(map + (long long)p * g.nvox);
}
// Element i of a plane through a 32-bit byte offset (a plane holds at most
// 2^30 elements of at most 4 bytes): the plane's base stays in scalar
// registers and one vector offset serves all eight planes (an element index
// scaled in 64 bits would take a 64-bit vector address per plane).
__device__ __forceinline__ float ldp(gptr<float> p, unsigned i) { return ldg(p, i * 4u); }
__device__ __forceinline__ float ldp(gptr<uint16_t> p, unsigned i) { return ldg(p, i * 2u); }
__device__ __forceinline__ void stp(__attribute__((address_space(1))) float* p, unsigned i, float v) {
    *(__attribute__((address_space(1))) float*)((__attribute__((address_space(1))) char*)p + i * 4u) = v;
}
__device__ __forceinline__ void stp(__attribute__((address_space(1))) uint16_t* p, unsigned i, float v) {
    *(__attribute__((address_space(1))) uint16_t*)((__attribute__((address_space(1))) char*)p + i * 2u) = f2bf(v);
}

// workgroup blk of ngroups of the update
template <typename T, bool Pool>
__device__ __forceinline__ void map_update_block(int blk, int ngroups, const GridC& g, const CamC& c, const GridD& gd,
                                                 T* __restrict__ map, const float* __restrict__ depth,
                                                 const float* __restrict__ rgb, const MapUpdC& mp, const MapAux& aux,
                                                 int nseg) {
    extern __shared__ int sstart[];    // [nseg + 1] exclusive prefix of the segment lengths
    __shared__ PosePair sp;
    __shared__ int lcnt[4];
    __shared__ int wsum[4];
    // segment lengths -> exclusive prefix sums: each thread sums one
    // contiguous chunk, the chunk sums are scanned across the workgroup
    // (shuffle scan per wavefront, then the four wavefront totals)
    int per = (nseg + 255) / 256;
    int lo = threadIdx.x * per, hi = min(lo + per, nseg);
    int s = 0;
    for (int i = lo; i < hi; ++i) {
        sstart[i] = s;
        s += aux.segcnt[i];
    }
    if (threadIdx.x == 0) sp = *reinterpret_cast<const PosePair*>(aux.pose);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int excl = incl - s;
    for (int w = 0; w < wv; ++w) excl += wsum[w];
    for (int i = lo; i < hi; ++i) sstart[i] += excl;
    if (threadIdx.x == 0) sstart[nseg] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    const Pose32& P = sp.f;
    const Pose64& Q = sp.d;
    const int total = sstart[nseg];
    // one brick per wavefront at a time: lane `lane` owns voxel (lane & 7,
    // lane >> 3) of each of the brick's 8 z-slices, so every load and store
    // of a slice is 64 consecutive elements; no workgroup barrier per brick
    const int nwaves = ngroups * 4;
    int cnt = 0;
    // brick of list entry e: the segment holding e (binary search over the
    // prefix sums), then its list slot
    auto brick_of = [&](int e) {
        int a = 0, z = nseg;
        while (z - a > 1) {
            int mid = (a + z) >> 1;
            if (sstart[mid] <= e) a = mid; else z = mid;
        }
        return aux.list[a * 256 + (e - sstart[a])];
    };
    // the next brick's index is loaded while this one is processed, so the
    // list read is off each brick's chain of memory round trips
    int b_next = blk * 4 + wv < total ? brick_of(blk * 4 + wv) : 0;
    for (int e = blk * 4 + wv; e < total; e += nwaves) {
        const int b = b_next;
        if (e + nwaves < total) b_next = brick_of(e + nwaves);
        // the brick's summary, issued with the depth gathers below
        const float bm_old = aux.bmax[b];
        const int bx = b % g.nb, by = (b / g.nb) % g.nb, bz = b / (g.nb * g.nb);
        const int i = (bx << 3) | (lane & 7), j = (by << 3) | (lane >> 3);
        // decisions for the lane's 8 voxels in single precision
        int pix[8];
        float Dv[8];
        bool upd[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int k = (bz << 3) | h;
            float x[3] = {g.o[0] + g.s * ((float)i + 0.5f), g.o[1] + g.s * ((float)j + 0.5f),
                          g.o[2] + g.s * ((float)k + 0.5f)};
            float d[3] = {x[0] - P.t[0], x[1] - P.t[1], x[2] - P.t[2]};
            float X[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) X[q] = (P.R[0][q] * d[0] + P.R[1][q] * d[1]) + P.R[2][q] * d[2];
            upd[h] = false;
            pix[h] = 0;
            Dv[h] = 0.0f;
            if (X[2] > 0.0f) {
                float uu = c.fx * (X[0] / X[2]) + c.cx;
                float vv = c.fy * (X[1] / X[2]) + c.cy;
                if (uu >= 0.0f && uu < (float)c.W && vv >= 0.0f && vv < (float)c.H) {
                    pix[h] = (int)vv * c.W + (int)uu;
                    upd[h] = true;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 8; ++h)
            if (upd[h]) Dv[h] = ldg(as_global(depth), (unsigned)pix[h] * 4u);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            if (upd[h]) {
                const int k = (bz << 3) | h;
                float x[3] = {g.o[0] + g.s * ((float)i + 0.5f), g.o[1] + g.s * ((float)j + 0.5f),
                              g.o[2] + g.s * ((float)k + 0.5f)};
                float d[3] = {x[0] - P.t[0], x[1] - P.t[1], x[2] - P.t[2]};
                float X2 = (P.R[0][2] * d[0] + P.R[1][2] * d[1]) + P.R[2][2] * d[2];
                upd[h] = depth_ok(Dv[h]) && X2 <= Dv[h] + mp.trunc32;
            }
        }
        // a listed brick none of whose voxels this frame updates (in the
        // frustum but behind the observed surfaces) keeps its values and its
        // summary: nothing more to read or write
        {
            int any = 0;
#pragma unroll
            for (int h = 0; h < 8; ++h) any |= upd[h] ? 1 : 0;
            if (!__any(any)) continue;
        }
        // brick-pool map: the brick's slot, handed out the first time one of
        // its voxels is updated and filled with the values its voxels read as;
        // with the pool full the brick's update is dropped and counted
        long long slot = b;
        bool fresh = false;
        float pvar = 0.0f;
        if constexpr (Pool) {
            int sl = aux.table[b];
            if (sl < 0) {
                int got = -1;
                if (lane == 0) {
                    const int s2 = atomicAdd(&aux.pool[0], 1);
                    if (s2 < aux.capacity) {
                        aux.table[b] = s2;
                        got = s2;
                    } else {
                        // pool full: give the ticket back, count the drop
                        atomicSub(&aux.pool[0], 1);
                        atomicAdd(&aux.pool[1], 1);
                    }
                }
                sl = __shfl(got, 0, 64);
                fresh = sl >= 0;
                pvar = stored<T>(*aux.var0);
            }
            if (sl < 0) continue;
            slot = sl;
        }
        // occupancy of voxels this update leaves alone is read only where it
        // can decide the brick's free-space bit: in a brick holding a voxel
        // above 0 before the update (in a free brick every such voxel is <= 0)
        const bool need_occ = !fresh && !(bm_old <= 0.0f);
        float m = -INFINITY;
        // the lane's eight z-slices in groups of two: a group's plane and
        // colour loads are all issued before any of them is used (one memory
        // round trip per group, not per voxel; groups of four cost more in
        // registers, hence waves, than they save), through global-space
        // plane pointers with 32-bit element offsets (a plane holds at most
        // 2^30 elements)
        const unsigned base = (unsigned)((slot << 9) | lane);
#pragma unroll
        for (int h0 = 0; h0 < 8; h0 += 2) {
            float lv[2][8], lc[2][3];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int h = h0 + hh;
                const unsigned id = base | (unsigned)(h << 6);
                if (upd[h]) {
                    if (!fresh) {
#pragma unroll
                        for (int pl = 0; pl < 8; ++pl) lv[hh][pl] = ldp(plane_g(map, g, pl), id);
                    }
                    const int px = pix[h];
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) lc[hh][ch] = ldg(as_global(rgb), (unsigned)(3 * px + ch) * 4u);
                } else if (need_occ) {
                    lv[hh][0] = ldp(plane_g(map, g, 0), id);
                }
            }
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int h = h0 + hh;
                const int k = (bz << 3) | h;
                const unsigned id = base | (unsigned)(h << 6);
                if (!upd[h]) {
                    if (fresh) {
#pragma unroll
                        for (int ch = 0; ch < 4; ++ch) {
                            stp(plane_w(map, g, ch), id, ch == 0 ? g.pocc : g.prgb);
                            stp(plane_w(map, g, 4 + ch), id, pvar);
                        }
                        m = fmaxf(m, g.pocc);
                    } else if (need_occ) {
                        m = fmaxf(m, lv[hh][0]);
                    }
                    continue;
                }
                // values in double precision: camera depth of the voxel centre,
                // truncated negative SDF, Gaussian product in precision form
                double dd0 = (gd.o[0] + gd.s * ((double)i + 0.5)) - Q.t[0];
                double dd1 = (gd.o[1] + gd.s * ((double)j + 0.5)) - Q.t[1];
                double dd2 = (gd.o[2] + gd.s * ((double)k + 0.5)) - Q.t[2];
                double zc = Q.R[0][2] * dd0 + Q.R[1][2] * dd1 + Q.R[2][2] * dd2;
                double f0 = zc - (double)Dv[h];
                if (f0 < -mp.trunc) f0 = -mp.trunc;
                // App. D: new precision = old + update precision; new mean =
                // inverse of the new precision times the precision-weighted sum.
                // The four channels of a voxel are always updated together with
                // one update precision, so their variances are normally equal bit
                // for bit: the precision algebra is then done once (same inputs,
                // same operations, same results as per channel).  Channels are
                // valued one after another (few double-precision registers live).
                const float vs0 = fresh ? pvar : lv[hh][4];
                const bool same = fresh || (lv[hh][4] == lv[hh][5] && lv[hh][5] == lv[hh][6] && lv[hh][6] == lv[hh][7]);
                double lam = 1.0 / (double)vs0;
                double var2 = 1.0 / (lam + mp.lam_u);
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) {
                    if (ch > 0 && !same) {
                        lam = 1.0 / (double)lv[hh][4 + ch];
                        var2 = 1.0 / (lam + mp.lam_u);
                    }
                    const double mu = fresh ? (double)(ch == 0 ? g.pocc : g.prgb) : (double)lv[hh][ch];
                    const double fc = ch == 0 ? f0 : (double)lc[hh][ch - 1];
                    float nm = (float)(var2 * (lam * mu + mp.lam_u * fc));
                    stp(plane_w(map, g, ch), id, nm);
                    stp(plane_w(map, g, 4 + ch), id, (float)var2);
                    if (ch == 0) m = fmaxf(m, stored<T>(nm));
                }
                ++cnt;
            }
        }
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        if (lane == 0) {
            // The summary keeps an exact sign: in a brick that held a voxel
            // above 0, every voxel was read and m is the largest occupancy;
            // in a free brick the voxels left alone are <= 0, so m > 0 is the
            // largest occupancy and m <= 0 (or no update) leaves the brick
            // free.  The free-space bit toggles when the sign changes (each
            // brick has one owner per launch, so toggles of one word touch
            // different bits).
            const bool was_free = bm_old <= 0.0f;
            const float bm_new = (was_free && !(m > 0.0f)) ? fmaxf(m, bm_old) : m;
            const bool now_free = bm_new <= 0.0f;
            aux.bmax[b] = bm_new;
            if (was_free != now_free) atomicXor(&aux.bits[b >> 5], 1u << (b & 31));
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0) lcnt[wv] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) aux.counts[blk] = lcnt[0] + lcnt[1] + lcnt[2] + lcnt[3];
}

template <typename T, bool Pool>
__global__ __launch_bounds__(256) void k_map_update(GridC g, CamC c, GridD gd, T* __restrict__ map,
                                                    const float* __restrict__ depth,
                                                    const float* __restrict__ rgb, MapUpdC mp, MapAux aux,
                                                    int nseg) {
    map_update_block<T, Pool>(blockIdx.x, gridDim.x, g, c, gd, map, depth, rgb, mp, aux, nseg);
}

// batched: every filter culls / updates its map at its posterior mean with
// its slot's frame
__global__ __launch_bounds__(256) void k_cull_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    cull_block(blockIdx.x - b.start[a], D.g, D.c, &D.S->pose, D.aux);
}

__global__ __launch_bounds__(256) void k_dilate_bits_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    dilate_block(blockIdx.x - b.start[a], D.g.nb, D.aux.bits);
}

template <typename T, bool Pool>
__global__ __launch_bounds__(256) void k_map_update_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    const prism_frame& fr = D.slots[b.slot[a]];
    map_update_block<T, Pool>(blockIdx.x - b.start[a], D.upd_groups, D.g, D.c, D.gd, (T*)D.map, (const float*)fr.depth,
                        (const float*)fr.rgb, D.mp, D.aux, D.nseg);
}

// ---------------------------------------------------------------------------
// descent mapping: one gradient step on the marked bricks
// ---------------------------------------------------------------------------
// Every brick on the run's list (bricks some ray of some gradient pass
// touched; count first) takes the step mean <- mean - lr (grad + (mean -
// mean0) / var) per voxel and channel, with mean0 the brick's means before the
// run's first step (copied into `save` the first time the brick is visited,
// recorded in `saved`) and var the map's variance, which descent leaves
// unchanged.  One workgroup per brick, two voxels per thread, all four
// channels.  grad is cleared behind the step, the brick summary and
// free-space bit follow the new occupancy means, and each workgroup writes its
// share of the previous-belief term 1/2 sum (mean - mean0)^2 / var at the
// means before the step.  Bricks off the list have zero gradient and means
// equal to mean0: the step leaves them as they are.
__global__ __launch_bounds__(256) void k_gd_update(GridC g, float* __restrict__ map, MapAux aux,
                                                   float* __restrict__ save, double* __restrict__ grad,
                                                   const int* __restrict__ list, unsigned* __restrict__ saved,
                                                   double lr_occ, double lr_rgb, double* __restrict__ partials) {
    __shared__ double wsum[4];
    __shared__ float wmax[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int count = list[0];
    double cost = 0.0;
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int b = list[1 + e];
        const bool first = !((saved[b >> 5] >> (b & 31)) & 1u);
        float mu[4][2], mu0[4][2], var[4][2];
        double gr[4][2];
        const long long id0 = ((long long)b << 9) | threadIdx.x;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const long long e2 = (long long)ch * g.nvox + id0 + 256 * h;
                mu[ch][h] = map[e2];
                var[ch][h] = map[(long long)(4 + ch) * g.nvox + id0 + 256 * h];
                gr[ch][h] = grad[e2];
                if (!first) mu0[ch][h] = save[e2];
            }
        float m = -INFINITY;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const double lr = ch ? lr_rgb : lr_occ;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const long long e2 = (long long)ch * g.nvox + id0 + 256 * h;
                if (first) {
                    save[e2] = mu[ch][h];
                    mu0[ch][h] = mu[ch][h];
                }
                const double lam = 1.0 / (double)var[ch][h];
                const double diff = (double)mu[ch][h] - (double)mu0[ch][h];
                cost += 0.5 * lam * diff * diff;
                const float nm = (float)((double)mu[ch][h] - lr * (gr[ch][h] + lam * diff));
                map[e2] = nm;
                grad[e2] = 0.0;
                if (ch == 0) m = fmaxf(m, nm);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        if (lane == 0) wmax[wv] = m;
        __syncthreads();   // every thread has read `saved` and its values
        if (threadIdx.x == 0) {
            const float mb = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
            bool was_free = aux.bmax[b] <= 0.0f, now_free = mb <= 0.0f;
            aux.bmax[b] = mb;
            if (was_free != now_free) atomicXor(&aux.bits[b >> 5], 1u << (b & 31));
            if (first) atomicOr(&saved[b >> 5], 1u << (b & 31));
        }
        __syncthreads();   // wmax is reused by the next brick
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off, 64);
    if (lane == 0) wsum[wv] = cost;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// cost[0] = sum of the data partials + sum of the previous-belief partials
__global__ __launch_bounds__(256) void k_gd_cost(const double* __restrict__ pd, int nd,
                                                 const double* __restrict__ pp, int np, double* __restrict__ cost) {
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < nd; i += 256) a += pd[i];
    for (int i = threadIdx.x; i < np; i += 256) a += pp[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cost[0] = red[0];
}

__global__ __launch_bounds__(256) void k_clear_words(unsigned* __restrict__ w, int n) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) w[i] = 0u;
}

int gd_update_groups(const GridC& g) {
    int nbricks = g.nb * g.nb * g.nb;
    return nbricks < kUpdateGrid ? nbricks : kUpdateGrid;
}

hipError_t launch_gd_clear(unsigned* words, int n, hipStream_t st) {
    k_clear_words<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(words, n);
    return hipGetLastError();
}

hipError_t launch_gd_update(const GridC& g, float* map, const MapAux& aux, float* save, double* grad,
                            const int* list, unsigned* saved, double lr_occ, double lr_rgb, double* partials,
                            hipStream_t st) {
    k_gd_update<<<gd_update_groups(g), 256, 0, st>>>(g, map, aux, save, grad, list, saved, lr_occ, lr_rgb,
                                                     partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_dilate(g, aux, st);
}

hipError_t launch_gd_cost(const double* pd, int nd, const double* pp, int np, double* cost, hipStream_t st) {
    k_gd_cost<<<1, 256, 0, st>>>(pd, nd, pp, np, cost);
    return hipGetLastError();
}

static unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_dilate(const GridC& g, const MapAux& aux, hipStream_t st) {
    k_dilate_bits<<<(unsigned)((free_words(g.nb) + 255) / 256), 256, 0, st>>>(g.nb, aux.bits);
    return hipGetLastError();
}

static hipError_t launch_pack(const GridC& g, const MapAux& aux, hipStream_t st) {
    int nbricks = g.nb * g.nb * g.nb;
    int nwords = (nbricks + 31) >> 5;
    k_pack_bits<<<(unsigned)((nwords + 255) / 256), 256, 0, st>>>(nbricks, aux);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_dilate(g, aux, st);
}


hipError_t launch_map_init(const GridC& g, int dtype, void* map, float occ0, float rgb0, float var0,
                           const MapAux& aux, hipStream_t st) {
    int nbricks = g.nb * g.nb * g.nb;
    if (aux.table) {
        k_pool_init<<<(unsigned)((nbricks + 255) / 256), 256, 0, st>>>(nbricks, g.pocc, var0, aux);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_pack(g, aux, st);
    }
    if (dtype == PRISM_BF16)
        k_map_init<uint16_t><<<blocks_for(g.nvox), 256, 0, st>>>(g.nvox, (uint16_t*)map, occ0, rgb0, var0, aux,
                                                                 nbricks);
    else
        k_map_init<float><<<blocks_for(g.nvox), 256, 0, st>>>(g.nvox, (float*)map, occ0, rgb0, var0, aux, nbricks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pack(g, aux, st);
}

hipError_t launch_brick_max(const GridC& g, int dtype, const void* map, const MapAux& aux, hipStream_t st) {
    unsigned nbricks = (unsigned)(g.nb * g.nb * g.nb);
    if (dtype == PRISM_BF16)
        k_brick_max<uint16_t><<<nbricks, 256, 0, st>>>(g, (const uint16_t*)map, aux);
    else
        k_brick_max<float><<<nbricks, 256, 0, st>>>(g, (const float*)map, aux);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pack(g, aux, st);
}

hipError_t launch_from_dense(const GridC& g, int dtype, void* map, const float* mean4, const float* var4,
                             const MapAux& aux, hipStream_t st) {
    if (dtype == PRISM_BF16)
        k_from_dense<uint16_t><<<blocks_for(g.nvox), 256, 0, st>>>(g.n, g.nb, (uint16_t*)map, mean4, var4);
    else
        k_from_dense<float><<<blocks_for(g.nvox), 256, 0, st>>>(g.n, g.nb, (float*)map, mean4, var4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_brick_max(g, dtype, map, aux, st);
}

hipError_t launch_to_dense(const GridC& g, int dtype, const void* map, float* mean4, float* var4,
                           const MapAux& aux, hipStream_t st) {
    if (g.table) {
        const long long nvox = (long long)g.n * g.n * g.n;
        if (dtype == PRISM_BF16)
            k_pool_to_dense<uint16_t><<<blocks_for(nvox), 256, 0, st>>>(g, (const uint16_t*)map, aux, mean4, var4);
        else
            k_pool_to_dense<float><<<blocks_for(nvox), 256, 0, st>>>(g, (const float*)map, aux, mean4, var4);
        return hipGetLastError();
    }
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

// workgroups of the update kernel, sized to the work: a view frustum holds
// roughly a tenth of a room's bricks, and a workgroup walks four bricks at a
// time, so nb^3 / 32 workgroups give each wavefront about one brick (every
// workgroup first scans the segment lengths, a fixed cost that many idle
// workgroups would multiply); at least 64 (or every brick), at most
// kUpdateGrid
static int update_grid(const GridC& g) {
    int nbricks = g.nb * g.nb * g.nb;
    int ng = nbricks / 32;
    if (ng < 64) ng = nbricks < 64 ? nbricks : 64;
    return ng < kUpdateGrid ? ng : kUpdateGrid;
}

hipError_t launch_map_update(const GridC& g, const CamC& c, const GridD& gd, int dtype, void* map,
                             const prism_pose* pose, const float* depth, const float* rgb, double trunc, double lam_u,
                             const MapAux& aux, int64_t* n_updated, hipStream_t st, hipEvent_t t_begin,
                             hipEvent_t t_end) {
    int nbricks = g.nb * g.nb * g.nb;
    int nseg = (nbricks + 255) / 256;
    k_cull<<<nseg, 256, 0, st>>>(g, c, pose, aux);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    MapUpdC mp{(float)trunc, trunc, lam_u};
    int ng = update_grid(g);
    size_t lds = (size_t)(nseg + 1) * sizeof(int);
    if (t_begin && (e = hipEventRecord(t_begin, st)) != hipSuccess) return e;
    const bool pool = aux.table != nullptr;
    if (dtype == PRISM_BF16 && pool)
        k_map_update<uint16_t, true><<<ng, 256, lds, st>>>(g, c, gd, (uint16_t*)map, depth, rgb, mp, aux, nseg);
    else if (dtype == PRISM_BF16)
        k_map_update<uint16_t, false><<<ng, 256, lds, st>>>(g, c, gd, (uint16_t*)map, depth, rgb, mp, aux, nseg);
    else if (pool)
        k_map_update<float, true><<<ng, 256, lds, st>>>(g, c, gd, (float*)map, depth, rgb, mp, aux, nseg);
    else
        k_map_update<float, false><<<ng, 256, lds, st>>>(g, c, gd, (float*)map, depth, rgb, mp, aux, nseg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!n_updated) {
        if ((e = launch_dilate(g, aux, st)) != hipSuccess) return e;
        return t_end ? hipEventRecord(t_end, st) : hipSuccess;
    }
    k_dilate_bits_sum<<<(unsigned)((free_words(g.nb) + 255) / 256), 256, 0, st>>>(g.nb, aux.bits, aux.counts, ng,
                                                                                 n_updated);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return t_end ? hipEventRecord(t_end, st) : hipSuccess;
}

int map_update_groups(const GridC& g) { return update_grid(g); }

// A batched update launches the workgroups of every filter of the batch
// together, which fills the GPU with fewer per map: half of a lone map's
// grid (each wavefront walks about two bricks; on the 16-stream mix 198
// against 203 us per launch, while a lone 256^3 map's update takes 43
// against 40 us with half its grid)
int map_update_groups_batch(const GridC& g) {
    const int nbricks = g.nb * g.nb * g.nb;
    const int ng = update_grid(g) / 2;
    return ng >= 64 ? ng : (nbricks < 64 ? nbricks : 64);
}

hipError_t launch_cull_batch(const BatchArgs& b, hipStream_t st) {
    k_cull_batch<<<b.start[b.n], 256, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_dilate_batch(const BatchArgs& b, hipStream_t st) {
    k_dilate_bits_batch<<<b.start[b.n], 256, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_map_update_batch(const BatchArgs& b, int dtype, bool pool, int max_nseg, hipStream_t st) {
    size_t lds = (size_t)(max_nseg + 1) * sizeof(int);
    if (dtype == PRISM_BF16 && pool)
        k_map_update_batch<uint16_t, true><<<b.start[b.n], 256, lds, st>>>(b);
    else if (dtype == PRISM_BF16)
        k_map_update_batch<uint16_t, false><<<b.start[b.n], 256, lds, st>>>(b);
    else if (pool)
        k_map_update_batch<float, true><<<b.start[b.n], 256, lds, st>>>(b);
    else
        k_map_update_batch<float, false><<<b.start[b.n], 256, lds, st>>>(b);
    return hipGetLastError();
}

}  // namespace prism
