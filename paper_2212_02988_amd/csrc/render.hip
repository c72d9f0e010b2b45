// Ray-marching emission (App. B), its pose Jacobian with the fused normal-
// equation reduction, anchor normals, and the adjoint w.r.t. map means.
//
// Work split of render and render_jacobian: four lanes per ray (a quad), an
// 8x2 pixel strip per wave, an 8x8 tile per workgroup, blockIdx.y = frame.
// A single frame is only ~10^5 rays, so the march is latency-bound: the four
// lanes of a ray evaluate interleaved samples (lane s takes k0 + s + 4 j,
// j < kPerLane) and two DPP quad permutations find the first crossing of the
// trip, which shortens each ray's chain of dependent gathers four-fold and
// gives the GPU four times more waves to overlap.  Samples in bricks whose
// occupancy is <= 0 everywhere are decided without touching the map
// (free-space bits in LDS; every cell reads the dilated bit of its base
// corner's 2x2x2 block of bricks).  At the hit the quad splits the
// double-precision shading and the Jacobian by channel: lane 0 occupancy /
// depth, lanes 1-3 one colour each.
//
// The adjoint takes four lanes per ray as well (8x8 pixels per workgroup):
// from the given hit index it recomputes the two samples, nothing to march,
// and lane s scatters the gradient of plane s.
#include "common.hpp"
#include "launch.hpp"

namespace prism {

constexpr int kLanes = 4;       // lanes per ray in render / render_jacobian
constexpr int kPerLane = 4;     // samples per lane per trip

template <typename T, bool Pool>
__device__ __forceinline__ float occ_at(const GridC& g, const T* occ, const Cell& c) {
    float v[8];
    corners<T, Pool>(g, occ, c, g.occ_out, g.pocc, v);
    return trilerp(v, c.w);
}

// Occupancy of a cell that straddles the grid's boundary (on every axis one
// of its two corner planes is inside; dense maps): corners outside take the
// outside value.  A brick-order element index is a sum of one term per
// axis, ((x >> 3) * brick stride + (x & 7) * voxel stride), so the two
// candidates per axis are formed once, from coordinates clamped into the
// grid (a clamped corner is loaded and then replaced), and each corner is
// three adds away: a few dozen instructions instead of eight corners each
// tested and indexed on its own.
template <typename T>
__device__ __forceinline__ float occ_partial(const GridC& g, const T* occ, const Cell& c) {
    const unsigned bs[3] = {512u, 512u * (unsigned)g.nb, 512u * (unsigned)(g.nb * g.nb)};
    const unsigned vs[3] = {1u, 8u, 64u};
    unsigned off[3][2];
    bool ok[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int x = c.i[a] + d;    // in [-1, n] for a straddling cell
            ok[a][d] = (unsigned)x < (unsigned)g.n;
            const unsigned xc = (unsigned)min(max(x, 0), g.n - 1);
            off[a][d] = (__umul24(xc >> 3, bs[a]) + (xc & 7u) * vs[a]) * (unsigned)sizeof(T);
        }
    float v[8];
    const gptr<T> pl = as_global(occ);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const float x = ldg(pl, off[0][dx] + off[1][dy] + off[2][dz]);
        v[q] = (ok[0][dx] && ok[1][dy] && ok[2][dz]) ? x : g.occ_out;
    }
    return trilerp(v, c.w);
}

// True if the free-space bits prove that the sample's occupancy is <= 0:
// every corner of its cell lies inside the grid and in bricks whose largest
// occupancy mean is <= 0.  Each lerp of values <= 0 with a weight in [0, 1]
// is <= 0 under round-to-nearest (rounding is monotonic and 0 is
// representable), so the single-precision recipe would have produced a value
// <= 0 as well and the sample cannot be the hit when tau == 0.
__device__ __forceinline__ bool bit_of(lds_u32* bits, int b) { return (bits[b >> 5] >> (b & 31)) & 1u; }

// The workgroup's LDS copy of the free-space bits: w the plain bits, then,
// when dil > 0, the dilated bits at word offset dil (w NULL: no skipping)
struct FreeBits {
    lds_u32* w;
    int dil;
};

// A cell within one brick takes the brick's bit.  A cell that spans bricks
// lies in the 2x2x2 block of bricks of its base corner: one dilated bit
// covers it (the same LDS read for every lane); without the dilated bits
// each spanned brick is tested.
__device__ __forceinline__ bool cell_free(const GridC& g, const FreeBits& fb, const CellAddr& a) {
    if (fb.dil) return bit_of(fb.w + (a.cross ? fb.dil : 0), a.b0);
    if (!a.cross) return bit_of(fb.w, a.b0);
    const int sx = a.dx != 1 ? 1 : 0, sy = a.dy != 8 ? g.nb : 0, sz = a.dz != 64 ? g.nb * g.nb : 0;
    bool all = true;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        all &= bit_of(fb.w, a.b0 + ((q & 1) ? sx : 0) + ((q & 2) ? sy : 0) + ((q & 4) ? sz : 0));
    return all;
}

// Occupancy of marched sample fk (an integer held in a float), or -1 when the
// free-space bits prove it is <= 0 (fb: the workgroup's LDS copy, present
// only when tau == 0).  Most marched samples are decided by the bits alone,
// so that path takes only the cell's base corner and its brick: with the
// dilated bits every cell inside the grid reads the one bit of the 2x2x2
// bricks from its base brick, whether or not the cell spans bricks (a
// spanned brick is in that block; a cell within one brick loses little from
// the coarser test).  The corner addressing and the weights are formed only
// for samples that read the map.
enum BitsMode { kNoBits = 0, kPlainBits = 1, kDilatedBits = 2 };

// grid coordinate of a marched sample and its cell's base corner
struct SamplePos {
    float gc[3];
    int i[3];
};

__device__ __forceinline__ SamplePos sample_pos(const RayCoef& rc, float fk) {
    SamplePos p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.gc[a] = sample_gc(rc, fk, a);
        p.i[a] = floor_i32(p.gc[a]);
    }
    return p;
}

template <typename T, bool Pool, int Bits, bool DilTested = false>
__device__ __forceinline__ float march_sample(const GridC& g, const T* occ, const FreeBits& fb, const SamplePos& p) {
    const float* gc = p.gc;
    const int* i = p.i;
    const unsigned lim = (unsigned)(g.n - 1);
    if (max(max((unsigned)i[0], (unsigned)i[1]), (unsigned)i[2]) < lim) {
        // all 8 corners inside: indices >= 0 and < 2^10, so 24-bit products
        const unsigned bx = (unsigned)i[0] >> 3, by = (unsigned)i[1] >> 3, bz = (unsigned)i[2] >> 3;
        const int b0 = (int)(__umul24(bz, (unsigned)(g.nb * g.nb)) + __umul24(by, (unsigned)g.nb) + bx);
        if constexpr (Bits == kDilatedBits && !DilTested) {
            // bit b0 of the dilated bits (the bit-field extract takes the low 5 bits of b0)
            if (__builtin_amdgcn_ubfe(fb.w[fb.dil + (b0 >> 5)], (unsigned)b0, 1u)) return -1.0f;
        }
        const int lx = i[0] & 7, ly = i[1] & 7, lz = i[2] & 7;
        CellAddr a;
        a.b0 = b0;
        a.base = (b0 << 9) | (lz << 6) | (ly << 3) | lx;
        a.dx = lx == 7 ? 512 - 7 : 1;
        a.dy = ly == 7 ? 512 * g.nb - 56 : 8;
        a.dz = lz == 7 ? 512 * g.nb * g.nb - 448 : 64;
        a.cross = (lx == 7) | (ly == 7) | (lz == 7);
        // plain bits only (the dilated ones did not fit in LDS): per spanned brick
        if constexpr (Bits == kPlainBits)
            if (cell_free(g, fb, a)) return -1.0f;
        // inside the grid g >= 0, where g - floor(g) is exact and fract(g) equals it
        float w[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) w[q] = __builtin_amdgcn_fractf(gc[q]);
        if constexpr (Pool) {
            // brick-pool map: a single-brick cell through its slot (a brick
            // without one reads as the prior everywhere, and the trilinear
            // blend of equal values is that value); others corner by corner
            if (!a.cross) {
                const int slot = g.table[b0];
                if (slot < 0) return g.pocc;
                a.base = (slot << 9) | (a.base & 511);
            } else {
                Cell cl;
#pragma unroll
                for (int q = 0; q < 3; ++q) { cl.i[q] = i[q]; cl.w[q] = w[q]; }
                return occ_at<T, Pool>(g, occ, cl);
            }
        }
        float v[8];
        corners_in_g(as_global(occ), a, v);
        return trilerp(v, w);
    }
    // Every corner outside the grid (on some axis both i and i + 1 are): the
    // blend of 8 equal outside values is that value, lerp(a, a, w) = a.
    if (max(max((unsigned)i[0] + 1u, (unsigned)i[1] + 1u), (unsigned)i[2] + 1u) > (unsigned)g.n) return g.occ_out;
    Cell cl;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        cl.i[q] = i[q];
        cl.w[q] = gc[q] - (float)i[q];
    }
    if constexpr (!Pool) return occ_partial(g, occ, cl);
    return occ_at<T, Pool>(g, occ, cl);
}

// double-precision sample point k of the ray with direction dir (world)
__device__ __forceinline__ void grid_coord64(const GridD& gd, const CamD& cd, const Pose64& P, const double dir[3],
                                             int k, double gc[3]) {
    double dk = cd.dn + (double)k * cd.step;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double p = P.t[a] + dk * dir[a];
        gc[a] = (p - gd.o[a]) * gd.inv_s - 0.5;
    }
}

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

struct BlockPose {
    Pose64 d;
    Pose32 f;
};

// The prologue of a marching workgroup, one barrier: thread 0's pose loads
// are issued first and are in flight while every thread copies the
// free-space bits to LDS — both bitmaps when they fit, else the plain bits,
// else none (no skipping): free_lds_words words, which the launch allocates.
__device__ __forceinline__ FreeBits block_setup(const GridC& g, const unsigned* __restrict__ gbits, unsigned* lbits,
                                                const prism_pose* pose, BlockPose* sp) {
    prism_pose raw;
    if (threadIdx.x == 0) raw = *pose;
    FreeBits fb{nullptr, 0};
    const int nwords = free_words(g.nb), nl = gbits ? free_lds_words(nwords) : 0;
    if ((reinterpret_cast<uintptr_t>(gbits) & 15) == 0) {
        // 16-byte copies (the workgroup's LDS copy is 16-byte aligned), then the tail
        const int n4 = nl >> 2;
        const uint4* g4 = reinterpret_cast<const uint4*>(gbits);
        uint4* l4 = reinterpret_cast<uint4*>(lbits);
        for (int i = threadIdx.x; i < n4; i += blockDim.x) l4[i] = g4[i];
        for (int i = (n4 << 2) + threadIdx.x; i < nl; i += blockDim.x) lbits[i] = gbits[i];
    } else {
        for (int i = threadIdx.x; i < nl; i += blockDim.x) lbits[i] = gbits[i];
    }
    if (threadIdx.x == 0) {
        quat_to_rot64(raw, sp->d.R);
        for (int i = 0; i < 3; ++i) sp->d.t[i] = raw.t[i];
        sp->f = to32(sp->d);
    }
    __syncthreads();
    if (nl) {
        fb.w = (lds_u32*)lbits;
        fb.dil = nl > nwords ? nwords : 0;
    }
    return fb;
}

__device__ __forceinline__ const BlockPose& block_pose(const prism_pose* pose, BlockPose* sp) {
    if (threadIdx.x == 0) {
        sp->d = load_pose64(pose);
        sp->f = to32(sp->d);
    }
    __syncthreads();
    return *sp;
}

// ---------------------------------------------------------------------------
// quad (four lanes per ray) march and shading
// ---------------------------------------------------------------------------
// minimum over the four lanes of a quad (DPP quad permutations: lanes 1,0,3,2
// then 2,3,0,1; a lane whose partner is inactive keeps its own value)
__device__ __forceinline__ int quad_min(int x) {
    x = min(x, __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));
    x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));
    return x;
}

// lane 0 of each quad to all four lanes (DPP quad_perm 0,0,0,0; whole quads
// are active together)
__device__ __forceinline__ float quad_bcast0f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x00, 0xF, 0xF, false));
}

// sum over the quad (DPP quad permutations 1,0,3,2 then 2,3,0,1; every lane
// ends with (x0 + x1) + (x2 + x3) up to the order of each addition)
__device__ __forceinline__ double quad_xchg(double x, int ctrl_is_2301) {
    const long long b = __double_as_longlong(x);
    int lo, hi;
    if (ctrl_is_2301) {
        lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x4E, 0xF, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x4E, 0xF, 0xF, false);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double quad_sum(double x) {
    x += quad_xchg(x, 0);
    x += quad_xchg(x, 1);
    return x;
}

__device__ __forceinline__ double quad_bcast0(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x00, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x00, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// first sample index whose occupancy exceeds tau (strictly), or -1; every
// lane of the quad returns the same value
template <typename T, bool Pool, int Bits>
__device__ __forceinline__ int march_quad_b(const GridC& g, const CamC& c, const RayCoef& rc, const T* occ,
                                            const FreeBits& fb, int s) {
    constexpr int G = kLanes * kPerLane;
    // the sample index as a float, advanced exactly (K < 2^24); the last trip's
    // samples past K - 1 are evaluated like any other and ignored
    float fk0 = (float)s;
    // The sample recipe is monotone in k on every axis, so once a sample's
    // cell lies past the grid on an axis the ray moves away from it along,
    // so do all later cells: their occupancy is the outside value.  When that
    // value cannot cross tau the ray has no first crossing left.  The test
    // per axis: cell index < lo (ray not moving up) or >= hi (not moving down).
    const bool stop_outside = !(g.occ_out > c.tau);
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = rc.B[a] <= 0.0f ? -1 : INT_MIN;
        hi[a] = rc.B[a] >= 0.0f ? g.n : INT_MAX;
    }
    for (int k0 = 0; k0 < c.K; k0 += G, fk0 += (float)G) {
        float f[kPerLane];
        bool gone = false;
        if constexpr (Bits == kDilatedBits) {
            // the round's free-space tests first, as straight-line code, so its
            // LDS reads are in flight together (a sample outside the grid reads
            // word 0 and ignores it); then the samples the bits do not decide,
            // whose position is formed again (a few instructions, fewer live
            // registers than keeping it)
            const unsigned lim = (unsigned)(g.n - 1);
            unsigned word[kPerLane];
            int b0[kPerLane];
            bool in[kPerLane];
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) {
                const SamplePos p = sample_pos(rc, fk0 + (float)(j * kLanes));
                const int* i = p.i;
                in[j] = max(max((unsigned)i[0], (unsigned)i[1]), (unsigned)i[2]) < lim;
                const int b = (int)(__umul24((unsigned)i[2] >> 3, (unsigned)(g.nb * g.nb)) +
                                    __umul24((unsigned)i[1] >> 3, (unsigned)g.nb) + ((unsigned)i[0] >> 3));
                b0[j] = in[j] ? b : 0;
                word[j] = fb.w[fb.dil + (b0[j] >> 5)];
                if (j == kPerLane - 1) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) gone |= (i[a] < lo[a]) | (i[a] >= hi[a]);
                }
            }
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) {
                const bool fr = in[j] && __builtin_amdgcn_ubfe(word[j], (unsigned)b0[j], 1u);
                f[j] = fr ? -1.0f
                          : march_sample<T, Pool, Bits, true>(g, occ, fb, sample_pos(rc, fk0 + (float)(j * kLanes)));
            }
        } else {
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) {
                const SamplePos p = sample_pos(rc, fk0 + (float)(j * kLanes));
                f[j] = march_sample<T, Pool, Bits>(g, occ, fb, p);
                if (j == kPerLane - 1) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) gone |= (p.i[a] < lo[a]) | (p.i[a] >= hi[a]);
                }
            }
        }
        int first = 0x7fffffff;
#pragma unroll
        for (int j = kPerLane - 1; j >= 0; --j) {
            int k = k0 + j * kLanes + s;
            if (k < c.K && f[j] > c.tau) first = k;
        }
        first = quad_min(first);
        if (first != 0x7fffffff) return first;
        // lane 3 holds the trip's last sample (DPP quad_perm 3,3,3,3)
        if (stop_outside && __builtin_amdgcn_update_dpp(0, (int)gone, 0xFF, 0xF, 0xF, false)) return -1;
    }
    return -1;
}

// the march with the workgroup's free-space bits mode fixed (one uniform
// branch per ray instead of one per sample)
template <typename T, bool Pool>
__device__ __forceinline__ int march_quad(const GridC& g, const CamC& c, const RayCoef& rc, const T* occ,
                                          const FreeBits& fb, int s) {
    if (fb.w && fb.dil) return march_quad_b<T, Pool, kDilatedBits>(g, c, rc, occ, fb, s);
    if (fb.w) return march_quad_b<T, Pool, kPlainBits>(g, c, rc, occ, fb, s);
    return march_quad_b<T, Pool, kNoBits>(g, c, rc, occ, fb, s);
}

// This lane's share of the shading at a valid hit: plane s (0 occupancy,
// 1..3 colour) at samples k*-1 and k*, in double precision, plus the
// double-precision interpolation weights.
struct QuadShade {
    double v0, v1;          // plane s at samples k*-1, k*
    double f0, f1;          // occupancy at k*-1, k* (from lane 0)
    double alpha, value;    // alpha and this lane's output (depth or colour)
    float w0[3], w1[3];
    float d0, d1;
    float cv0[8], cv1[8];   // plane s at the corners of the two cells (as corners() gives them)
};

// Trilinear value of one plane in double precision at a marched sample:
// cell from the decision recipe, weights from the double-precision grid
// coordinate, blended along x, then y, then z (seven linear blends, each one
// fused multiply-add; the same trilinear interpolant as the sum of the
// corners weighted by products of 1-D hat weights, to rounding).  The
// corners are the ones corners() gathered; a corner outside the grid takes
// the double-precision outside value.
__device__ __forceinline__ double lerp64(double a, double b, double w) { return __builtin_fma(w, b - a, a); }

__device__ __forceinline__ double tri64c(const GridC& g, const float v[8], const double gc[3], const int cell[3],
                                         double outv) {
    const double w0 = gc[0] - (double)cell[0], w1 = gc[1] - (double)cell[1], w2 = gc[2] - (double)cell[2];
    // a cell inside the grid (the usual case) needs no test per corner
    const unsigned lim = (unsigned)(g.n - 1);
    const bool inside = (unsigned)cell[0] < lim && (unsigned)cell[1] < lim && (unsigned)cell[2] < lim;
    double V[8];
    if (inside) {
#pragma unroll
        for (int q = 0; q < 8; ++q) V[q] = (double)v[q];
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int i = cell[0] + (q & 1), j = cell[1] + ((q >> 1) & 1), k = cell[2] + (q >> 2);
            bool in = (unsigned)i < (unsigned)g.n && (unsigned)j < (unsigned)g.n && (unsigned)k < (unsigned)g.n;
            V[q] = in ? (double)v[q] : outv;
        }
    }
    const double l00 = lerp64(V[0], V[1], w0), l10 = lerp64(V[2], V[3], w0);
    const double l01 = lerp64(V[4], V[5], w0), l11 = lerp64(V[6], V[7], w0);
    return lerp64(lerp64(l00, l10, w1), lerp64(l01, l11, w1), w2);
}

template <typename T, bool Pool>
__device__ __forceinline__ QuadShade shade_quad(const GridC& g, const GridD& gd, const CamD& cd, const Pose64& P,
                                                int u, int v, const T* map, const Cell& c0, const Cell& c1, int k,
                                                int s) {
    // values only from here (the hit index and cells are decided): the
    // double-precision arithmetic may fuse multiplies and adds
#pragma clang fp contract(fast)
    QuadShade q;
    double rc[3], dir[3], gc0[3], gc1[3];
    pixel_dir64(cd, u, v, rc);
#pragma unroll
    for (int a = 0; a < 3; ++a) dir[a] = P.R[a][0] * rc[0] + P.R[a][1] * rc[1] + P.R[a][2] * rc[2];
    grid_coord64(gd, cd, P, dir, k - 1, gc0);
    grid_coord64(gd, cd, P, dir, k, gc1);
    double d0 = cd.dn + (double)(k - 1) * cd.step;
    double d1 = cd.dn + (double)k * cd.step;
    const T* pl = map + (long long)s * g.nvox;
    double outv = s == 0 ? gd.occ_out : gd.rgb_out;
    float outv32 = s == 0 ? g.occ_out : g.rgb_out, priorv = s == 0 ? g.pocc : g.prgb;
    // the lane's plane at both cells, gathered once (the Jacobian row reuses them)
    corners<T, Pool>(g, pl, c0, outv32, priorv, q.cv0);
    corners<T, Pool>(g, pl, c1, outv32, priorv, q.cv1);
    q.v0 = tri64c(g, q.cv0, gc0, c0.i, outv);
    q.v1 = tri64c(g, q.cv1, gc1, c1.i, outv);
    q.f0 = quad_bcast0(q.v0);
    q.f1 = quad_bcast0(q.v1);
    q.alpha = (cd.tau - q.f0) / (q.f1 - q.f0);
    q.value = s == 0 ? q.alpha * d1 + (1.0 - q.alpha) * d0 : q.alpha * q.v1 + (1.0 - q.alpha) * q.v0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.w0[a] = (float)(gc0[a] - (double)c0.i[a]);
        q.w1[a] = (float)(gc1[a] - (double)c1.i[a]);
    }
    q.d0 = (float)d0;
    q.d1 = (float)d1;
    return q;
}

// This lane's row of the 4x6 Jacobian d(depth, r, g, b)/d(delta), k* fixed.
// Lane 0 forms d(alpha)/d(delta) from the occupancy gradients and shares it.
__device__ __forceinline__ void jac_row_quad(const GridC& g, const QuadShade& q, const float dir[3], int s,
                                             float row[6]) {
    float a0[3], a1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) { a0[i] = q.d0 * dir[i]; a1[i] = q.d1 * dir[i]; }
    float G0[3], G1[3], cr[3], r0[6], r1[6];
    trigrad(q.cv0, q.w0, G0);
    trigrad(q.cv1, q.w1, G1);
#pragma unroll
    for (int i = 0; i < 3; ++i) { G0[i] *= g.inv_s; G1[i] *= g.inv_s; r0[i] = G0[i]; r1[i] = G1[i]; }
    cross3(a0, G0, cr);
#pragma unroll
    for (int i = 0; i < 3; ++i) r0[3 + i] = cr[i];
    cross3(a1, G1, cr);
#pragma unroll
    for (int i = 0; i < 3; ++i) r1[3 + i] = cr[i];
    // lane 0: d(alpha) = -[(1-alpha) df0 + alpha df1] / (f1 - f0)
    float al = (float)q.alpha;
    float inv_den = (float)(1.0 / (q.f1 - q.f0));
    float dal[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) dal[m] = quad_bcast0f(-((1.0f - al) * r0[m] + al * r1[m]) * inv_den);
    if (s == 0) {
#pragma unroll
        for (int m = 0; m < 6; ++m) row[m] = (q.d1 - q.d0) * dal[m];
    } else {
        float dc = (float)(q.v1 - q.v0);
#pragma unroll
        for (int m = 0; m < 6; ++m) row[m] = dc * dal[m] + al * r1[m] + (1.0f - al) * r0[m];
    }
}

// quad tile mapping: 8x8 pixels per 256-thread workgroup, 8x2 per wave
__device__ __forceinline__ void quad_pixel(const CamC& c, int blk, int& u, int& v, int& s) {
    int tiles_x = (c.W + 7) >> 3;
    int bx = blk % tiles_x, by = blk / tiles_x;
    int t = threadIdx.x;
    s = t & 3;
    int r = t >> 2;    // 0..63 ray of the tile
    u = (bx << 3) + (r & 7);
    v = (by << 3) + (r >> 3);
}

// ---------------------------------------------------------------------------
// render
// ---------------------------------------------------------------------------
// workgroup blk (8x8 pixel tile) of frame `frame`, rendered at *pose
template <typename T, bool Pool>
__device__ __forceinline__ void render_block(int blk, int frame, const GridC& g, const CamC& c, const GridD& gd,
                                             const CamD& cd, const T* __restrict__ map,
                                             const unsigned* __restrict__ gbits, const prism_pose* __restrict__ pose,
                                             float* __restrict__ depth, float* __restrict__ rgb,
                                             uint8_t* __restrict__ mask, int32_t* __restrict__ hit_k) {
    __shared__ BlockPose sp;
    extern __shared__ __align__(16) unsigned lbits[];
    const FreeBits fb = block_setup(g, gbits, lbits, pose, &sp);
    const BlockPose& P = sp;
    int u, v, s;
    quad_pixel(c, blk, u, v, s);
    if (u >= c.W || v >= c.H) return;   // whole quads leave together
    float dir[3];
    ray_dir32(c, P.f, u, v, dir);
    const RayCoef rc = ray_coef(g, c, P.f, dir);
    int k = march_quad<T, Pool>(g, c, rc, map, fb, s);
    long long pix = (long long)frame * c.W * c.H + (long long)v * c.W + u;
    if (s == 0) {
        if (hit_k) hit_k[pix] = k;
        mask[pix] = k >= 1 ? 1 : 0;
    }
    if (k >= 1) {
        Cell c0 = sample_cell(rc, k - 1), c1 = sample_cell(rc, k);
        QuadShade q = shade_quad<T, Pool>(g, gd, cd, P.d, u, v, map, c0, c1, k, s);
        if (s == 0)
            depth[pix] = (float)q.value;
        else
            rgb[3 * pix + s - 1] = (float)q.value;
    } else {
        if (s == 0)
            depth[pix] = 0.0f;
        else
            rgb[3 * pix + s - 1] = 0.0f;
    }
}

template <typename T, bool Pool>
// at least 6 waves per SIMD (80 VGPRs, no spills): the march hides gather
// latency with waves; 7 or 8 would spill the double-precision shading
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_render(GridC g, CamC c, GridD gd, CamD cd, const T* __restrict__ map,
                                                const unsigned* __restrict__ gbits,
                                                const prism_pose* __restrict__ poses,
                                                float* __restrict__ depth, float* __restrict__ rgb,
                                                uint8_t* __restrict__ mask, int32_t* __restrict__ hit_k) {
    render_block<T, Pool>(blockIdx.x, blockIdx.y, g, c, gd, cd, map, gbits, poses + blockIdx.y, depth, rgb, mask, hit_k);
}

// batched: every filter renders its next anchor from its updated map at its
// posterior mean
template <typename T, bool Pool>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_render_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    render_block<T, Pool>(blockIdx.x - b.start[a], 0, D.g, D.c, D.gd, D.cd, (const T*)D.map, D.bits, &D.S->pose, D.a_depth,
                    D.a_rgb, D.a_mask, nullptr);
}

// ---------------------------------------------------------------------------
// normals of a rendered depth image
// ---------------------------------------------------------------------------
__device__ __forceinline__ void normals_block(int blk, const CamC& c, int n_frames, const float* __restrict__ depth,
                                              const uint8_t* __restrict__ mask, float disc,
                                              float* __restrict__ normals, uint8_t* __restrict__ nmask,
                                              const int* __restrict__ counts, int ngroups,
                                              int64_t* __restrict__ n_updated,
                                              int64_t* __restrict__ n_updated_total) {
    // in a filter step, the first workgroup also totals the preceding map
    // update (before any thread returns: the sum synchronises the workgroup)
    __shared__ long long part[4];
    if (n_updated && blk == 0) sum_counts_block(counts, ngroups, n_updated, part, n_updated_total);
    long long npix = (long long)c.W * c.H;
    long long gid = (long long)blk * blockDim.x + threadIdx.x;
    if (gid >= npix * n_frames) return;
    long long f = gid / npix;
    int p = (int)(gid - f * npix);
    int u = p % c.W, v = p / c.W;
    const float* D = depth + f * npix;
    const uint8_t* M = mask + f * npix;
    // the five masks and depths in one round of loads (a border pixel reads
    // itself in place of its missing neighbours; it is never valid), then
    // one store of the result
    const bool inner = u > 0 && v > 0 && u < c.W - 1 && v < c.H - 1;
    const int pl = inner ? p - 1 : p, pr = inner ? p + 1 : p;
    const int pu = inner ? p - c.W : p, pd = inner ? p + c.W : p;
    const bool m = (M[p] & M[pl] & M[pr] & M[pu] & M[pd]) != 0;   // masks are 0 / 1
    const float d = D[p], dl = D[pl], dr = D[pr], du = D[pu], dd = D[pd];
    float o[3] = {0.0f, 0.0f, 0.0f};
    uint8_t ok = 0;
    if (inner && m &&
        !(fabsf(dl - d) > disc || fabsf(dr - d) > disc || fabsf(du - d) > disc || fabsf(dd - d) > disc)) {
        float xl = ((float)(u - 1) + 0.5f - c.cx) * c.ifx, xr = ((float)(u + 1) + 0.5f - c.cx) * c.ifx;
        float x0 = ((float)u + 0.5f - c.cx) * c.ifx;
        float yu = ((float)(v - 1) + 0.5f - c.cy) * c.ify, yd = ((float)(v + 1) + 0.5f - c.cy) * c.ify;
        float y0 = ((float)v + 0.5f - c.cy) * c.ify;
        float a[3] = {dr * xr - dl * xl, dr * y0 - dl * y0, dr - dl};
        float b[3] = {dd * x0 - du * x0, dd * yd - du * yu, dd - du};
        float n[3];
        cross3(a, b, n);
        float len = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (len > 0.0f) {
            float sgn = (n[0] * x0 + n[1] * y0 + n[2]) * d < 0.0f ? 1.0f : -1.0f;
            float il = sgn / len;
            o[0] = n[0] * il;
            o[1] = n[1] * il;
            o[2] = n[2] * il;
            ok = 1;
        }
    }
    float* N = normals + 3 * gid;
    N[0] = o[0];
    N[1] = o[1];
    N[2] = o[2];
    nmask[gid] = ok;
}

__global__ __launch_bounds__(256) void k_normals(CamC c, int n_frames, const float* __restrict__ depth,
                                                 const uint8_t* __restrict__ mask, float disc,
                                                 float* __restrict__ normals, uint8_t* __restrict__ nmask,
                                                 const int* __restrict__ counts, int ngroups,
                                                 int64_t* __restrict__ n_updated,
                                                 int64_t* __restrict__ n_updated_total) {
    normals_block(blockIdx.x, c, n_frames, depth, mask, disc, normals, nmask, counts, ngroups, n_updated,
                  n_updated_total);
}

__global__ __launch_bounds__(256) void k_normals_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    normals_block(blockIdx.x - b.start[a], D.c, 1, D.a_depth, D.a_mask, D.normal_disc, D.a_normals, D.a_nmask,
                  D.aux.counts, D.upd_groups, &D.S->n_updated, &D.S->n_updated_total);
}

// ---------------------------------------------------------------------------
// render + P1 Jacobian + gated weighted normal equations
// ---------------------------------------------------------------------------
// workgroup blk (8x8 pixel tile) of frame `frame` at *pose; the
// workgroup's 29 sums go to partial_row
template <typename T, bool Pool>
__device__ __forceinline__ void render_jac_block(int blk, int frame, const GridC& g, const CamC& c, const GridD& gd,
                                                 const CamD& cd, const T* __restrict__ map,
                                                 const unsigned* __restrict__ gbits, const prism_pose* __restrict__ pose,
                                                 const float* __restrict__ obs_depth,
                                                 const float* __restrict__ obs_rgb, const WeightsC& wt,
                                                 float* __restrict__ depth, float* __restrict__ rgb,
                                                 uint8_t* __restrict__ mask, float* __restrict__ Jout,
                                                 float* __restrict__ resid, uint8_t* __restrict__ rowmask,
                                                 double* __restrict__ partial_row) {
    __shared__ BlockPose sp;
    __shared__ double lds[kRedLds];
    extern __shared__ __align__(16) unsigned lbits[];
    const FreeBits fb = block_setup(g, gbits, lbits, pose, &sp);
    const BlockPose& P = sp;
    int u, v, s;
    quad_pixel(c, blk, u, v, s);
    // this lane's row in single precision, reduced over the workgroup by
    // block_reduce29f (single precision within 32 lanes, then double)
    float pacc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) pacc[q] = 0.0f;
    if (u < c.W && v < c.H) {
        float dir[3];
        ray_dir32(c, P.f, u, v, dir);
        const RayCoef rc = ray_coef(g, c, P.f, dir);
        int k = march_quad<T, Pool>(g, c, rc, map, fb, s);
        long long pix = (long long)frame * c.W * c.H + (long long)v * c.W + u;
        float row[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        double r = 0.0;
        int rm = 0;
        bool valid = k >= 1;
        double value = 0.0;
        if (valid) {
            Cell c0 = sample_cell(rc, k - 1), c1 = sample_cell(rc, k);
            QuadShade q = shade_quad<T, Pool>(g, gd, cd, P.d, u, v, map, c0, c1, k, s);
            value = q.value;
            float D = obs_depth[pix];
            if (depth_ok(D)) {
                jac_row_quad(g, q, dir, s, row);
                r = s == 0 ? value - (double)D : value - (double)obs_rgb[3 * pix + s - 1];
                // colour gate on |r_r| + |r_g| + |r_b| (lanes 1-3), depth gate on lane 0
                double l1 = s == 0 ? 0.0 : fabs(r);
                l1 = quad_sum(l1);
                bool use_depth = fabs(quad_bcast0(r)) <= wt.gate_depth;
                bool use_rgb = l1 <= wt.gate_rgb;
                rm = (use_depth ? 1 : 0) | (use_rgb ? 2 : 0);
                if (s == 0 ? use_depth : use_rgb)
                    neq_add32(pacc, row, (float)r, row_weight(wt, s != 0, r));
                if (rm && s == 0) pacc[28] = 1.0f;
            }
            if (!rm) {
#pragma unroll
                for (int m = 0; m < 6; ++m) row[m] = 0.0f;
                r = 0.0;
            }
        }
        if (s == 0) {
            if (depth) depth[pix] = valid ? (float)value : 0.0f;
            if (mask) mask[pix] = valid ? 1 : 0;
            if (rowmask) rowmask[pix] = (uint8_t)rm;
        } else if (rgb) {
            rgb[3 * pix + s - 1] = valid ? (float)value : 0.0f;
        }
        if (Jout) {
            float* jo = Jout + 24 * pix + 6 * s;
#pragma unroll
            for (int m = 0; m < 6; ++m) jo[m] = row[m];
        }
        if (resid) resid[4 * pix + s] = (float)r;
    }
    block_reduce29f(pacc, lds, partial_row);
}

template <typename T, bool Pool>
// at least 5 waves per SIMD (96 VGPRs, no spills; 4 without the cap)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_render_jac(GridC g, CamC c, GridD gd, CamD cd, const T* __restrict__ map,
                                                    const unsigned* __restrict__ gbits,
                                                    const prism_pose* __restrict__ poses,
                                                    const float* __restrict__ obs_depth,
                                                    const float* __restrict__ obs_rgb, WeightsC wt,
                                                    float* __restrict__ depth, float* __restrict__ rgb,
                                                    uint8_t* __restrict__ mask, float* __restrict__ Jout,
                                                    float* __restrict__ resid, uint8_t* __restrict__ rowmask,
                                                    double* __restrict__ partials) {
    render_jac_block<T, Pool>(blockIdx.x, blockIdx.y, g, c, gd, cd, map, gbits, poses + blockIdx.y, obs_depth, obs_rgb,
                              wt, depth, rgb, mask, Jout, resid, rowmask,
                              partials + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * PRISM_NEQ);
}

// batched: the render-through objective of every filter at its current
// iterate with its slot's frame (one frame each)
template <typename T, bool Pool>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_render_jac_batch(BatchArgs b) {
    const int a = batch_agent(b, blockIdx.x);
    const AgentDesc& D = *b.d[a];
    const prism_frame& fr = D.slots[b.slot[a]];
    const int blk = blockIdx.x - b.start[a];
    render_jac_block<T, Pool>(blk, 0, D.g, D.c, D.gd, D.cd, (const T*)D.map, D.bits, &D.S->iter,
                              (const float*)fr.depth, (const float*)fr.rgb, b.irls ? D.w_irls : D.w, nullptr, nullptr,
                              nullptr, nullptr, nullptr, nullptr, D.partials + (long long)blk * PRISM_NEQ);
}

// ---------------------------------------------------------------------------
// adjoint of render w.r.t. map means (atomic scatter) and pose
// ---------------------------------------------------------------------------
// Four lanes per ray, as in the render: lane s recomputes plane s of the
// forward pass at the ray's first crossing (the plane's corners at the two
// cells, the double-precision shading, its row of the Jacobian) and scatters
// its share of the upstream gradient to the plane's 16 corners.  The 64 rays
// of an 8x8 tile reach a few hundred distinct voxels through 1024 corners per
// plane: the contributions are summed in an LDS table per plane (open
// addressing on the voxel index), and each distinct (plane, voxel) then costs
// one global atomic.  A corner that finds no slot within a few probes is
// added to global memory directly.
constexpr int kVjpSlots = 512;   // per plane (power of two)
constexpr int kVjpProbes = 8;

struct VjpAgg {
    int key[4][kVjpSlots];       // voxel index, -1 = empty
    float val[4][kVjpSlots];
};

__device__ __forceinline__ void vjp_add(VjpAgg& A, int s, int id, float val, float* __restrict__ grad_mean,
                                        long long nvox) {
    const unsigned h = ((unsigned)id * 2654435761u) >> (32 - 9);
#pragma unroll 1
    for (int p = 0; p < kVjpProbes; ++p) {
        const int slot = (int)((h + p) & (kVjpSlots - 1));
        const int prev = atomicCAS(&A.key[s][slot], -1, id);
        if (prev == -1 || prev == id) {
            __hip_atomic_fetch_add(&A.val[s][slot], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
    }
    atomicAdd(grad_mean + (long long)s * nvox + id, val);
}

// coef * (trilinear weight) into plane s at the in-grid corners of the cell
__device__ __forceinline__ void vjp_cell(const GridC& g, VjpAgg& A, int s, const Cell& cl, const float w[3],
                                         float coef, float* __restrict__ grad_mean) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const int i = cl.i[0] + dx, j = cl.i[1] + dy, k = cl.i[2] + dz;
        if ((unsigned)i >= (unsigned)g.n || (unsigned)j >= (unsigned)g.n || (unsigned)k >= (unsigned)g.n) continue;
        const float hw = (dx ? w[0] : 1.0f - w[0]) * (dy ? w[1] : 1.0f - w[1]) * (dz ? w[2] : 1.0f - w[2]);
        vjp_add(A, s, (int)vidx(g, i, j, k), coef * hw, grad_mean, g.nvox);
    }
}

// sum over the quad in single precision (every lane ends with (x0 + x1) + (x2 + x3))
__device__ __forceinline__ float quad_sumf(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
    return x;
}

__global__ __launch_bounds__(256) void k_render_vjp(GridC g, CamC c, GridD gd, CamD cd, const float* __restrict__ map,
                                                    const prism_pose* __restrict__ poses,
                                                    const int32_t* __restrict__ hit_k,
                                                    const float* __restrict__ g_depth,
                                                    const float* __restrict__ g_rgb,
                                                    float* __restrict__ grad_mean,
                                                    double* __restrict__ partials) {
    __shared__ BlockPose sp;
    __shared__ double lds[kRedLds];
    __shared__ VjpAgg A;
    for (int e = threadIdx.x; e < 4 * kVjpSlots; e += 256) {
        (&A.key[0][0])[e] = -1;
        (&A.val[0][0])[e] = 0.0f;
    }
    const BlockPose& P = block_pose(poses + blockIdx.y, &sp);   // synchronises the workgroup
    int u, v, s;
    quad_pixel(c, blockIdx.x, u, v, s);
    double acc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) acc[q] = 0.0;
    if (u < c.W && v < c.H) {
        const long long pix = (long long)blockIdx.y * c.W * c.H + (long long)v * c.W + u;
        const int k = hit_k[pix];
        if (k >= 1 && k < c.K) {   // the same for the four lanes of a ray
            float dir[3];
            ray_dir32(c, P.f, u, v, dir);
            const RayCoef rc = ray_coef(g, c, P.f, dir);
            const Cell c0 = sample_cell(rc, k - 1), c1 = sample_cell(rc, k);
            const QuadShade q = shade_quad<float, false>(g, gd, cd, P.d, u, v, map, c0, c1, k, s);
            // the forward pass's crossing test on lane 0's occupancy corners
            const int crossing = trilerp(q.cv1, c1.w) > c.tau && !(trilerp(q.cv0, c0.w) > c.tau) ? 1 : 0;
            if (__builtin_amdgcn_update_dpp(0, crossing, 0x00, 0xF, 0xF, false)) {
                const float gs = s == 0 ? g_depth[pix] : g_rgb[3 * pix + s - 1];
                // pose: the upstream gradient times this output's Jacobian row
                float row[6];
                jac_row_quad(g, q, dir, s, row);
#pragma unroll
                for (int m = 0; m < 6; ++m) acc[m] = (double)(gs * row[m]);
                // means: every output depends on the two occupancies through
                // alpha; colour plane s also through its own blend
                const float ga = quad_sumf(gs * (s == 0 ? q.d1 - q.d0 : (float)q.v1 - (float)q.v0));
                const float al = (float)q.alpha;
                const float inv_den = (float)(1.0 / (q.f1 - q.f0));
                const float k0 = s == 0 ? -ga * (1.0f - al) * inv_den : gs * (1.0f - al);
                const float k1 = s == 0 ? -ga * al * inv_den : gs * al;
                vjp_cell(g, A, s, c0, q.w0, k0, grad_mean);
                vjp_cell(g, A, s, c1, q.w1, k1, grad_mean);
            }
        }
    }
    block_reduce29(acc, lds, partials + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * PRISM_NEQ);
    __syncthreads();
    // one global atomic per distinct (plane, voxel) of the tile
    for (int e = threadIdx.x; e < 4 * kVjpSlots; e += 256) {
        const int key = (&A.key[0][0])[e];
        if (key < 0) continue;
        atomicAdd(grad_mean + (long long)(e / kVjpSlots) * g.nvox + key, (&A.val[0][0])[e]);
    }
}

// ---------------------------------------------------------------------------
// gradient of the map-filter objective w.r.t. the map means (descent mapping)
// ---------------------------------------------------------------------------
// Per-workgroup accumulation table: the rays of an 8x8 tile touch a few
// hundred distinct (plane, voxel) pairs through thousands of trilinear
// corner contributions, so the contributions are summed in LDS first and each
// distinct pair costs one global atomic.  Open addressing on the voxel index
// (brick order) per plane; a contribution that finds no slot within a few
// probes goes straight to global memory.
constexpr int kAggSlots = 512;   // per plane (power of two)
constexpr int kAggProbes = 8;

struct GdAgg {
    int key[4][kAggSlots];      // voxel index, -1 = empty
    double val[4][kAggSlots];
};

// Sets the brick's bit; the caller that flips it appends the brick to the
// list of bricks the step has to visit.
__device__ __forceinline__ void mark_brick(unsigned* __restrict__ marks, int* __restrict__ list, int b) {
    const unsigned bit = 1u << (b & 31);
    if (marks[b >> 5] & bit) return;
    const unsigned old = atomicOr(marks + (b >> 5), bit);
    if (!(old & bit)) {
        const int at = atomicAdd(list, 1);
        list[1 + at] = b;
    }
}

__device__ __forceinline__ void agg_add(GdAgg& A, int s, long long id, double val, double* __restrict__ grad,
                                        long long nvox, unsigned* __restrict__ marks, int* __restrict__ list) {
    const int key = (int)id;
    unsigned h = ((unsigned)key * 2654435761u) >> (32 - 9);
#pragma unroll 1
    for (int p = 0; p < kAggProbes; ++p) {
        const int slot = (int)((h + p) & (kAggSlots - 1));
        const int prev = atomicCAS(&A.key[s][slot], -1, key);
        if (prev == -1 || prev == key) {
            __hip_atomic_fetch_add(&A.val[s][slot], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
    }
    unsafeAtomicAdd(grad + (long long)s * nvox + id, val);
    mark_brick(marks, list, (int)(id >> 9));
}

// coef * (trilinear weight) for the in-grid corners of the cell
__device__ __forceinline__ void agg_cell(const GridC& g, GdAgg& A, int s, const Cell& cl, const float w[3],
                                         double coef, double* __restrict__ grad, unsigned* __restrict__ marks,
                                         int* __restrict__ list) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const int i = cl.i[0] + dx, j = cl.i[1] + dy, k = cl.i[2] + dz;
        if ((unsigned)i >= (unsigned)g.n || (unsigned)j >= (unsigned)g.n || (unsigned)k >= (unsigned)g.n) continue;
        const double hw = (double)(dx ? w[0] : 1.0f - w[0]) * (double)(dy ? w[1] : 1.0f - w[1]) *
                          (double)(dz ? w[2] : 1.0f - w[2]);
        agg_add(A, s, vidx(g, i, j, k), coef * hw, grad, g.nvox, marks, list);
    }
}

// One frame's rows of the map-filter objective at the current means: the
// render-through rows (same validity, gates and weights as the P1 objective)
// give the cost sum w r^2 (per-workgroup partial) and, through the adjoint of
// the emission with the first crossing held, dE/dmean = sum 2 w r d(out)/dmean
// accumulated in double precision into grad [4][n^3] (brick order).  Every
// brick that receives a contribution is marked, and appended to `list`
// (count first) the first time.
__global__ __launch_bounds__(256) void k_gd_grad(GridC g, CamC c, GridD gd, CamD cd, const float* __restrict__ map,
                                                 const unsigned* __restrict__ gbits,
                                                 const prism_pose* __restrict__ pose,
                                                 const float* __restrict__ obs_depth,
                                                 const float* __restrict__ obs_rgb, WeightsC wt,
                                                 double* __restrict__ grad, unsigned* __restrict__ marks,
                                                 int* __restrict__ list, double* __restrict__ partials) {
    __shared__ BlockPose sp;
    __shared__ double wsum[4];
    __shared__ GdAgg A;
    extern __shared__ __align__(16) unsigned lbits[];
    for (int e = threadIdx.x; e < 4 * kAggSlots; e += 256) {
        (&A.key[0][0])[e] = -1;
        (&A.val[0][0])[e] = 0.0;
    }
    const FreeBits fb = block_setup(g, gbits, lbits, pose, &sp);   // synchronises the workgroup
    const BlockPose& P = sp;
    int u, v, s;
    quad_pixel(c, blockIdx.x, u, v, s);
    double cost = 0.0;
    if (u < c.W && v < c.H) {
        float dir[3];
        ray_dir32(c, P.f, u, v, dir);
        const RayCoef rc = ray_coef(g, c, P.f, dir);
        const int k = march_quad<float, false>(g, c, rc, map, fb, s);
        const long long pix = (long long)v * c.W + u;
        const float D = obs_depth[pix];
        if (k >= 1 && depth_ok(D)) {   // the same for the four lanes of a ray
            const Cell c0 = sample_cell(rc, k - 1), c1 = sample_cell(rc, k);
            const QuadShade q = shade_quad<float, false>(g, gd, cd, P.d, u, v, map, c0, c1, k, s);
            const double r = s == 0 ? q.value - (double)D : q.value - (double)obs_rgb[3 * pix + s - 1];
            double l1 = s == 0 ? 0.0 : fabs(r);
            l1 = quad_sum(l1);
            const bool use_depth = fabs(quad_bcast0(r)) <= wt.gate_depth;
            const bool use_rgb = l1 <= wt.gate_rgb;
            const bool keep = s == 0 ? use_depth : use_rgb;
            const double w = s == 0 ? wt.w_depth : wt.w_rgb;
            const double gout = keep ? 2.0 * w * r : 0.0;   // dE / d(this lane's output)
            if (keep) cost = w * r * r;
            // every output depends on the two occupancies through alpha
            const double d0 = cd.dn + (double)(k - 1) * cd.step, d1 = cd.dn + (double)k * cd.step;
            double ga = gout * (s == 0 ? d1 - d0 : q.v1 - q.v0);
            ga += __shfl_xor(ga, 1, 64);
            ga += __shfl_xor(ga, 2, 64);
            const double inv_den = 1.0 / (q.f1 - q.f0);
            double k0, k1;   // coefficients of this lane's plane at the cells of samples k*-1, k*
            if (s == 0) {
                k0 = -ga * (1.0 - q.alpha) * inv_den;
                k1 = -ga * q.alpha * inv_den;
            } else {
                k0 = gout * (1.0 - q.alpha);
                k1 = gout * q.alpha;
            }
            if (k0 != 0.0) agg_cell(g, A, s, c0, q.w0, k0, grad, marks, list);
            if (k1 != 0.0) agg_cell(g, A, s, c1, q.w1, k1, grad, marks, list);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cost;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    // one global atomic per distinct (plane, voxel) of the tile
    for (int e = threadIdx.x; e < 4 * kAggSlots; e += 256) {
        const int key = (&A.key[0][0])[e];
        if (key < 0) continue;
        const int pl = e / kAggSlots;
        unsafeAtomicAdd(grad + (long long)pl * g.nvox + key, (&A.val[0][0])[e]);
        mark_brick(marks, list, key >> 9);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int render_blocks(const CamC& c) { return ((c.W + 7) >> 3) * ((c.H + 7) >> 3); }
int vjp_blocks(const CamC& c) { return render_blocks(c); }

static size_t bits_lds(const GridC& g, const unsigned* bits) {
    return bits ? (size_t)free_lds_words(free_words(g.nb)) * 4 : 0;
}

hipError_t launch_render(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, int dtype, const void* map,
                         const unsigned* bits, const prism_pose* poses, int n_frames, float* depth, float* rgb,
                         uint8_t* mask, int32_t* hit_k, hipStream_t st) {
    dim3 grid(render_blocks(c), n_frames);
    size_t lds = bits_lds(g, bits);
    const bool pool = g.table != nullptr;
    const uint16_t* mh = (const uint16_t*)map;
    const float* mf = (const float*)map;
    if (dtype == PRISM_BF16 && pool)
        k_render<uint16_t, true><<<grid, 256, lds, st>>>(g, c, gd, cd, mh, bits, poses, depth, rgb, mask, hit_k);
    else if (dtype == PRISM_BF16)
        k_render<uint16_t, false><<<grid, 256, lds, st>>>(g, c, gd, cd, mh, bits, poses, depth, rgb, mask, hit_k);
    else if (pool)
        k_render<float, true><<<grid, 256, lds, st>>>(g, c, gd, cd, mf, bits, poses, depth, rgb, mask, hit_k);
    else
        k_render<float, false><<<grid, 256, lds, st>>>(g, c, gd, cd, mf, bits, poses, depth, rgb, mask, hit_k);
    return hipGetLastError();
}

hipError_t launch_render_batch(const BatchArgs& b, int dtype, bool pool, int max_lds_words, hipStream_t st) {
    // every filter copies free_lds_words of its bits to LDS (block_setup):
    // the allocation is the largest of these over the batch
    size_t lds = (size_t)max_lds_words * 4;
    if (dtype == PRISM_BF16 && pool)
        k_render_batch<uint16_t, true><<<b.start[b.n], 256, lds, st>>>(b);
    else if (dtype == PRISM_BF16)
        k_render_batch<uint16_t, false><<<b.start[b.n], 256, lds, st>>>(b);
    else if (pool)
        k_render_batch<float, true><<<b.start[b.n], 256, lds, st>>>(b);
    else
        k_render_batch<float, false><<<b.start[b.n], 256, lds, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_render_jac_batch(const BatchArgs& b, int dtype, bool pool, int max_lds_words, hipStream_t st) {
    size_t lds = (size_t)max_lds_words * 4;
    if (dtype == PRISM_BF16 && pool)
        k_render_jac_batch<uint16_t, true><<<b.start[b.n], 256, lds, st>>>(b);
    else if (dtype == PRISM_BF16)
        k_render_jac_batch<uint16_t, false><<<b.start[b.n], 256, lds, st>>>(b);
    else if (pool)
        k_render_jac_batch<float, true><<<b.start[b.n], 256, lds, st>>>(b);
    else
        k_render_jac_batch<float, false><<<b.start[b.n], 256, lds, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_normals_batch(const BatchArgs& b, hipStream_t st) {
    k_normals_batch<<<b.start[b.n], 256, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_normals(const CamC& c, int n_frames, const float* depth, const uint8_t* mask, float disc,
                          float* normals, uint8_t* nmask, const int* counts, int ngroups, int64_t* n_updated,
                          int64_t* n_updated_total, hipStream_t st) {
    long long n = (long long)c.W * c.H * n_frames;
    k_normals<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(c, n_frames, depth, mask, disc, normals, nmask, counts,
                                                           ngroups, n_updated, n_updated_total);
    return hipGetLastError();
}

hipError_t launch_render_jac(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, int dtype,
                             const void* map, const unsigned* bits, const prism_pose* poses, int n_frames,
                             const float* obs_depth, const float* obs_rgb, const WeightsC& w, float* depth,
                             float* rgb, uint8_t* mask, float* J, float* resid, uint8_t* rowmask, double* partials,
                             hipStream_t st) {
    dim3 grid(render_blocks(c), n_frames);
    size_t lds = bits_lds(g, bits);
    const bool pool = g.table != nullptr;
    const uint16_t* mh = (const uint16_t*)map;
    const float* mf = (const float*)map;
    if (dtype == PRISM_BF16 && pool)
        k_render_jac<uint16_t, true><<<grid, 256, lds, st>>>(g, c, gd, cd, mh, bits, poses, obs_depth, obs_rgb, w,
                                                             depth, rgb, mask, J, resid, rowmask, partials);
    else if (dtype == PRISM_BF16)
        k_render_jac<uint16_t, false><<<grid, 256, lds, st>>>(g, c, gd, cd, mh, bits, poses, obs_depth, obs_rgb, w,
                                                              depth, rgb, mask, J, resid, rowmask, partials);
    else if (pool)
        k_render_jac<float, true><<<grid, 256, lds, st>>>(g, c, gd, cd, mf, bits, poses, obs_depth, obs_rgb, w,
                                                          depth, rgb, mask, J, resid, rowmask, partials);
    else
        k_render_jac<float, false><<<grid, 256, lds, st>>>(g, c, gd, cd, mf, bits, poses, obs_depth, obs_rgb, w,
                                                           depth, rgb, mask, J, resid, rowmask, partials);
    return hipGetLastError();
}

hipError_t launch_gd_grad(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, const float* map,
                          const unsigned* bits, const prism_pose* pose, const float* obs_depth, const float* obs_rgb,
                          const WeightsC& w, double* grad, unsigned* marks, int* list, double* partials,
                          hipStream_t st) {
    k_gd_grad<<<render_blocks(c), 256, bits_lds(g, bits), st>>>(g, c, gd, cd, map, bits, pose, obs_depth, obs_rgb, w,
                                                                grad, marks, list, partials);
    return hipGetLastError();
}

hipError_t launch_render_vjp(const GridC& g, const CamC& c, const GridD& gd, const CamD& cd, const float* map,
                             const prism_pose* poses, int n_frames, const int32_t* hit_k, const float* g_depth,
                             const float* g_rgb, float* grad_mean, double* partials, hipStream_t st) {
    dim3 grid(vjp_blocks(c), n_frames);
    k_render_vjp<<<grid, 256, 0, st>>>(g, c, gd, cd, map, poses, hit_k, g_depth, g_rgb, grad_mean, partials);
    return hipGetLastError();
}

}  // namespace prism
