// Device-side building blocks shared by the gfx950 kernels.
//
// Single-precision decision recipe.  Every integer the kernels derive from
// floating point (interpolation cell, hit sample, pixel of a voxel, anchor
// pixel of a point) is computed in IEEE single precision with a fixed
// operation order and no contraction (this library is built with
// -ffp-contract=off; division is IEEE correctly rounded).  The order is:
//   ray:    rx = ((float)u + 0.5f - cx) * ifx;  ry likewise;
//           dir_i = (R_i0 rx + R_i1 ry) + R_i2
//   sample: per ray B_i = (dir_i * dstep) * inv_s and
//           A_i = ((t_i + d_near * dir_i) - o_i) * inv_s - 0.5f; for sample k
//           g_i = fma((float)k, B_i, A_i);  cell = floor(g);  w = g - cell;
//           occupancy = lerp_z(lerp_y(lerp_x(corners))) with
//           lerp(a, b, w) = fma(w, b - a, a)
//           (fma: one rounding of the exact a*b + c, written out explicitly)
//   voxel:  x_i = o_i + s ((float)i + 0.5f);  d = x - t;
//           X_a = (R_0a d_0 + R_1a d_1) + R_2a d_2;
//           u = fx (X_0 / X_2) + cx,  v = fy (X_1 / X_2) + cy
// where R, t are the pose rounded to float after the quaternion -> matrix
// conversion in double precision, and ifx = (float)(1/fx), inv_s =
// (float)(1/voxel), dstep = (float)((d_far - d_near)/(K - 1)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#include "../../include/prism.h"

namespace prism {

constexpr int kBrick = 8;          // brick edge (voxels)
constexpr int kBrickVox = 512;     // voxels per brick

// ---------------------------------------------------------------------------
// per-call constants (computed on the host, passed by value)
// ---------------------------------------------------------------------------
struct GridC {
    float o[3];
    float s, inv_s;
    float occ_out, rgb_out;
    int n;       // voxels per axis
    int nb;      // bricks per axis
    long long nvox;   // plane stride in elements: n^3 (dense), capacity * 512 (brick pool)
    const int* table;   // brick-pool maps: slot of each brick or -1; NULL for dense maps
    float pocc, prgb;   // brick-pool maps: occupancy / colour a voxel without a slot reads as
                        // (the outside values as the storage type holds them)
};

struct CamC {
    float ifx, ify, fx, fy, cx, cy;
    float dn, dstep, tau;
    int W, H, K;
};

// Double-precision copies of the parameters for the value path: once the
// integer decisions are taken, values (sample points, interpolation weights,
// occupancies, depths, colours, camera depths of voxels) are computed in
// double precision from the definitions and rounded once on output.
struct GridD {
    double o[3];
    double s;
    double occ_out, rgb_out;
    double inv_s;   // 1 / s
};

struct CamD {
    double fx, fy, cx, cy;
    double dn, step, tau;
    double ifx, ify;   // 1 / fx, 1 / fy
};

// Derived data and scratch that live in the map buffer after the planes.
struct MapAux {
    float* bmax;      // [nb^3] largest occupancy mean of each brick
    unsigned* bits;   // [2 ceil(nb^3/32)] bit b set iff bmax[b] <= 0 (free-space bricks), then the
                      // dilated bits: bit b set iff bits b + {0, 1} + {0, nb} + {0, nb^2} are all
                      // set (past the last brick: 0), i.e. for a brick off the grid's last layers
                      // the 2x2x2 block of bricks with lowest corner b is free
    int* counts;      // [kUpdateGrid] updated voxels per workgroup of the last update
    int* list;        // [nb^3] bricks in the view frustum, in 256-brick segments
    int* segcnt;      // [ceil(nb^3/256)] entries used in each segment
    void* pose;       // Pose32 then Pose64 of the current update (256 bytes)
    // brick-pool maps only (NULL for dense maps)
    int* table;       // [nb^3] slot of each brick, -1 without one
    int* pool;        // [0] slots handed out, [1] brick updates dropped (pool full)
    float* var0;      // variance a brick's voxels take when it is given a slot
    int capacity;     // slots in the pool
};

constexpr int kUpdateGrid = 2048;   // workgroups of the map-update kernel

// words of one free-space bitmap (one bit per brick)
__host__ __device__ inline int free_words(int nb) { return (nb * nb * nb + 31) >> 5; }

// LDS words a render workgroup keeps of a grid's free-space bits: both
// bitmaps when they fit, else the plain bits (cells that span bricks are then
// tested brick by brick), else none (no skipping)
constexpr int kMaxLdsWords = 12288;   // 48 KB
__host__ __device__ inline int free_lds_words(int nwords) {
    return 2 * nwords <= kMaxLdsWords ? 2 * nwords : nwords <= kMaxLdsWords ? nwords : 0;
}

// ---------------------------------------------------------------------------
// pose -> single-precision rotation/translation
// ---------------------------------------------------------------------------
struct Pose32 {
    float R[3][3];
    float t[3];
};

struct Pose64 {
    double R[3][3];
    double t[3];
};

__device__ inline void quat_to_rot64(const prism_pose& p, double R[3][3]) {
    double w = p.q[0], x = p.q[1], y = p.q[2], z = p.q[3];
    double nrm = sqrt(w * w + x * x + y * y + z * z);
    w /= nrm; x /= nrm; y /= nrm; z /= nrm;
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ inline Pose64 load_pose64(const prism_pose* pp) {
    Pose64 o;
    prism_pose p = *pp;
    quat_to_rot64(p, o.R);
    for (int i = 0; i < 3; ++i) o.t[i] = p.t[i];
    return o;
}

// The current camera relative to the anchor camera, as the tracking objective
// uses it: R, t (current -> anchor) in single precision for the association
// recipe, both poses in double precision for the values.  A filter keeps its
// own copy, formed whenever its iterate changes (predict, Gauss-Newton step).
struct Rel32 {
    float R[3][3], t[3];   // current camera -> anchor camera (association recipe)
    Pose64 cur, prev;      // both poses in double precision (values)
};

__device__ __forceinline__ void rel_of(const prism_pose* pose, const prism_pose* pose_prev, Rel32& rel) {
    Pose64 P = load_pose64(pose), Q = load_pose64(pose_prev);
    double d[3] = {P.t[0] - Q.t[0], P.t[1] - Q.t[1], P.t[2] - Q.t[2]};
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            rel.R[a][b] = (float)((Q.R[0][a] * P.R[0][b] + Q.R[1][a] * P.R[1][b]) + Q.R[2][a] * P.R[2][b]);
        rel.t[a] = (float)((Q.R[0][a] * d[0] + Q.R[1][a] * d[1]) + Q.R[2][a] * d[2]);
    }
    rel.cur = P;
    rel.prev = Q;
}

__device__ __forceinline__ void pixel_dir64(const CamD& c, int u, int v, double r[3]) {
    r[0] = (((double)u + 0.5) - c.cx) * c.ifx;
    r[1] = (((double)v + 0.5) - c.cy) * c.ify;
    r[2] = 1.0;
}

__device__ inline Pose32 to32(const Pose64& p) {
    Pose32 o;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) o.R[i][j] = (float)p.R[i][j];
        o.t[i] = (float)p.t[i];
    }
    return o;
}

// ---------------------------------------------------------------------------
// map storage
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ld(const float* p, long long i) { return p[i]; }
__device__ __forceinline__ float ld(const uint16_t* p, long long i) {
    return __uint_as_float(((uint32_t)p[i]) << 16);
}
__device__ __forceinline__ void st(float* p, long long i, float v) { p[i] = v; }
// single precision -> BF16, round to nearest even (gfx950's conversion
// instruction; a NaN stays a NaN)
__device__ __forceinline__ uint16_t f2bf(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ void st(uint16_t* p, long long i, float v) { p[i] = f2bf(v); }

// Element index within a plane of voxel (i, j, k), all in [0, n): brick order
// (brick b, then z, y, x inside the brick); in a brick-pool map the brick's
// slot replaces b, and -1 means the brick has none (the voxel then reads as
// the grid's outside values).
template <bool Pool = false>
__device__ __forceinline__ long long vidx(const GridC& g, int i, int j, int k) {
    long long b = ((long long)(k >> 3) * g.nb + (j >> 3)) * g.nb + (i >> 3);
    const long long loc = ((k & 7) << 6) | ((j & 7) << 3) | (i & 7);
    if constexpr (Pool) {
        const int slot = g.table[b];
        return slot < 0 ? -1 : ((long long)slot << 9) | loc;
    }
    return (b << 9) | loc;
}

// ---------------------------------------------------------------------------
// the single-precision ray/sample recipe
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ray_dir32(const CamC& c, const Pose32& P, int u, int v, float dir[3]) {
    float rx = ((float)u + 0.5f - c.cx) * c.ifx;
    float ry = ((float)v + 0.5f - c.cy) * c.ify;
#pragma unroll
    for (int a = 0; a < 3; ++a) dir[a] = (P.R[a][0] * rx + P.R[a][1] * ry) + P.R[a][2];
}

// trilinear cell of a sample (base corner) and the weights within it
struct Cell {
    int i[3];
    float w[3];
};

// Per-ray coefficients of the sample recipe: the continuous grid coordinate
// of sample k is A + k B per axis, with
//   B = (dir * dstep) / voxel,  A = ((t + d_near dir) - origin) / voxel - 1/2
// (single precision, this operation order, 1/voxel as a rounded factor).
struct RayCoef {
    float A[3], B[3];
};

__device__ __forceinline__ RayCoef ray_coef(const GridC& g, const CamC& c, const Pose32& P, const float dir[3]) {
    RayCoef r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.B[a] = (dir[a] * c.dstep) * g.inv_s;
        r.A[a] = ((P.t[a] + c.dn * dir[a]) - g.o[a]) * g.inv_s - 0.5f;
    }
    return r;
}

// continuous grid coordinate of sample fk (an integer held in a float) on axis a
__device__ __forceinline__ float sample_gc(const RayCoef& r, float fk, int a) {
    return __builtin_fmaf(fk, r.B[a], r.A[a]);
}

// floor(x) as an integer in one instruction (saturating outside the int range)
__device__ __forceinline__ int floor_i32(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ Cell sample_cell(const RayCoef& r, int k) {
    Cell o;
    const float fk = (float)k;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float gc = sample_gc(r, fk, a);
        float fl = floorf(gc);
        o.i[a] = (int)fl;
        o.w[a] = gc - fl;
    }
    return o;
}

__device__ __forceinline__ float lerp32(float a, float b, float w) { return __builtin_fmaf(w, b - a, a); }

// Addressing of a trilinear cell whose 8 corners are all inside the grid:
// the base corner's element index within a plane (32 bits: n <= 1024) and the
// steps to its +x, +y and +z neighbours, which jump to the next brick when the
// base sits on a brick's last voxel along that axis.
struct CellAddr {
    int base, dx, dy, dz;
    int b0;       // brick of the base corner
    bool cross;   // the cell spans more than one brick
};

__device__ __forceinline__ bool cell_inside(const GridC& g, const Cell& c) {
    const unsigned lim = (unsigned)(g.n - 1);
    return (unsigned)c.i[0] < lim && (unsigned)c.i[1] < lim && (unsigned)c.i[2] < lim;
}

__device__ __forceinline__ CellAddr cell_addr(const GridC& g, const Cell& c) {
    CellAddr a;
    const int lx = c.i[0] & 7, ly = c.i[1] & 7, lz = c.i[2] & 7;
    a.b0 = ((c.i[2] >> 3) * g.nb + (c.i[1] >> 3)) * g.nb + (c.i[0] >> 3);
    a.base = (a.b0 << 9) | (lz << 6) | (ly << 3) | lx;
    a.dx = lx == 7 ? 512 - 7 : 1;
    a.dy = ly == 7 ? 512 * g.nb - 56 : 8;
    a.dz = lz == 7 ? 512 * g.nb * g.nb - 448 : 64;
    a.cross = (lx == 7) | (ly == 7) | (lz == 7);
    return a;
}


// Explicit address spaces for the hottest loads: through a global-space
// pointer with a 32-bit byte offset the compiler can use a scalar base and a
// single vector offset register per load (instead of a flat load with a
// 64-bit vector address), and LDS-space pointers become LDS reads.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
using lds_u32 = const __attribute__((address_space(3))) unsigned;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
    return (gptr<T>)p;
}

__device__ __forceinline__ float ldg(gptr<float> p, unsigned byte_off) {
    return *(gptr<float>)((gptr<char>)p + byte_off);
}
__device__ __forceinline__ float ldg(gptr<uint16_t> p, unsigned byte_off) {
    return __uint_as_float(((uint32_t) * (gptr<uint16_t>)((gptr<char>)p + byte_off)) << 16);
}

// corners_in through a global-space plane pointer (byte offsets; a plane is
// at most 2^30 elements of at most 4 bytes, so offsets fit 32 bits)
template <typename T>
__device__ __forceinline__ void corners_in_g(gptr<T> plane, const CellAddr& a, float v[8]) {
    constexpr unsigned sz = sizeof(T);
    const unsigned o = (unsigned)a.base * sz, dx = (unsigned)a.dx * sz, dy = (unsigned)a.dy * sz,
                   dz = (unsigned)a.dz * sz;
    v[0] = ldg(plane, o);
    v[1] = ldg(plane, o + dx);
    v[2] = ldg(plane, o + dy);
    v[3] = ldg(plane, o + dy + dx);
    v[4] = ldg(plane, o + dz);
    v[5] = ldg(plane, o + dz + dx);
    v[6] = ldg(plane, o + dz + dy);
    v[7] = ldg(plane, o + dz + dy + dx);
}

// 8 corner values of one plane: out-of-grid corners take `outv`, corners in
// bricks without a slot (brick-pool maps) `priorv`
template <typename T, bool Pool>
__device__ __forceinline__ void corners(const GridC& g, const T* plane, const Cell& c, float outv, float priorv,
                                        float v[8]) {
    if (cell_inside(g, c)) {
        CellAddr a = cell_addr(g, c);
        if constexpr (!Pool) {
            corners_in_g(as_global(plane), a, v);
            return;
        }
        if (!a.cross) {
            // one brick: its slot, then the dense steps inside it
            const int slot = g.table[a.b0];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = priorv;
            if (slot >= 0) {
                a.base = (slot << 9) | (a.base & 511);
                corners_in_g(as_global(plane), a, v);
            }
            return;
        }
    }
    bool okx0 = (unsigned)c.i[0] < (unsigned)g.n, okx1 = (unsigned)(c.i[0] + 1) < (unsigned)g.n;
    bool oky0 = (unsigned)c.i[1] < (unsigned)g.n, oky1 = (unsigned)(c.i[1] + 1) < (unsigned)g.n;
    bool okz0 = (unsigned)c.i[2] < (unsigned)g.n, okz1 = (unsigned)(c.i[2] + 1) < (unsigned)g.n;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        bool ok = (dx ? okx1 : okx0) && (dy ? oky1 : oky0) && (dz ? okz1 : okz0);
        const long long e = ok ? vidx<Pool>(g, c.i[0] + dx, c.i[1] + dy, c.i[2] + dz) : -1;
        v[q] = e >= 0 ? ld(plane, e) : ok ? priorv : outv;
    }
}

// trilinear value from corners v[q], q = dx + 2 dy + 4 dz
__device__ __forceinline__ float trilerp(const float v[8], const float w[3]) {
    float l00 = lerp32(v[0], v[1], w[0]);
    float l10 = lerp32(v[2], v[3], w[0]);
    float l01 = lerp32(v[4], v[5], w[0]);
    float l11 = lerp32(v[6], v[7], w[0]);
    float m0 = lerp32(l00, l10, w[1]);
    float m1 = lerp32(l01, l11, w[1]);
    return lerp32(m0, m1, w[2]);
}

// gradient of the trilinear interpolant w.r.t. the grid coordinate
__device__ __forceinline__ void trigrad(const float v[8], const float w[3], float gr[3]) {
    float wx0 = 1.0f - w[0], wy0 = 1.0f - w[1], wz0 = 1.0f - w[2];
    gr[0] = wy0 * wz0 * (v[1] - v[0]) + w[1] * wz0 * (v[3] - v[2]) + wy0 * w[2] * (v[5] - v[4]) +
            w[1] * w[2] * (v[7] - v[6]);
    gr[1] = wx0 * wz0 * (v[2] - v[0]) + w[0] * wz0 * (v[3] - v[1]) + wx0 * w[2] * (v[6] - v[4]) +
            w[0] * w[2] * (v[7] - v[5]);
    gr[2] = wx0 * wy0 * (v[4] - v[0]) + w[0] * wy0 * (v[5] - v[1]) + wx0 * w[1] * (v[6] - v[2]) +
            w[0] * w[1] * (v[7] - v[3]);
}

// ---------------------------------------------------------------------------
// reductions of the 29-double normal equations
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

constexpr int kRedLds = 32 * 16;   // doubles of LDS scratch for block_reduce29

// Reduce a per-thread 29-vector over the block (blockDim.x a multiple of 64,
// <= 1024) into out[0..28] (written by threads 0..28).  lds: kRedLds doubles.
//
// Within a wave the 29 sums use a halving exchange instead of 29 separate
// butterfly reductions: at the step with offset o (16, 8, 4, 2, 1) each lane
// keeps the half of its remaining values selected by its lane bit o, sends
// the other half to lane ^ o and adds what it receives.  After five steps
// lane l holds value l & 31 summed over its 32-lane half, one more exchange
// (offset 32) completes the wave sum: 32 double shuffles per wave instead of
// 29 * 6.  Summation order is fixed, so results are deterministic.
__device__ inline void block_reduce29(double acc[PRISM_NEQ], double* lds, double* out) {
    double v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = q < PRISM_NEQ ? acc[q] : 0.0;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int half = 16; half >= 1; half >>= 1) {
        bool hi = (lane & half) != 0;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            double send = hi ? v[j] : v[j + half];
            double keep = hi ? v[j + half] : v[j];
            v[j] = keep + __shfl_xor(send, half, 64);
        }
    }
    double w = v[0] + __shfl_xor(v[0], 32, 64);   // value (lane & 31), whole wave
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // one row of 32 per wavefront: the stores of a wavefront and the loads of
    // each step of the sum below hit consecutive doubles (no bank conflicts)
    if (lane < 32) lds[wv * 32 + lane] = w;
    __syncthreads();
    if (threadIdx.x < PRISM_NEQ) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += lds[k * 32 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// The same for single-precision per-lane sums (a pixel's or ray's few rows):
// the five halving steps inside each 32-lane half run in single precision
// (one 4-byte exchange per value instead of two), each lane widens its one
// remaining value, and the step across halves and the sum over waves are in
// double precision.  A single-precision sum spans at most 32 lanes (relative
// error below 32 ulp of the sum of magnitudes); the order is fixed, so
// results are deterministic.
__device__ inline void block_reduce29f(const float acc[PRISM_NEQ], double* lds, double* out) {
    float v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = q < PRISM_NEQ ? acc[q] : 0.0f;
    const int lane = threadIdx.x & 63;
    // transposing halving within each 32-lane half: after the step of width
    // h a lane keeps the h values of the half of its index set selected by
    // its lane bit h, each summed with the same value of a partner lane
    // whose bit h differs.  Width 16: the row swap of v[j] and v[j + 16]
    // hands lanes 0-15 (32-47) their partner's v[j] and lanes 16-31 (48-63)
    // their partner's v[j + 16]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 16]), false,
                                                        false);
        v[j] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    // widths 8, 4, 2, 1 inside 16-lane rows: the partner read by DPP is
    // lane ^ 8 (row rotate by 8), lane ^ 7 (half-row mirror), lane ^ 2 and
    // lane ^ 1 (quad permutations); at each width all lanes that agree on
    // the bits already used hold the same index set, so any partner that
    // differs in bit h and agrees on the higher bits serves
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int h = 8 >> step;
        const bool hi = (lane & h) != 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j >= h) break;
            int a = __float_as_int(v[j]), b = __float_as_int(v[j + h]);
            int pa, pb;
            if (step == 0) {
                pa = __builtin_amdgcn_update_dpp(0, a, 0x128, 0xF, 0xF, false);
                pb = __builtin_amdgcn_update_dpp(0, b, 0x128, 0xF, 0xF, false);
            } else if (step == 1) {
                pa = __builtin_amdgcn_update_dpp(0, a, 0x141, 0xF, 0xF, false);
                pb = __builtin_amdgcn_update_dpp(0, b, 0x141, 0xF, 0xF, false);
            } else if (step == 2) {
                pa = __builtin_amdgcn_update_dpp(0, a, 0x4E, 0xF, 0xF, false);
                pb = __builtin_amdgcn_update_dpp(0, b, 0x4E, 0xF, 0xF, false);
            } else {
                pa = __builtin_amdgcn_update_dpp(0, a, 0xB1, 0xF, 0xF, false);
                pb = __builtin_amdgcn_update_dpp(0, b, 0xB1, 0xF, 0xF, false);
            }
            const float lo = v[j] + __int_as_float(pa), up = v[j + h] + __int_as_float(pb);
            v[j] = hi ? up : lo;
        }
    }
    // lane l holds index l & 31 summed over its 32-lane half; the halves are
    // added in double precision through the 32-lane swap
    const double h = (double)v[0];
    const unsigned hl = (unsigned)__double2loint(h), hh = (unsigned)__double2hiint(h);
    const auto sl = __builtin_amdgcn_permlane32_swap(hl, hl, false, false);
    const auto sh = __builtin_amdgcn_permlane32_swap(hh, hh, false, false);
    const double w = __hiloint2double((int)sh[0], (int)sl[0]) + __hiloint2double((int)sh[1], (int)sl[1]);
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // one row of 32 per wavefront: the stores of a wavefront and the loads of
    // each step of the sum below hit consecutive doubles (no bank conflicts)
    if (lane < 32) lds[wv * 32 + lane] = w;
    __syncthreads();
    if (threadIdx.x < PRISM_NEQ) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += lds[k * 32 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// one residual row (Jacobian row j, residual r, weight w) into the
// 29-double normal equations, products formed in double precision
__device__ __forceinline__ void neq_add(double acc[PRISM_NEQ], const float j[6], double r, double w) {
    double jd[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) jd[a] = (double)j[a];
    int q = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b) acc[q++] += w * jd[a] * jd[b];
#pragma unroll
    for (int a = 0; a < 6; ++a) acc[21 + a] += w * jd[a] * r;
    acc[27] += w * r * r;
}

// the same in single precision, for one pixel's few rows (fused multiply-
// adds: these sums are values, no decision depends on their rounding)
__device__ __forceinline__ void neq_add32(float acc[PRISM_NEQ], const float j[6], float r, float w) {
    float wj[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) wj[a] = w * j[a];
    int q = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b, ++q) acc[q] = fmaf(wj[a], j[b], acc[q]);
#pragma unroll
    for (int a = 0; a < 6; ++a) acc[21 + a] = fmaf(wj[a], r, acc[21 + a]);
    acc[27] = fmaf(w * r, r, acc[27]);
}

// Weights and gates of the objective rows.  irls != 0: a kept row of the L1
// objective (App. E.3) is reweighted at its current residual r by
// h / max(|r|, f), with h = 1/(2b) and f = floor * b for its kind (b = 1/sqrt(w)).
struct WeightsC {
    double w_depth, w_rgb, gate_depth, gate_rgb;
    float irls_h_depth, irls_h_rgb, irls_f_depth, irls_f_rgb;
    int irls;
};

// weight of a kept depth (rgb = false) or colour row with residual r
__device__ __forceinline__ float row_weight(const WeightsC& wt, bool rgb, double r) {
    if (!wt.irls) return (float)(rgb ? wt.w_rgb : wt.w_depth);
    return (rgb ? wt.irls_h_rgb : wt.irls_h_depth) / fmaxf(fabsf((float)r), rgb ? wt.irls_f_rgb : wt.irls_f_depth);
}

__device__ __forceinline__ bool depth_ok(float d) { return d > 0.0f && isfinite(d); }

// *n_updated = sum of counts[0..ngroups) (ngroups <= 2048) by a whole
// 256-thread workgroup: every lane issues its (up to 8) loads before adding,
// so the sum costs one memory round trip, not ngroups / 64 of them
__device__ inline void sum_counts_block(const int* __restrict__ counts, int ngroups, int64_t* __restrict__ n_updated,
                                        long long* part, int64_t* __restrict__ total = nullptr) {
    int v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        int i = threadIdx.x + 256 * r;
        v[r] = i < ngroups ? counts[i] : 0;
    }
    long long t = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) t += v[r];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long sum = part[0] + part[1] + part[2] + part[3];
        *n_updated = sum;
        if (total) *total += sum;
    }
}

}  // namespace prism
