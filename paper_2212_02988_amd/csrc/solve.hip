// FP64 state-filter algebra on the device (App. E.1-E.3, Sec. 4.3.2):
// linearised transition + propagation + split into pose prior and velocity
// conditional; Gauss-Newton step of the MAP pose objective; Laplace
// covariance (squared-Jacobian Hessian, with the dynamics prior), its EMA,
// and the product with the velocity conditional; the same over the 15-D
// state with an accelerometer bias; predictive rollouts.
//
// Each kernel is one workgroup per filter (256 threads for the prediction,
// 512 for the Gauss-Newton and Laplace kernels, which first reduce the block
// partial sums of the normal equations in a fixed order): matrix products
// are spread over the threads, and the small Cholesky factorisations run on
// one thread.  Everything stays on the device so a filter step can be
// captured in a HIP graph.
#include "common.hpp"
#include "launch.hpp"
#include "se3.hpp"

namespace prism {

// ---------------------------------------------------------------------------
// small helpers (row-major matrices in LDS)
// ---------------------------------------------------------------------------
// C[r x c] = A[r x k] * op(B);  op(B) = B [k x c] or B^T (B stored [c x k])
__device__ inline void mm(const double* A, const double* B, double* C, int r, int k, int c, bool bT) {
    for (int e = threadIdx.x; e < r * c; e += blockDim.x) {
        int i = e / c, j = e % c;
        double s = 0.0;
        for (int q = 0; q < k; ++q) s += A[i * k + q] * (bT ? B[j * k + q] : B[q * c + j]);
        C[e] = s;
    }
    __syncthreads();
}

__device__ inline void symmetrize(double* A, int n) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        int i = e / n, j = e % n;
        if (i < j) {
            double s = 0.5 * (A[i * n + j] + A[j * n + i]);
            A[i * n + j] = s;
            A[j * n + i] = s;
        }
    }
    __syncthreads();
}

// In-place lower Cholesky of an N x N matrix (single thread); false if not
// positive definite.  Sizes are compile-time constants and every loop is
// unrolled so the matrix stays in registers.
template <int N>
__device__ inline bool chol(double* A) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double s = A[j * N + j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= A[j * N + k] * A[j * N + k];
        ok = ok && (s > 0.0);
        double d = sqrt(fmax(s, 1e-300));
        double id = 1.0 / d;
        A[j * N + j] = d;
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            double t = A[i * N + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= A[i * N + k] * A[j * N + k];
            A[i * N + j] = t * id;
        }
#pragma unroll
        for (int i = 0; i < j; ++i) A[i * N + j] = 0.0;
    }
    return ok;
}

// solve L L^T x = b in place (single thread)
template <int N>
__device__ inline void chol_solve(const double* L, double* b) {
    double id[N];
#pragma unroll
    for (int i = 0; i < N; ++i) id[i] = 1.0 / L[i * N + i];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i * N + k] * b[k];
        b[i] = s * id[i];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < N; ++k) s -= L[k * N + i] * b[k];
        b[i] = s * id[i];
    }
}

// inverse from the Cholesky factor (in LDS), one column per thread (< N)
template <int N>
__device__ inline void chol_inverse(const double* L, double* Ainv) {
    if ((int)threadIdx.x < N) {
        double x[N];
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = (i == (int)threadIdx.x) ? 1.0 : 0.0;
        chol_solve<N>(L, x);
#pragma unroll
        for (int i = 0; i < N; ++i) Ainv[i * N + threadIdx.x] = x[i];
    }
    __syncthreads();
}

// Fixed-order block sum of partial normal equations (nblocks rows of 29
// doubles) into lds_out[29].  The rows are read as one flat array with
// coalesced loads: thread t < 29 G (G = row groups) reads elements t, t + 29 G,
// ... which all belong to column t mod 29, keeping eight independent partial
// sums in flight; the G sums of each column are then added in row-group order.
// (Each thread reading whole rows made every load instruction touch 64 cache
// lines, which one workgroup's vector memory path takes serially.)
// With sg given, the filter state is copied into ls on the way: its words
// are loaded together with the first partials (not one round trip before
// them) and stored to LDS before the sum's barrier.
__device__ inline void sum_partials(const double* __restrict__ partials, int nblocks, double* lds_red,
                                    double* lds_out, const prism_filter_state* __restrict__ sg = nullptr,
                                    prism_filter_state* ls = nullptr) {
    constexpr int kStateWords = (int)(sizeof(prism_filter_state) / 8);
    static_assert(sizeof(prism_filter_state) % 8 == 0 && kStateWords <= 2 * 256, "state copied in two words per thread");
    const int bd = min((int)blockDim.x, kRedLds);
    const int G = bd / PRISM_NEQ, span = G * PRISM_NEQ;
    const int t = threadIdx.x;
    unsigned long long sw0 = 0, sw1 = 0;
    const int t1 = t + (int)blockDim.x;
    if (sg) {
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(sg);
        if (t < kStateWords) sw0 = src[t];
        if (t1 < kStateWords) sw1 = src[t1];
    }
    double acc = 0.0;
    if (t < span) {
        const long long total = (long long)nblocks * PRISM_NEQ;
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        long long e = t;
        for (; e + 7LL * span < total; e += 8LL * span) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = partials[e + u * (long long)span];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += x[u];
        }
        for (; e < total; e += span) a[0] += partials[e];
        acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        lds_red[t] = acc;
    }
    if (ls) {
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(ls);
        if (t < kStateWords) dst[t] = sw0;
        if (t1 < kStateWords) dst[t1] = sw1;
    }
    __syncthreads();
    if (t < PRISM_NEQ) {
        double sum = 0.0;
        for (int r = 0; r < G; ++r) sum += lds_red[r * PRISM_NEQ + t];
        lds_out[t] = sum;
    }
    __syncthreads();
}

__device__ inline void unpack_H(const double* neq, double* H, double* g) {
    int q = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b) {
            H[a * 6 + b] = neq[q];
            H[b * 6 + a] = neq[q];
            ++q;
        }
    for (int a = 0; a < 6; ++a) g[a] = neq[21 + a];
}

// The state lives in global memory; each kernel copies it into LDS once
// (one parallel round trip), works on the copy and writes it back, so the
// single-thread parts never wait on dependent global loads.
__device__ inline void state_in(const prism_filter_state* g, prism_filter_state* l) {
    const unsigned long long* s = reinterpret_cast<const unsigned long long*>(g);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(l);
    for (int i = threadIdx.x; i < (int)(sizeof(prism_filter_state) / 8); i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

__device__ inline void state_out(const prism_filter_state* l, prism_filter_state* g) {
    __syncthreads();
    const unsigned long long* s = reinterpret_cast<const unsigned long long*>(l);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(g);
    for (int i = threadIdx.x; i < (int)(sizeof(prism_filter_state) / 8); i += blockDim.x) d[i] = s[i];
}

// ---------------------------------------------------------------------------
// predict + split
// ---------------------------------------------------------------------------
// Mean of the Euler transition (App. B, E.1) of one state, on one thread:
// new velocities (vnew = v', w' = v + u du, w + u_w du with du = dt, or dt^2
// as printed), E = Exp(w' dt) with its left Jacobian Jl, and the new pose
// (t + v' dt, E R).
__device__ inline void transition_mean_t0(const prism_pose& pose, const double* v0, const double* w0,
                                          const double* u, const TransC& tc, double* vnew, double* E, double* Jl,
                                          prism_pose& pr) {
    double v[3], w[3];
    for (int i = 0; i < 3; ++i) {
        v[i] = v0[i] + u[i] * tc.du;
        w[i] = w0[i] + u[3 + i] * tc.du;
        vnew[i] = v[i];
        vnew[3 + i] = w[i];
    }
    double phi[3] = {w[0] * tc.dt, w[1] * tc.dt, w[2] * tc.dt};
    double Ex[9], Jx[9], R[9], R2[9];
    so3_exp(phi, Ex, Jx);
    for (int e = 0; e < 9; ++e) { E[e] = Ex[e]; Jl[e] = Jx[e]; }
    quat_to_R9(pose.q, R);
    mat3mul(Ex, R, R2);
    for (int i = 0; i < 3; ++i) pr.t[i] = pose.t[i] + v[i] * tc.dt;
    R9_to_quat(R2, pr.q);
}

// Covariance of the linearised transition (App. E.2), whole workgroup:
// T2 = M P M^T + G Q G^T (symmetrised) in the error state (dt, dtheta, dv,
// dw), with E, Jl from transition_mean_t0; P, M, G, T1, T2: LDS [144].
__device__ inline void transition_cov(const double* E, const double* Jl, const TransC& tc, const double* P,
                                      double* M, double* G, double* T1, double* T2) {
    for (int e = threadIdx.x; e < 144; e += blockDim.x) {
        M[e] = 0.0;
        G[e] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) {
            M[i * 12 + i] = 1.0;
            M[i * 12 + 6 + i] = tc.dt;
            M[(6 + i) * 12 + 6 + i] = 1.0;
            M[(9 + i) * 12 + 9 + i] = 1.0;
            G[i * 12 + i] = 1.0;
            G[i * 12 + 6 + i] = tc.dt;
            G[(3 + i) * 12 + 3 + i] = 1.0;
            G[(6 + i) * 12 + 6 + i] = 1.0;
            G[(9 + i) * 12 + 9 + i] = 1.0;
            for (int j = 0; j < 3; ++j) {
                M[(3 + i) * 12 + 3 + j] = E[i * 3 + j];
                M[(3 + i) * 12 + 9 + j] = tc.dt * Jl[i * 3 + j];
                G[(3 + i) * 12 + 9 + j] = tc.dt * Jl[i * 3 + j];
            }
        }
    }
    __syncthreads();
    mm(M, P, T1, 12, 12, 12, false);       // M P
    mm(T1, M, T2, 12, 12, 12, true);       // M P M^T
    // G Q G^T with Q diagonal
    for (int e = threadIdx.x; e < 144; e += blockDim.x) {
        int i = e / 12, j = e % 12;
        double s = 0.0;
        for (int q = 0; q < 12; ++q) s += G[i * 12 + q] * tc.q[q] * G[j * 12 + q];
        T2[e] += s;
    }
    __syncthreads();
    symmetrize(T2, 12);
}

__device__ __forceinline__ void predict_block(prism_filter_state* __restrict__ Sg, const double* __restrict__ u,
                                              const TransC& tc, Rel32* __restrict__ rel) {
    __shared__ double M[144], G[144], T1[144], T2[144], P[144], Spp[36], L[36], Sinv[36];
    __shared__ double vnew[6], E[9], Jl[9];
    __shared__ int ok;
    __shared__ prism_filter_state Ls;
    state_in(Sg, &Ls);
    prism_filter_state* S = &Ls;
    if (threadIdx.x == 0) {
        S->flags = 0;
        for (int i = 0; i < 6; ++i) S->u[i] = u[i];
        prism_pose pr;
        transition_mean_t0(S->pose, S->v, S->w, u, tc, vnew, E, Jl, pr);
        S->prior = pr;
        S->iter = pr;
        if (rel) rel_of(&S->iter, &S->anchor, *rel);
        for (int i = 0; i < 6; ++i) S->vel_prior[i] = vnew[i];
    }
    for (int e = threadIdx.x; e < 144; e += blockDim.x) P[e] = S->P[e];
    __syncthreads();
    transition_cov(E, Jl, tc, P, M, G, T1, T2);
    // split: Spp, D = Svp Spp^-1, Sv = Svv - D Svp^T
    for (int e = threadIdx.x; e < 36; e += blockDim.x) {
        int i = e / 6, j = e % 6;
        Spp[e] = T2[i * 12 + j];
        L[e] = T2[i * 12 + j];
    }
    __syncthreads();
    if (threadIdx.x == 0) ok = chol<6>(L);
    __syncthreads();
    if (!ok) {
        // the predicted pose block is not positive definite: the step keeps
        // the predicted mean and joint covariance, and no pose objective is
        // solved (the Gauss-Newton and Laplace kernels see the flag)
        for (int e = threadIdx.x; e < 144; e += blockDim.x) S->P[e] = T2[e];
        if (threadIdx.x == 0) S->flags |= PRISM_FLAG_CHOL_FALLBACK | PRISM_FLAG_PRIOR_NOT_PD;
        state_out(S, Sg);
        return;
    }
    chol_inverse<6>(L, Sinv);
    symmetrize(Sinv, 6);
    // D = Svp Sinv
    for (int e = threadIdx.x; e < 36; e += blockDim.x) {
        int i = e / 6, j = e % 6;
        double s = 0.0;
        for (int q = 0; q < 6; ++q) s += T2[(6 + i) * 12 + q] * Sinv[q * 6 + j];
        T1[e] = s;   // D
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 36; e += blockDim.x) {
        int i = e / 6, j = e % 6;
        double s = 0.0;
        for (int q = 0; q < 6; ++q) s += T1[i * 6 + q] * T2[(6 + j) * 12 + q];
        P[e] = T2[(6 + i) * 12 + 6 + j] - s;   // Sv (reuse P)
    }
    __syncthreads();
    symmetrize(P, 6);
    for (int e = threadIdx.x; e < 36; e += blockDim.x) {
        S->Lp[e] = Sinv[e];
        S->D[e] = T1[e];
        S->Sv[e] = P[e];
    }
    state_out(S, Sg);
}

// The 15-D state (pose, velocities, accelerometer bias b): the linear
// control u[0..2] is the body-frame specific force f, the acceleration
// a = R (f - b) + g with the state's rotation R; then the mean transition
// above with a as the linear acceleration.  Ra = R (f - b) and R are kept
// for the linearisation.  One thread.
__device__ inline void transition_mean_bias_t0(const prism_pose& pose, const double* v0, const double* w0,
                                               const double* b, const double* u, const TransC& tc, double* vnew,
                                               double* E, double* Jl, double* Ra, double* R0, prism_pose& pr) {
    double R[9];
    quat_to_R9(pose.q, R);
    const double f[3] = {u[0] - b[0], u[1] - b[1], u[2] - b[2]};
    double a[6];
    for (int i = 0; i < 3; ++i) {
        Ra[i] = R[i * 3] * f[0] + R[i * 3 + 1] * f[1] + R[i * 3 + 2] * f[2];
        a[i] = Ra[i] + tc.g[i];
        a[3 + i] = u[3 + i];
    }
    for (int e = 0; e < 9; ++e) R0[e] = R[e];
    transition_mean_t0(pose, v0, w0, a, tc, vnew, E, Jl, pr);
}

// Covariance of the linearised 15-D transition, whole workgroup: the blocks
// of transition_cov plus the acceleration's dependence on the rotation and
// the bias at the start of the step, da = -[R (f - b)]x dtheta - R db,
// entering v' over du and t' through v' dt; the bias is a random walk.
// P, M, G, T1, T2: LDS [225].
__device__ inline void transition_cov_bias(const double* E, const double* Jl, const double* Ra, const double* R0,
                                           const TransC& tc, const double* P, double* M, double* G, double* T1,
                                           double* T2) {
    constexpr int N = 15;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        M[e] = 0.0;
        G[e] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double K[9] = {0.0, -Ra[2], Ra[1], Ra[2], 0.0, -Ra[0], -Ra[1], Ra[0], 0.0};
        for (int i = 0; i < 3; ++i) {
            M[i * N + i] = 1.0;
            M[i * N + 6 + i] = tc.dt;
            M[(6 + i) * N + 6 + i] = 1.0;
            M[(9 + i) * N + 9 + i] = 1.0;
            M[(12 + i) * N + 12 + i] = 1.0;
            G[i * N + i] = 1.0;
            G[i * N + 6 + i] = tc.dt;
            G[(3 + i) * N + 3 + i] = 1.0;
            G[(6 + i) * N + 6 + i] = 1.0;
            G[(9 + i) * N + 9 + i] = 1.0;
            G[(12 + i) * N + 12 + i] = 1.0;
            for (int j = 0; j < 3; ++j) {
                M[(3 + i) * N + 3 + j] = E[i * 3 + j];
                M[(3 + i) * N + 9 + j] = tc.dt * Jl[i * 3 + j];
                G[(3 + i) * N + 9 + j] = tc.dt * Jl[i * 3 + j];
                const double vth = -tc.du * K[i * 3 + j], vb = -tc.du * R0[i * 3 + j];
                M[(6 + i) * N + 3 + j] = vth;
                M[(6 + i) * N + 12 + j] = vb;
                M[i * N + 3 + j] = tc.dt * vth;
                M[i * N + 12 + j] = tc.dt * vb;
            }
        }
    }
    __syncthreads();
    mm(M, P, T1, N, N, N, false);       // M P
    mm(T1, M, T2, N, N, N, true);       // M P M^T
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        int i = e / N, j = e % N;
        double s = 0.0;
        for (int q = 0; q < N; ++q) s += G[i * N + q] * tc.q[q] * G[j * N + q];
        T2[e] += s;
    }
    __syncthreads();
    symmetrize(T2, N);
}

// predict + split of the 15-D state: the pose prior as for the 12-D state,
// the 9-D conditional of (v, w, b) given the pose into X
__device__ __forceinline__ void predict_block_bias(prism_filter_state* __restrict__ Sg,
                                                   prism_filter_bias_state* __restrict__ X,
                                                   const double* __restrict__ u, const TransC& tc,
                                                   Rel32* __restrict__ rel) {
    constexpr int N = 15, NR = 9;
    __shared__ double M[N * N], G[N * N], T1[N * N], T2[N * N], P[N * N], L[36], Sinv[36];
    __shared__ double vnew[6], E[9], Jl[9], Ra[3], R0[9], b[3];
    __shared__ int ok;
    __shared__ prism_filter_state Ls;
    state_in(Sg, &Ls);
    prism_filter_state* S = &Ls;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) P[e] = X->P[e];
    if (threadIdx.x < 3) b[threadIdx.x] = X->b[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        S->flags = 0;
        for (int i = 0; i < 6; ++i) S->u[i] = u[i];
        prism_pose pr;
        transition_mean_bias_t0(S->pose, S->v, S->w, b, u, tc, vnew, E, Jl, Ra, R0, pr);
        S->prior = pr;
        S->iter = pr;
        if (rel) rel_of(&S->iter, &S->anchor, *rel);
        for (int i = 0; i < 6; ++i) S->vel_prior[i] = vnew[i];
    }
    __syncthreads();
    transition_cov_bias(E, Jl, Ra, R0, tc, P, M, G, T1, T2);
    for (int e = threadIdx.x; e < 36; e += blockDim.x) L[e] = T2[(e / 6) * N + e % 6];
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) X->P[e] = T2[e];
    for (int e = threadIdx.x; e < 144; e += blockDim.x) S->P[e] = T2[(e / 12) * N + e % 12];
    if (threadIdx.x < 6) X->rest_prior[threadIdx.x] = vnew[threadIdx.x];
    else if (threadIdx.x < NR) X->rest_prior[threadIdx.x] = b[threadIdx.x - 6];
    __syncthreads();
    if (threadIdx.x == 0) ok = chol<6>(L);
    __syncthreads();
    if (!ok) {
        // no MAP problem: the step keeps the predicted mean and covariance
        if (threadIdx.x == 0) S->flags |= PRISM_FLAG_CHOL_FALLBACK | PRISM_FLAG_PRIOR_NOT_PD;
        state_out(S, Sg);
        return;
    }
    chol_inverse<6>(L, Sinv);
    symmetrize(Sinv, 6);
    // D = P_rp Sinv [9 x 6], Sv = P_rr - D P_rp^T [9 x 9]
    for (int e = threadIdx.x; e < NR * 6; e += blockDim.x) {
        int i = e / 6, j = e % 6;
        double s = 0.0;
        for (int q = 0; q < 6; ++q) s += T2[(6 + i) * N + q] * Sinv[q * 6 + j];
        T1[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NR * NR; e += blockDim.x) {
        int i = e / NR, j = e % NR;
        double s = 0.0;
        for (int q = 0; q < 6; ++q) s += T1[i * 6 + q] * T2[(6 + j) * N + q];
        P[e] = T2[(6 + i) * N + 6 + j] - s;
    }
    __syncthreads();
    symmetrize(P, NR);
    for (int e = threadIdx.x; e < 36; e += blockDim.x) S->Lp[e] = Sinv[e];
    for (int e = threadIdx.x; e < NR * 6; e += blockDim.x) X->D[e] = T1[e];
    for (int e = threadIdx.x; e < NR * NR; e += blockDim.x) X->Sv[e] = P[e];
    state_out(S, Sg);
}

__global__ __launch_bounds__(256) void k_predict(prism_filter_state* __restrict__ Sg,
                                                 prism_filter_bias_state* __restrict__ X,
                                                 const double* __restrict__ u, TransC tc, Rel32* __restrict__ rel) {
    if (X)
        predict_block_bias(Sg, X, u, tc, rel);
    else
        predict_block(Sg, u, tc, rel);
}

// ---------------------------------------------------------------------------
// one Gauss-Newton step of the MAP pose objective
// ---------------------------------------------------------------------------
// thread 0: one Gauss-Newton step on the state copy
__device__ inline void gn_step_body(prism_filter_state* S, const double* neq) {
    if (S->flags & PRISM_FLAG_CHOL_FALLBACK) return;
    if (!(neq[28] > 0.0)) S->flags |= PRISM_FLAG_NO_VALID_PIXELS;
    double H[36], g[6], A[36], b[6], e[6];
    unpack_H(neq, H, g);
    prism_pose it = S->iter, pr = S->prior;
    pose_err(it, pr, e);
    for (int i = 0; i < 6; ++i) {
        double le = 0.0;
        for (int j = 0; j < 6; ++j) {
            A[i * 6 + j] = 2.0 * H[i * 6 + j] + S->Lp[i * 6 + j];
            le += S->Lp[i * 6 + j] * e[j];
        }
        b[i] = -(2.0 * g[i] + le);
    }
    if (!chol<6>(A)) {
        S->flags |= PRISM_FLAG_CHOL_FALLBACK;
        S->iter = pr;
        return;
    }
    chol_solve<6>(A, b);
    retract(it, b);
    S->iter = it;
}

__device__ __forceinline__ void gn_step_block(prism_filter_state* __restrict__ Sg,
                                              const double* __restrict__ partials, int nblocks,
                                              Rel32* __restrict__ rel) {
    __shared__ double red[kRedLds], neq[PRISM_NEQ];
    __shared__ prism_filter_state Ls;
    sum_partials(partials, nblocks, red, neq, Sg, &Ls);
    if (threadIdx.x == 0) gn_step_body(&Ls, neq);
    __syncthreads();
    if (threadIdx.x == 0) {
        Sg->iter = Ls.iter;
        Sg->flags = Ls.flags;
        if (rel) rel_of(&Ls.iter, &Ls.anchor, *rel);
    }
}

__global__ __launch_bounds__(512) void k_gn_step(prism_filter_state* __restrict__ Sg,
                                                 const double* __restrict__ partials, int nblocks,
                                                 Rel32* __restrict__ rel) {
    gn_step_block(Sg, partials, nblocks, rel);
}

// ---------------------------------------------------------------------------
// Laplace covariance, EMA, product with the velocity conditional
// ---------------------------------------------------------------------------
// The product with the 9-D conditional of (v, w, b) of the 15-D state:
// joint covariance [[Sb, Sb D^T], [D Sb, Sv + D Sb D^T]] over 15 dimensions,
// means rest_prior + D e; the leading 12x12 block also into S->P.
__device__ inline void combine_bias(prism_filter_state* S, prism_filter_bias_state* __restrict__ X,
                                    const double* Sb, const double* e) {
    constexpr int N = 15, NR = 9;
    __shared__ double D9[NR * 6], T9[NR * 6], P15[N * N];
    for (int i = threadIdx.x; i < NR * 6; i += blockDim.x) D9[i] = X->D[i];
    __syncthreads();
    mm(D9, Sb, T9, NR, 6, 6, false);   // D Sb
    for (int e2 = threadIdx.x; e2 < N * N; e2 += blockDim.x) {
        int i = e2 / N, j = e2 % N;
        double s;
        if (i < 6 && j < 6) s = Sb[i * 6 + j];
        else if (i < 6) s = T9[(j - 6) * 6 + i];
        else if (j < 6) s = T9[(i - 6) * 6 + j];
        else {
            s = X->Sv[(i - 6) * NR + (j - 6)];
            for (int q = 0; q < 6; ++q) s += T9[(i - 6) * 6 + q] * D9[(j - 6) * 6 + q];
        }
        P15[e2] = s;
    }
    __syncthreads();
    symmetrize(P15, N);
    for (int e2 = threadIdx.x; e2 < N * N; e2 += blockDim.x) X->P[e2] = P15[e2];
    for (int e2 = threadIdx.x; e2 < 144; e2 += blockDim.x) S->P[e2] = P15[(e2 / 12) * N + e2 % 12];
    if (threadIdx.x == 0) {
        double vm[NR];
        for (int i = 0; i < NR; ++i) {
            vm[i] = X->rest_prior[i];
            for (int j = 0; j < 6; ++j) vm[i] += D9[i * 6 + j] * e[j];
        }
        for (int i = 0; i < 3; ++i) {
            S->v[i] = vm[i];
            S->w[i] = vm[3 + i];
            X->b[i] = vm[6 + i];
        }
    }
}

__device__ __forceinline__ void laplace_combine_block(prism_filter_state* __restrict__ Sg,
                                                      prism_filter_bias_state* __restrict__ X,
                                                      const double* __restrict__ partials, int nblocks, double ema,
                                                      double min_inliers, double lap_h) {
    __shared__ double red[kRedLds], neq[PRISM_NEQ];
    __shared__ double A[36], Sl[36], Sb[36], D[36], T[36], P[144], e[6];
    __shared__ int ok;
    __shared__ prism_filter_state Ls;
    prism_filter_state* S = &Ls;
    sum_partials(partials, nblocks, red, neq, Sg, &Ls);
    if (threadIdx.x < PRISM_NEQ) S->neq[threadIdx.x] = neq[threadIdx.x];
    if (S->flags & PRISM_FLAG_PRIOR_NOT_PD) {
        // predicted mean and covariance as they are (the covariance was
        // written by the predict kernel); the Laplace EMA is left unchanged
        if (threadIdx.x == 0) {
            if (!(neq[28] > 0.0)) S->flags |= PRISM_FLAG_NO_VALID_PIXELS;
            if (neq[28] < min_inliers) S->flags |= PRISM_FLAG_LOW_INLIERS;
            for (int i = 0; i < 3; ++i) { S->v[i] = S->vel_prior[i]; S->w[i] = S->vel_prior[3 + i]; }
            if (X)
                for (int i = 0; i < 3; ++i) X->b[i] = X->rest_prior[6 + i];
            S->iter = S->prior;
            S->pose = S->prior;
            S->anchor = S->prior;
            S->step += 1;
        }
        state_out(S, Sg);
        return;
    }
    if (threadIdx.x == 0) {
        if (!(neq[28] > 0.0)) S->flags |= PRISM_FLAG_NO_VALID_PIXELS;
        // fewer contributing pixels at the final iterate than the filter asks for
        if (neq[28] < min_inliers) S->flags |= PRISM_FLAG_LOW_INLIERS;
        double H[36], g[6];
        unpack_H(neq, H, g);
        // Laplace precision lap_h H + Lp (Sec. 5.1 prints lap_h = 2)
        for (int i = 0; i < 36; ++i) A[i] = lap_h * H[i] + S->Lp[i];
        ok = !(S->flags & PRISM_FLAG_CHOL_FALLBACK) && chol<6>(A);
        if (!ok) {
            S->flags |= PRISM_FLAG_CHOL_FALLBACK;
            S->iter = S->prior;
        }
    }
    __syncthreads();
    if (ok) {
        chol_inverse<6>(A, Sl);
    } else {
        // prior pose covariance = Lp^-1
        if (threadIdx.x == 0) {
            for (int i = 0; i < 36; ++i) T[i] = S->Lp[i];
            chol<6>(T);
        }
        __syncthreads();
        chol_inverse<6>(T, Sl);
    }
    symmetrize(Sl, 6);
    if (threadIdx.x < 36) {
        int i = threadIdx.x;
        S->S_lap[i] = Sl[i];
        Sb[i] = S->has_sbar ? ema * S->Sbar[i] + (1.0 - ema) * Sl[i] : Sl[i];
        D[i] = S->D[i];
    }
    if (threadIdx.x == 0) pose_err(S->iter, S->prior, e);
    __syncthreads();
    if (X) {
        combine_bias(S, X, Sb, e);
        if (threadIdx.x < 36) S->Sbar[threadIdx.x] = Sb[threadIdx.x];
        if (threadIdx.x == 0) {
            S->has_sbar = 1;
            S->pose = S->iter;
            S->anchor = S->iter;
            S->step += 1;
        }
        state_out(S, Sg);
        return;
    }
    // joint covariance [[Sb, Sb D^T], [D Sb, Sv + D Sb D^T]]
    mm(D, Sb, T, 6, 6, 6, false);   // D Sb
    for (int e2 = threadIdx.x; e2 < 144; e2 += blockDim.x) {
        int i = e2 / 12, j = e2 % 12;
        double s;
        if (i < 6 && j < 6) s = Sb[i * 6 + j];
        else if (i < 6) s = T[(j - 6) * 6 + i];           // (D Sb)^T = Sb D^T
        else if (j < 6) s = T[(i - 6) * 6 + j];
        else {
            s = S->Sv[(i - 6) * 6 + (j - 6)];
            for (int q = 0; q < 6; ++q) s += T[(i - 6) * 6 + q] * D[(j - 6) * 6 + q];
        }
        P[e2] = s;
    }
    __syncthreads();
    symmetrize(P, 12);
    for (int e2 = threadIdx.x; e2 < 144; e2 += blockDim.x) S->P[e2] = P[e2];
    if (threadIdx.x < 36) S->Sbar[threadIdx.x] = Sb[threadIdx.x];
    if (threadIdx.x == 0) {
        S->has_sbar = 1;
        double vm[6];
        for (int i = 0; i < 6; ++i) {
            vm[i] = S->vel_prior[i];
            for (int j = 0; j < 6; ++j) vm[i] += D[i * 6 + j] * e[j];
        }
        for (int i = 0; i < 3; ++i) { S->v[i] = vm[i]; S->w[i] = vm[3 + i]; }
        S->pose = S->iter;
        S->anchor = S->iter;
        S->step += 1;
    }
    state_out(S, Sg);
}

__global__ __launch_bounds__(512) void k_laplace_combine(prism_filter_state* __restrict__ Sg,
                                                         prism_filter_bias_state* __restrict__ X,
                                                         const double* __restrict__ partials, int nblocks,
                                                         double ema, double min_inliers, double lap_h) {
    laplace_combine_block(Sg, X, partials, nblocks, ema, min_inliers, lap_h);
}

// the left, world-frame retraction of n poses by n tangent increments
__global__ __launch_bounds__(256) void k_pose_retract(const prism_pose* __restrict__ poses,
                                                      const double* __restrict__ delta, int n,
                                                      prism_pose* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    prism_pose p = poses[i];
    double d[6];
    for (int a = 0; a < 6; ++a) d[a] = delta[6 * i + a];
    retract(p, d);
    out[i] = p;
}

__device__ __forceinline__ void first_frame_block(prism_filter_state* __restrict__ S) {
    if (threadIdx.x == 0) {
        S->anchor = S->pose;
        S->step = 1;
        S->flags = 0;
    }
}

__global__ void k_first_frame(prism_filter_state* __restrict__ S) { first_frame_block(S); }

// batched: one workgroup per filter
__global__ __launch_bounds__(256) void k_predict_batch(BatchArgs b) {
    const AgentDesc& D = *b.d[blockIdx.x];
    if (D.X)
        predict_block_bias(D.S, D.X, (const double*)D.slots[b.slot[blockIdx.x]].u, D.tc, D.rel);
    else
        predict_block(D.S, (const double*)D.slots[b.slot[blockIdx.x]].u, D.tc, D.rel);
}

__global__ __launch_bounds__(512) void k_gn_step_batch(BatchArgs b) {
    const AgentDesc& D = *b.d[blockIdx.x];
    gn_step_block(D.S, D.partials, D.obj_blocks, D.rel);
}

__global__ __launch_bounds__(512) void k_laplace_combine_batch(BatchArgs b) {
    const AgentDesc& D = *b.d[blockIdx.x];
    laplace_combine_block(D.S, D.X, D.partials, D.obj_blocks, D.ema, D.min_inliers, D.lap_h);
}

__global__ __launch_bounds__(64) void k_first_frame_batch(BatchArgs b) { first_frame_block(b.d[blockIdx.x]->S); }

// ---------------------------------------------------------------------------
// predictive rollouts from the state belief
// ---------------------------------------------------------------------------
// One workgroup per sample; its first thread draws the start state from the
// belief, x0 = x (+) L z0 with P = L L^T (tangent order t, theta, v, w; the
// pose part is the left retraction), then runs the generative transition
// with process noise n = sqrt(Q) z_j for each of the k controls:
//   v' = v + u_v du + n_v,  w' = w + u_w du + n_w,
//   t' = t + v' dt + n_t,   R' = Exp(n_theta) Exp(w' dt) R
// (du = dt, or dt^2 in the printed form).  The 15-D state (X non-NULL)
// draws 15 components per row (the bias last), takes the acceleration
// R (u_v - b) + g with the draw's rotation and bias, and walks the bias by
// n_b.  If P is not positive definite every sample starts at the mean and
// *flags gets PRISM_FLAG_CHOL_FALLBACK (else 0; written by the first
// workgroup).
__global__ __launch_bounds__(64) void k_rollout_sample(const prism_filter_state* __restrict__ S,
                                                       const prism_filter_bias_state* __restrict__ X,
                                                       const double* __restrict__ u, int k,
                                                       const double* __restrict__ noise, TransC tc,
                                                       prism_pose* __restrict__ poses, int32_t* __restrict__ flags) {
    __shared__ double A[225];
    __shared__ int ok;
    const int N = X ? 15 : 12;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) A[e] = X ? X->P[e] : S->P[e];
    __syncthreads();
    if (threadIdx.x == 0) ok = X ? chol<15>(A) : chol<12>(A);
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (blockIdx.x == 0 && flags) *flags = ok ? 0 : PRISM_FLAG_CHOL_FALLBACK;
    const double* z = noise + (long long)blockIdx.x * (k + 1) * N;
    double e[15];
    for (int i = 0; i < N; ++i) {
        double acc = 0.0;
        if (ok)
            for (int j = 0; j <= i; ++j) acc += A[i * N + j] * z[j];
        e[i] = acc;
    }
    prism_pose x = S->pose;
    retract(x, e);
    double v[3], w[3], b[3], sq[15];
    for (int i = 0; i < 3; ++i) {
        v[i] = S->v[i] + e[6 + i];
        w[i] = S->w[i] + e[9 + i];
        b[i] = X ? X->b[i] + e[12 + i] : 0.0;
    }
    for (int i = 0; i < N; ++i) sq[i] = sqrt(tc.q[i]);
    for (int j = 0; j < k; ++j) {
        const double* zj = z + (j + 1) * N;
        const double* uj = u + 6 * j;
        double n[15];
        for (int i = 0; i < N; ++i) n[i] = sq[i] * zj[i];
        if (X) {
            double R[9];
            quat_to_R9(x.q, R);
            const double f[3] = {uj[0] - b[0], uj[1] - b[1], uj[2] - b[2]};
            for (int i = 0; i < 3; ++i) {
                const double a = R[i * 3] * f[0] + R[i * 3 + 1] * f[1] + R[i * 3 + 2] * f[2] + tc.g[i];
                v[i] = v[i] + a * tc.du + n[6 + i];
                w[i] = w[i] + uj[3 + i] * tc.du + n[9 + i];
            }
            for (int i = 0; i < 3; ++i) b[i] += n[12 + i];
        } else {
            for (int i = 0; i < 3; ++i) {
                v[i] = v[i] + uj[i] * tc.du + n[6 + i];
                w[i] = w[i] + uj[3 + i] * tc.du + n[9 + i];
            }
        }
        double phi[3] = {w[0] * tc.dt, w[1] * tc.dt, w[2] * tc.dt};
        double E1[9], E2[9], R[9], T[9], R2[9];
        so3_exp(n + 3, E1, nullptr);
        so3_exp(phi, E2, nullptr);
        quat_to_R9(x.q, R);
        mat3mul(E2, R, T);
        mat3mul(E1, T, R2);
        for (int i = 0; i < 3; ++i) x.t[i] = x.t[i] + v[i] * tc.dt + n[i];
        R9_to_quat(R2, x.q);
        poses[(long long)blockIdx.x * k + j] = x;
    }
}

// Closed-form (linearised) prediction of the belief over the k controls:
// mean[j] = (t, q, v, w) after control j (13 doubles), cov[j] = its 12x12
// covariance; the same propagation as the filter's prediction step.
__global__ __launch_bounds__(256) void k_rollout_moments(const prism_filter_state* __restrict__ S,
                                                         const double* __restrict__ u, int k, TransC tc,
                                                         double* __restrict__ mean, double* __restrict__ cov) {
    __shared__ double M[144], G[144], T1[144], T2[144], P[144];
    __shared__ double vnew[6], E[9], Jl[9], v[3], w[3];
    __shared__ prism_pose pose;
    if (threadIdx.x == 0) {
        pose = S->pose;
        for (int i = 0; i < 3; ++i) {
            v[i] = S->v[i];
            w[i] = S->w[i];
        }
    }
    for (int e = threadIdx.x; e < 144; e += blockDim.x) P[e] = S->P[e];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) {
            prism_pose pr;
            transition_mean_t0(pose, v, w, u + 6 * j, tc, vnew, E, Jl, pr);
            pose = pr;
            for (int i = 0; i < 3; ++i) {
                v[i] = vnew[i];
                w[i] = vnew[3 + i];
            }
            if (mean) {
                double* m = mean + 13 * j;
                for (int i = 0; i < 3; ++i) m[i] = pr.t[i];
                for (int i = 0; i < 4; ++i) m[3 + i] = pr.q[i];
                for (int i = 0; i < 6; ++i) m[7 + i] = vnew[i];
            }
        }
        __syncthreads();
        transition_cov(E, Jl, tc, P, M, G, T1, T2);
        for (int e = threadIdx.x; e < 144; e += blockDim.x) {
            P[e] = T2[e];
            if (cov) cov[144 * j + e] = T2[e];
        }
        __syncthreads();
    }
}

// The same for the 15-D state: mean[j] = (t, q, v, w, b) (16 doubles),
// cov[j] its 15x15 covariance.
__global__ __launch_bounds__(256) void k_rollout_moments_bias(const prism_filter_state* __restrict__ S,
                                                              const prism_filter_bias_state* __restrict__ X,
                                                              const double* __restrict__ u, int k, TransC tc,
                                                              double* __restrict__ mean, double* __restrict__ cov) {
    constexpr int N = 15;
    __shared__ double M[N * N], G[N * N], T1[N * N], T2[N * N], P[N * N];
    __shared__ double vnew[6], E[9], Jl[9], Ra[3], R0[9], v[3], w[3], b[3];
    __shared__ prism_pose pose;
    if (threadIdx.x == 0) {
        pose = S->pose;
        for (int i = 0; i < 3; ++i) {
            v[i] = S->v[i];
            w[i] = S->w[i];
            b[i] = X->b[i];
        }
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) P[e] = X->P[e];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) {
            prism_pose pr;
            transition_mean_bias_t0(pose, v, w, b, u + 6 * j, tc, vnew, E, Jl, Ra, R0, pr);
            pose = pr;
            for (int i = 0; i < 3; ++i) {
                v[i] = vnew[i];
                w[i] = vnew[3 + i];
            }
            if (mean) {
                double* m = mean + 16 * j;
                for (int i = 0; i < 3; ++i) m[i] = pr.t[i];
                for (int i = 0; i < 4; ++i) m[3 + i] = pr.q[i];
                for (int i = 0; i < 6; ++i) m[7 + i] = vnew[i];
                for (int i = 0; i < 3; ++i) m[13 + i] = b[i];
            }
        }
        __syncthreads();
        transition_cov_bias(E, Jl, Ra, R0, tc, P, M, G, T1, T2);
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            P[e] = T2[e];
            if (cov) cov[N * N * j + e] = T2[e];
        }
        __syncthreads();
    }
}

hipError_t launch_rollout(const prism_filter_state* S, const prism_filter_bias_state* X, const double* u, int k,
                          int n_samples, const double* noise, const TransC& tc, prism_pose* poses, double* mean,
                          double* cov, int32_t* flags, hipStream_t st) {
    if (mean || cov) {
        if (X)
            k_rollout_moments_bias<<<1, 256, 0, st>>>(S, X, u, k, tc, mean, cov);
        else
            k_rollout_moments<<<1, 256, 0, st>>>(S, u, k, tc, mean, cov);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_samples > 0) {
        k_rollout_sample<<<n_samples, 64, 0, st>>>(S, X, u, k, noise, tc, poses, flags);
        return hipGetLastError();
    }
    return hipSuccess;
}

// per-frame fixed-order sum of block partials; the first nvals values of
// each frame go to out[frame * stride + q]
__global__ __launch_bounds__(512) void k_finalize(const double* __restrict__ partials, int nblocks, int nvals,
                                                  double* __restrict__ out, int stride) {
    __shared__ double red[kRedLds], neq[PRISM_NEQ];
    sum_partials(partials + (long long)blockIdx.x * nblocks * PRISM_NEQ, nblocks, red, neq);
    if ((int)threadIdx.x < nvals) out[(long long)blockIdx.x * stride + threadIdx.x] = neq[threadIdx.x];
}

hipError_t launch_predict(prism_filter_state* S, prism_filter_bias_state* X, const double* u, const TransC& tc,
                          Rel32* rel, hipStream_t st) {
    k_predict<<<1, 256, 0, st>>>(S, X, u, tc, rel);
    return hipGetLastError();
}

hipError_t launch_gn_step(prism_filter_state* S, const double* partials, int nblocks, Rel32* rel,
                          hipStream_t st) {
    k_gn_step<<<1, 512, 0, st>>>(S, partials, nblocks, rel);
    return hipGetLastError();
}

hipError_t launch_laplace_combine(prism_filter_state* S, prism_filter_bias_state* X, const double* partials,
                                  int nblocks, double ema, double min_inliers, double lap_h, hipStream_t st) {
    k_laplace_combine<<<1, 512, 0, st>>>(S, X, partials, nblocks, ema, min_inliers, lap_h);
    return hipGetLastError();
}

hipError_t launch_pose_retract(const prism_pose* poses, const double* delta, int n, prism_pose* out, hipStream_t st) {
    k_pose_retract<<<(n + 255) / 256, 256, 0, st>>>(poses, delta, n, out);
    return hipGetLastError();
}

hipError_t launch_first_frame(prism_filter_state* S, hipStream_t st) {
    k_first_frame<<<1, 1, 0, st>>>(S);
    return hipGetLastError();
}

hipError_t launch_predict_batch(const BatchArgs& b, hipStream_t st) {
    k_predict_batch<<<b.n, 256, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_gn_step_batch(const BatchArgs& b, hipStream_t st) {
    k_gn_step_batch<<<b.n, 512, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_laplace_combine_batch(const BatchArgs& b, hipStream_t st) {
    k_laplace_combine_batch<<<b.n, 512, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_first_frame_batch(const BatchArgs& b, hipStream_t st) {
    k_first_frame_batch<<<b.n, 64, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblocks, int n_frames, int nvals, double* out,
                           int stride, hipStream_t st) {
    k_finalize<<<n_frames, 512, 0, st>>>(partials, nblocks, nvals, out, stride);
    return hipGetLastError();
}

}  // namespace prism
