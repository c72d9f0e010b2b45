// FP64 state-filter algebra on the device (App. E.1-E.3, Sec. 3.3.2):
// linearised transition + propagation + split into pose prior and velocity
// conditional; Gauss-Newton step of the MAP pose objective; Laplace
// covariance (squared-Jacobian Hessian, with the dynamics prior), its EMA,
// and the product with the velocity conditional.
//
// Each kernel is one workgroup of 256 threads per filter: the block partial
// sums of the normal equations are reduced in a fixed order, matrix products
// are spread over the threads, and the 6x6 Cholesky factorisations run on
// one thread.  Everything stays on the device so a filter step can be
// captured in a HIP graph.
#include "common.hpp"
#include "launch.hpp"

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

// in-place lower Cholesky of n x n (single thread); false if not PD
__device__ inline bool chol(double* A, int n) {
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return false;
        double d = sqrt(s);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / d;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return true;
}

// solve L L^T x = b in place (single thread)
__device__ inline void chol_solve(const double* L, double* b, int n) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

// inverse from the Cholesky factor, columns in parallel (threads < n)
__device__ inline void chol_inverse(const double* L, double* Ainv, int n) {
    if ((int)threadIdx.x < n) {
        double x[12];
        for (int i = 0; i < n; ++i) x[i] = (i == (int)threadIdx.x) ? 1.0 : 0.0;
        chol_solve(L, x, n);
        for (int i = 0; i < n; ++i) Ainv[i * n + threadIdx.x] = x[i];
    }
    __syncthreads();
}

__device__ inline void skew(const double v[3], double K[9]) {
    K[0] = 0.0;   K[1] = -v[2]; K[2] = v[1];
    K[3] = v[2];  K[4] = 0.0;   K[5] = -v[0];
    K[6] = -v[1]; K[7] = v[0];  K[8] = 0.0;
}

__device__ inline void mat3mul(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}

// Exp(phi) (Rodrigues) and the left Jacobian J_l(phi)
__device__ inline void so3_exp(const double phi[3], double R[9], double* Jl) {
    double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double th = sqrt(th2);
    double K[9], K2[9];
    skew(phi, K);
    mat3mul(K, K, K2);
    double a, b, c2, c3;
    if (th < 1e-6) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
        c2 = 0.5 - th2 / 24.0;
        c3 = 1.0 / 6.0 - th2 / 120.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
        c2 = b;
        c3 = (th - sin(th)) / (th2 * th);
    }
    for (int e = 0; e < 9; ++e) {
        double I = (e % 4 == 0) ? 1.0 : 0.0;
        R[e] = I + a * K[e] + b * K2[e];
        if (Jl) Jl[e] = I + c2 * K[e] + c3 * K2[e];
    }
}

__device__ inline void so3_log(const double R[9], double w[3]) {
    double c = (R[0] + R[4] + R[8] - 1.0) * 0.5;
    c = fmin(1.0, fmax(-1.0, c));
    double th = acos(c);
    double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    if (th < 1e-8) {
        for (int i = 0; i < 3; ++i) w[i] = 0.5 * v[i];
        return;
    }
    if (M_PI - th < 1e-6) {
        int k = (R[0] >= R[4] && R[0] >= R[8]) ? 0 : (R[4] >= R[8] ? 1 : 2);
        double ax[3];
        for (int i = 0; i < 3; ++i) ax[i] = (R[i * 3 + k] + (i == k ? 1.0 : 0.0)) * 0.5;
        double n = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
        for (int i = 0; i < 3; ++i) w[i] = th * ax[i] / n;
        return;
    }
    double f = th / (2.0 * sin(th));
    for (int i = 0; i < 3; ++i) w[i] = f * v[i];
}

__device__ inline void quat_to_R9(const double q[4], double R[9]) {
    prism_pose p;
    for (int i = 0; i < 4; ++i) p.q[i] = q[i];
    double M[3][3];
    quat_to_rot64(p, M);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i * 3 + j] = M[i][j];
}

// rotation matrix -> unit quaternion (w >= 0), largest-diagonal branch
__device__ inline void R9_to_quat(const double R[9], double q[4]) {
    double tr = R[0] + R[4] + R[8];
    if (tr > 0.0) {
        double s = 2.0 * sqrt(tr + 1.0);
        q[0] = 0.25 * s;
        q[1] = (R[7] - R[5]) / s;
        q[2] = (R[2] - R[6]) / s;
        q[3] = (R[3] - R[1]) / s;
    } else {
        int i = (R[0] >= R[4] && R[0] >= R[8]) ? 0 : (R[4] >= R[8] ? 1 : 2);
        int j = (i + 1) % 3, k = (i + 2) % 3;
        double s = 2.0 * sqrt(1.0 + R[i * 4] - R[j * 4] - R[k * 4]);
        q[0] = (R[k * 3 + j] - R[j * 3 + k]) / s;
        q[1 + i] = 0.25 * s;
        q[1 + j] = (R[j * 3 + i] + R[i * 3 + j]) / s;
        q[1 + k] = (R[k * 3 + i] + R[i * 3 + k]) / s;
    }
    if (q[0] < 0.0)
        for (int a = 0; a < 4; ++a) q[a] = -q[a];
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; ++a) q[a] /= n;
}

// tangent of pose a relative to pose b: (t_a - t_b, Log(R_a R_b^T))
__device__ inline void pose_err(const prism_pose& a, const prism_pose& b, double e[6]) {
    double Ra[9], Rb[9], M[9];
    quat_to_R9(a.q, Ra);
    quat_to_R9(b.q, Rb);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[i * 3 + j] = Ra[i * 3] * Rb[j * 3] + Ra[i * 3 + 1] * Rb[j * 3 + 1] + Ra[i * 3 + 2] * Rb[j * 3 + 2];
    for (int i = 0; i < 3; ++i) e[i] = a.t[i] - b.t[i];
    so3_log(M, e + 3);
}

// t <- t + dt, R <- Exp(dtheta) R
__device__ inline void retract(prism_pose& p, const double d[6]) {
    double E[9], R[9], R2[9];
    so3_exp(d + 3, E, nullptr);
    quat_to_R9(p.q, R);
    mat3mul(E, R, R2);
    for (int i = 0; i < 3; ++i) p.t[i] += d[i];
    R9_to_quat(R2, p.q);
}

// fixed-order block sum of partial normal equations into lds_out[29]
__device__ inline void sum_partials(const double* __restrict__ partials, int nblocks, double* lds_red,
                                    double* lds_out) {
    double acc[PRISM_NEQ];
#pragma unroll
    for (int q = 0; q < PRISM_NEQ; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < PRISM_NEQ; ++q) acc[q] += partials[(long long)b * PRISM_NEQ + q];
    block_reduce29(acc, lds_red, lds_out);
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

// ---------------------------------------------------------------------------
// predict + split
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_predict(prism_filter_state* __restrict__ S,
                                                 const double* __restrict__ u, TransC tc) {
    __shared__ double M[144], G[144], T1[144], T2[144], P[144], Spp[36], L[36], Sinv[36];
    __shared__ double vnew[6], E[9], Jl[9];
    __shared__ int ok;
    if (threadIdx.x == 0) {
        S->flags = 0;
        for (int i = 0; i < 6; ++i) S->u[i] = u[i];
        double v[3], w[3];
        for (int i = 0; i < 3; ++i) {
            v[i] = S->v[i] + u[i] * tc.dt;
            w[i] = S->w[i] + u[3 + i] * tc.dt;
            vnew[i] = v[i];
            vnew[3 + i] = w[i];
        }
        double phi[3] = {w[0] * tc.dt, w[1] * tc.dt, w[2] * tc.dt};
        double Ex[9], Jx[9], R[9], R2[9];
        so3_exp(phi, Ex, Jx);
        for (int e = 0; e < 9; ++e) { E[e] = Ex[e]; Jl[e] = Jx[e]; }
        quat_to_R9(S->pose.q, R);
        mat3mul(Ex, R, R2);
        prism_pose pr;
        for (int i = 0; i < 3; ++i) pr.t[i] = S->pose.t[i] + v[i] * tc.dt;
        R9_to_quat(R2, pr.q);
        S->prior = pr;
        S->iter = pr;
        for (int i = 0; i < 6; ++i) S->vel_prior[i] = vnew[i];
    }
    for (int e = threadIdx.x; e < 144; e += blockDim.x) {
        P[e] = S->P[e];
        M[e] = 0.0;
        G[e] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // error-state transition: rows/cols (dt, dtheta, dv, dw)
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
    // split: Spp, D = Svp Spp^-1, Sv = Svv - D Svp^T
    for (int e = threadIdx.x; e < 36; e += blockDim.x) {
        int i = e / 6, j = e % 6;
        Spp[e] = T2[i * 12 + j];
        L[e] = T2[i * 12 + j];
    }
    __syncthreads();
    if (threadIdx.x == 0) ok = chol(L, 6);
    __syncthreads();
    if (!ok) {
        if (threadIdx.x == 0) S->flags |= PRISM_FLAG_CHOL_FALLBACK;
        return;
    }
    chol_inverse(L, Sinv, 6);
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
}

// ---------------------------------------------------------------------------
// one Gauss-Newton step of the MAP pose objective
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gn_step(prism_filter_state* __restrict__ S,
                                                 const double* __restrict__ partials, int nblocks) {
    __shared__ double red[PRISM_NEQ * 16], neq[PRISM_NEQ];
    sum_partials(partials, nblocks, red, neq);
    if (threadIdx.x != 0) return;
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
    if (!chol(A, 6)) {
        S->flags |= PRISM_FLAG_CHOL_FALLBACK;
        S->iter = pr;
        return;
    }
    chol_solve(A, b, 6);
    retract(it, b);
    S->iter = it;
}

// ---------------------------------------------------------------------------
// Laplace covariance, EMA, product with the velocity conditional
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_laplace_combine(prism_filter_state* __restrict__ S,
                                                         const double* __restrict__ partials, int nblocks,
                                                         double ema) {
    __shared__ double red[PRISM_NEQ * 16], neq[PRISM_NEQ];
    __shared__ double A[36], Sl[36], Sb[36], D[36], T[36], P[144], e[6];
    __shared__ int ok;
    sum_partials(partials, nblocks, red, neq);
    if (threadIdx.x < PRISM_NEQ) S->neq[threadIdx.x] = neq[threadIdx.x];
    if (threadIdx.x == 0) {
        if (!(neq[28] > 0.0)) S->flags |= PRISM_FLAG_NO_VALID_PIXELS;
        double H[36], g[6];
        unpack_H(neq, H, g);
        for (int i = 0; i < 36; ++i) A[i] = 2.0 * H[i] + S->Lp[i];
        ok = !(S->flags & PRISM_FLAG_CHOL_FALLBACK) && chol(A, 6);
        if (!ok) {
            S->flags |= PRISM_FLAG_CHOL_FALLBACK;
            S->iter = S->prior;
        }
    }
    __syncthreads();
    if (ok) {
        chol_inverse(A, Sl, 6);
    } else {
        // prior pose covariance = Lp^-1
        if (threadIdx.x == 0) {
            for (int i = 0; i < 36; ++i) T[i] = S->Lp[i];
            chol(T, 6);
        }
        __syncthreads();
        chol_inverse(T, Sl, 6);
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
}

__global__ void k_first_frame(prism_filter_state* __restrict__ S) {
    S->anchor = S->pose;
    S->step = 1;
    S->flags = 0;
}

// per-frame fixed-order sum of block partials; the first nvals values of
// each frame go to out[frame * stride + q]
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int nblocks, int nvals,
                                                  double* __restrict__ out, int stride) {
    __shared__ double red[PRISM_NEQ * 16], neq[PRISM_NEQ];
    sum_partials(partials + (long long)blockIdx.x * nblocks * PRISM_NEQ, nblocks, red, neq);
    if ((int)threadIdx.x < nvals) out[(long long)blockIdx.x * stride + threadIdx.x] = neq[threadIdx.x];
}

hipError_t launch_predict(prism_filter_state* S, const double* u, const TransC& tc, hipStream_t st) {
    k_predict<<<1, 256, 0, st>>>(S, u, tc);
    return hipGetLastError();
}

hipError_t launch_gn_step(prism_filter_state* S, const double* partials, int nblocks, hipStream_t st) {
    k_gn_step<<<1, 256, 0, st>>>(S, partials, nblocks);
    return hipGetLastError();
}

hipError_t launch_laplace_combine(prism_filter_state* S, const double* partials, int nblocks, double ema,
                                  hipStream_t st) {
    k_laplace_combine<<<1, 256, 0, st>>>(S, partials, nblocks, ema);
    return hipGetLastError();
}

hipError_t launch_first_frame(prism_filter_state* S, hipStream_t st) {
    k_first_frame<<<1, 1, 0, st>>>(S);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblocks, int n_frames, int nvals, double* out,
                           int stride, hipStream_t st) {
    k_finalize<<<n_frames, 256, 0, st>>>(partials, nblocks, nvals, out, stride);
    return hipGetLastError();
}

}  // namespace prism
