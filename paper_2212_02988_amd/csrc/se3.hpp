// Rotations and pose increments in double precision (device side): skew
// matrices, SO(3) exponential (with its left Jacobian) and logarithm,
// quaternion <-> matrix, the pose error e = (t_a - t_b, Log(R_a R_b^T)) and
// the left, world-frame retraction t <- t + d_t, R <- Exp(d_theta) R.
#pragma once
#include "common.hpp"

namespace prism {

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
        // near pi: axis from the column of (R + I)/2 with the largest diagonal
        double ax0, ax1, ax2;
        if (R[0] >= R[4] && R[0] >= R[8]) {
            ax0 = (R[0] + 1.0) * 0.5; ax1 = R[3] * 0.5; ax2 = R[6] * 0.5;
        } else if (R[4] >= R[8]) {
            ax0 = R[1] * 0.5; ax1 = (R[4] + 1.0) * 0.5; ax2 = R[7] * 0.5;
        } else {
            ax0 = R[2] * 0.5; ax1 = R[5] * 0.5; ax2 = (R[8] + 1.0) * 0.5;
        }
        double n = sqrt(ax0 * ax0 + ax1 * ax1 + ax2 * ax2);
        w[0] = th * ax0 / n;
        w[1] = th * ax1 / n;
        w[2] = th * ax2 / n;
        return;
    }
    double f = th / (2.0 * sin(th));
    for (int i = 0; i < 3; ++i) w[i] = f * v[i];
}

// unit-quaternion rotation for the pose algebra (one reciprocal)
__device__ inline void quat_to_R9(const double q[4], double R[9]) {
    double in = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] * in, x = q[1] * in, y = q[2] * in, z = q[3] * in;
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// rotation matrix -> unit quaternion (w >= 0), branch on the largest of
// trace and diagonal (constant indices only, so nothing leaves registers)
__device__ inline void R9_to_quat(const double R[9], double q[4]) {
    double tr = R[0] + R[4] + R[8];
    if (tr > 0.0) {
        double s = 2.0 * sqrt(tr + 1.0), is = 1.0 / s;
        q[0] = 0.25 * s;
        q[1] = (R[7] - R[5]) * is;
        q[2] = (R[2] - R[6]) * is;
        q[3] = (R[3] - R[1]) * is;
    } else if (R[0] >= R[4] && R[0] >= R[8]) {
        double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]), is = 1.0 / s;
        q[0] = (R[7] - R[5]) * is;
        q[1] = 0.25 * s;
        q[2] = (R[1] + R[3]) * is;
        q[3] = (R[2] + R[6]) * is;
    } else if (R[4] >= R[8]) {
        double s = 2.0 * sqrt(1.0 + R[4] - R[8] - R[0]), is = 1.0 / s;
        q[0] = (R[2] - R[6]) * is;
        q[1] = (R[1] + R[3]) * is;
        q[2] = 0.25 * s;
        q[3] = (R[5] + R[7]) * is;
    } else {
        double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]), is = 1.0 / s;
        q[0] = (R[3] - R[1]) * is;
        q[1] = (R[2] + R[6]) * is;
        q[2] = (R[5] + R[7]) * is;
        q[3] = 0.25 * s;
    }
    if (q[0] < 0.0) {
        q[0] = -q[0]; q[1] = -q[1]; q[2] = -q[2]; q[3] = -q[3];
    }
    double in = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    q[0] *= in; q[1] *= in; q[2] *= in; q[3] *= in;
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

}  // namespace prism
