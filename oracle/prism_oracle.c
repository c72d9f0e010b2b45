/*
 * FP64 CPU oracle for the PRISM filter hot path (test infrastructure only).
 *
 * This file is the slow, plain reference the GPU library is checked
 * against.  It is NOT part of the product: only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header or constant with the GPU library.
 *
 * Paper: Mirchev et al., "PRISM: Probabilistic Real-Time Inference in
 * Spatial World Models", CoRL 2022 (arXiv 2212.02988).
 *
 *   render            App. B, ray-marching emission and depth-interpolation eq.
 *   render_jacobian   derivative of that emission w.r.t. a 6-DoF pose
 *                     perturbation, reduced to normal equations (Sec. 4.3.2
 *                     MAP objective; App. G Laplace / gating parameters)
 *   track_p2          App. E.3, point-to-plane + photometric surrogate
 *                     against the previous rendered frame
 *   normals           App. E.3, normal of the rendered depth image
 *   map_update        App. D, per-voxel Gaussian product in precision form;
 *                     App. G map-update mask and truncation
 *   render_vjp        adjoint of render w.r.t. voxel means and pose
 *
 * Every value is computed in double precision.  Where a floating-point
 * comparison decides an integer (the hit sample, the interpolation cell, the
 * pixel a voxel projects to, the anchor pixel a point associates with), the
 * caller can ask for that decision to be taken in IEEE single precision with
 * a fixed operation order ("decide32"), the precision the GPU kernels decide
 * in.  That recipe is written out below in plain C with no implicit
 * contraction (fmaf where the recipe fuses a multiply and an add).
 *
 * Layouts: dense maps are double [4][N][N][N] (channel, k, j, i), x fastest;
 * channel 0 occupancy, 1..3 RGB.  Images are row-major [H][W] (rgb [H][W][3]).
 * Poses are 7 doubles (tx, ty, tz, qw, qx, qy, qz), camera -> world.
 * Normal equations are 29 doubles: the 21 upper-triangular entries of
 * H = sum w J^T J (row-major), the 6 entries of g = sum w J^T r, the cost
 * sum w r^2 and the number of contributing pixels.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>


typedef struct {
    int32_t n;          /* voxels per axis */
    int32_t pad_;
    double voxel;       /* edge length (m) */
    double origin[3];   /* min corner (m) */
    double occ_out;     /* occupancy taken by corners outside the grid */
    double rgb_out;     /* colour taken by corners outside the grid */
} orc_grid;

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double d_near, d_far;
    int32_t n_samples;
    int32_t pad_;
    double tau;
} orc_camera;

typedef struct {
    double w_depth, w_rgb;      /* residual weights 1/b^2 */
    double gate_depth;          /* drop depth row if |r_d| > gate_depth */
    double gate_rgb;            /* drop colour rows if |r_c|_1 > gate_rgb */
} orc_weights;

/* ---------------------------------------------------------------------- */
/* small geometry                                                          */
/* ---------------------------------------------------------------------- */
static void quat_to_rot(const double *pose, double R[3][3]) {
    double w = pose[3], x = pose[4], y = pose[5], z = pose[6];
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

void orc_pose_to_rot(const double *pose, double *R9) {
    double R[3][3];
    quat_to_rot(pose, R);
    memcpy(R9, R, sizeof R);
}

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* camera-frame direction of pixel (u, v) with unit z (z-depth rays) */
static void pixel_dir(const orc_camera *c, int u, int v, double r[3]) {
    r[0] = ((u + 0.5) - c->cx) / c->fx;
    r[1] = ((v + 0.5) - c->cy) / c->fy;
    r[2] = 1.0;
}

/* ---------------------------------------------------------------------- */
/* single-precision decision recipe                                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    float R[3][3], t[3];
    float ifx, ify, fx, fy, cx, cy, dn, dstep, tau;
    float o[3], is, s, occ_out;
    int n, W, H, K;
} dec32;

static void dec32_init(dec32 *d, const orc_grid *g, const orc_camera *c, const double *pose) {
    double R[3][3];
    quat_to_rot(pose, R);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) d->R[i][j] = (float)R[i][j];
        d->t[i] = (float)pose[i];
        d->o[i] = g ? (float)g->origin[i] : 0.0f;
    }
    d->ifx = (float)(1.0 / c->fx);
    d->ify = (float)(1.0 / c->fy);
    d->fx = (float)c->fx;
    d->fy = (float)c->fy;
    d->cx = (float)c->cx;
    d->cy = (float)c->cy;
    d->dn = (float)c->d_near;
    d->dstep = c->n_samples > 1 ? (float)((c->d_far - c->d_near) / (c->n_samples - 1)) : 0.0f;
    d->tau = (float)c->tau;
    d->is = g ? (float)(1.0 / g->voxel) : 0.0f;
    d->s = g ? (float)g->voxel : 0.0f;
    d->occ_out = g ? (float)g->occ_out : 0.0f;
    d->n = g ? g->n : 0;
    d->W = c->width;
    d->H = c->height;
    d->K = c->n_samples;
}

static void dec32_dir(const dec32 *d, int u, int v, float dir[3]) {
    float rx = ((float)u + 0.5f - d->cx) * d->ifx;
    float ry = ((float)v + 0.5f - d->cy) * d->ify;
    for (int i = 0; i < 3; ++i) dir[i] = (d->R[i][0] * rx + d->R[i][1] * ry) + d->R[i][2];
}

/* occupancy at sample k along dir, single precision; also returns the cell.
 * Sample k sits at depth d_near + k*dstep along the ray (App. B sampling);
 * its continuous grid coordinate is written as A + k*B with the per-ray
 * terms B = (dir*dstep)/voxel and A = ((t + d_near*dir) - origin)/voxel - 1/2,
 * in this order, 1/voxel rounded once; A + k*B and each linear blend
 * a + w*(b - a) are rounded once (fmaf: the exact product-sum, one rounding). */
static float dec32_sample(const dec32 *d, const double *occ, const float dir[3], int k, int cell[3]) {
    float w[3];
    for (int a = 0; a < 3; ++a) {
        float B = (dir[a] * d->dstep) * d->is;
        float A = ((d->t[a] + d->dn * dir[a]) - d->o[a]) * d->is - 0.5f;
        float g = fmaf((float)k, B, A);
        float fl = floorf(g);
        /* samples more than 2^30 voxels away never reach the grid */
        int i0 = fl < -1073741824.0f ? -1073741824 : fl > 1073741824.0f ? 1073741824 : (int)fl;
        cell[a] = i0;
        w[a] = g - (float)i0;
    }
    float v[2][2][2];
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                int i = cell[0] + a, j = cell[1] + b, kk = cell[2] + c;
                if (i < 0 || j < 0 || kk < 0 || i >= d->n || j >= d->n || kk >= d->n)
                    v[c][b][a] = d->occ_out;
                else
                    v[c][b][a] = (float)occ[((size_t)kk * d->n + j) * d->n + i];
            }
    float l[2][2], m[2];
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b) l[c][b] = fmaf(w[0], v[c][b][1] - v[c][b][0], v[c][b][0]);
    for (int c = 0; c < 2; ++c) m[c] = fmaf(w[1], l[c][1] - l[c][0], l[c][0]);
    return fmaf(w[2], m[1] - m[0], m[0]);
}

/* ---------------------------------------------------------------------- */
/* double-precision trilinear field (App. B) with gradient                 */
/* ---------------------------------------------------------------------- */
typedef struct {
    const orc_grid *g;
    const double *mean;   /* [4][N^3] */
} field;

static double vox(const field *F, int ch, int i, int j, int k) {
    int n = F->g->n;
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n)
        return ch == 0 ? F->g->occ_out : F->g->rgb_out;
    return F->mean[(size_t)ch * n * n * n + ((size_t)k * n + j) * n + i];
}

/* continuous voxel coordinate of a world point (voxel centres at integers) */
static void grid_coord(const orc_grid *g, const double p[3], double gc[3]) {
    for (int a = 0; a < 3; ++a) gc[a] = (p[a] - g->origin[a]) / g->voxel - 0.5;
}

/* Trilinear value of channels [ch0, ch0+nch) at coordinate gc inside cell
 * `cell`; val[c] and gradient dval[c][3] w.r.t. the world point.  The
 * weights are the textbook sum over the 8 corners of the product of 1-D hat
 * weights. */
static void trilinear(const field *F, int ch0, int nch, const double gc[3], const int cell[3],
                      double *val, double (*dval)[3]) {
    double w[3];
    for (int a = 0; a < 3; ++a) w[a] = gc[a] - cell[a];
    for (int c = 0; c < nch; ++c) {
        val[c] = 0.0;
        if (dval) dval[c][0] = dval[c][1] = dval[c][2] = 0.0;
    }
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                double hx = cx ? w[0] : 1.0 - w[0];
                double hy = cy ? w[1] : 1.0 - w[1];
                double hz = cz ? w[2] : 1.0 - w[2];
                double sx = cx ? 1.0 : -1.0, sy = cy ? 1.0 : -1.0, sz = cz ? 1.0 : -1.0;
                for (int c = 0; c < nch; ++c) {
                    double V = vox(F, ch0 + c, cell[0] + cx, cell[1] + cy, cell[2] + cz);
                    val[c] += hx * hy * hz * V;
                    if (dval) {
                        dval[c][0] += sx * hy * hz * V / F->g->voxel;
                        dval[c][1] += hx * sy * hz * V / F->g->voxel;
                        dval[c][2] += hx * hy * sz * V / F->g->voxel;
                    }
                }
            }
}

static void floor_cell(const double gc[3], int cell[3], int n) {
    for (int a = 0; a < 3; ++a) {
        double g = gc[a];
        if (!(g > -2.0)) g = -2.0;       /* also catches NaN */
        if (g > n + 1.0) g = n + 1.0;
        cell[a] = (int)floor(g);
    }
}

/* ---------------------------------------------------------------------- */
/* one ray of the emission (App. B)                                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    int valid;          /* k* exists and k* >= 1 */
    int k;              /* k* (first sample whose occupancy exceeds tau), -1 if none */
    int cell0[3], cell1[3];
    double alpha, depth, rgb[3];
    double p0[3], p1[3];      /* bracketing sample points (world) */
    double d0, d1;            /* bracketing sample depths */
    double f0, f1;            /* bracketing occupancies */
    double c0[3], c1[3];      /* bracketing colours */
} ray_out;

typedef struct {
    const orc_grid *g;
    const orc_camera *c;
    field F;
    double R[3][3], t[3];
    int decide32;
    dec32 d32;
} render_ctx;

static void ctx_init(render_ctx *x, const orc_grid *g, const double *mean, const orc_camera *c,
                     const double *pose, int decide32) {
    x->g = g;
    x->c = c;
    x->F.g = g;
    x->F.mean = mean;
    quat_to_rot(pose, x->R);
    for (int a = 0; a < 3; ++a) x->t[a] = pose[a];
    x->decide32 = decide32;
    dec32_init(&x->d32, g, c, pose);
}

static double sample_depth(const orc_camera *c, int k) {
    double step = c->n_samples > 1 ? (c->d_far - c->d_near) / (c->n_samples - 1) : 0.0;
    return c->d_near + k * step;
}

static void sample_point(const render_ctx *x, const double dir[3], int k, double p[3]) {
    double dk = sample_depth(x->c, k);
    for (int a = 0; a < 3; ++a) p[a] = x->t[a] + dk * dir[a];
}

static void ray_eval(const render_ctx *x, int u, int v, ray_out *o) {
    double rc[3], dir[3];
    pixel_dir(x->c, u, v, rc);
    for (int a = 0; a < 3; ++a) dir[a] = x->R[a][0] * rc[0] + x->R[a][1] * rc[1] + x->R[a][2] * rc[2];
    memset(o, 0, sizeof *o);
    o->k = -1;
    int K = x->c->n_samples;
    int kstar = -1;
    int cell_prev[3] = {0, 0, 0}, cell_hit[3] = {0, 0, 0};
    if (x->decide32) {
        float dir32[3];
        int cell[3];
        dec32_dir(&x->d32, u, v, dir32);
        for (int k = 0; k < K; ++k) {
            float f = dec32_sample(&x->d32, x->F.mean, dir32, k, cell);
            if (f > x->d32.tau) { kstar = k; memcpy(cell_hit, cell, sizeof cell); break; }
            memcpy(cell_prev, cell, sizeof cell);
        }
    } else {
        for (int k = 0; k < K; ++k) {
            double p[3], gc[3], f;
            int cell[3];
            sample_point(x, dir, k, p);
            grid_coord(x->g, p, gc);
            floor_cell(gc, cell, x->g->n);
            trilinear(&x->F, 0, 1, gc, cell, &f, NULL);
            if (f > x->c->tau) { kstar = k; memcpy(cell_hit, cell, sizeof cell); break; }
            memcpy(cell_prev, cell, sizeof cell);
        }
    }
    o->k = kstar;
    if (kstar < 1) return;   /* no crossing, or the camera starts inside a solid */
    o->valid = 1;
    memcpy(o->cell0, cell_prev, sizeof cell_prev);
    memcpy(o->cell1, cell_hit, sizeof cell_hit);
    double gc0[3], gc1[3];
    sample_point(x, dir, kstar - 1, o->p0);
    sample_point(x, dir, kstar, o->p1);
    grid_coord(x->g, o->p0, gc0);
    grid_coord(x->g, o->p1, gc1);
    o->d0 = sample_depth(x->c, kstar - 1);
    o->d1 = sample_depth(x->c, kstar);
    trilinear(&x->F, 0, 1, gc0, o->cell0, &o->f0, NULL);
    trilinear(&x->F, 0, 1, gc1, o->cell1, &o->f1, NULL);
    trilinear(&x->F, 1, 3, gc0, o->cell0, o->c0, NULL);
    trilinear(&x->F, 1, 3, gc1, o->cell1, o->c1, NULL);
    double tau = x->c->tau;
    o->alpha = (tau - o->f0) / (o->f1 - o->f0);
    o->depth = o->alpha * o->d1 + (1.0 - o->alpha) * o->d0;
    for (int c = 0; c < 3; ++c) o->rgb[c] = o->alpha * o->c1[c] + (1.0 - o->alpha) * o->c0[c];
}

/* derivative of (depth, r, g, b) of a valid ray w.r.t. the pose perturbation
 * delta = (dt, dtheta): t <- t + dt, R <- Exp(dtheta) R. */
static void ray_jacobian(const render_ctx *x, const ray_out *o, double J[4][6]) {
    double gc0[3], gc1[3], f0, f1, df0[1][3], df1[1][3], c0[3], c1[3], G0[3][3], G1[3][3];
    grid_coord(x->g, o->p0, gc0);
    grid_coord(x->g, o->p1, gc1);
    trilinear(&x->F, 0, 1, gc0, o->cell0, &f0, df0);
    trilinear(&x->F, 0, 1, gc1, o->cell1, &f1, df1);
    trilinear(&x->F, 1, 3, gc0, o->cell0, c0, G0);
    trilinear(&x->F, 1, 3, gc1, o->cell1, c1, G1);
    /* dp/ddelta = [I | -[p - t]x] ;  for a row vector a: a dp = [a | (p - t) x a] */
    double a0[3], a1[3], rf0[6], rf1[6];
    for (int k = 0; k < 3; ++k) { a0[k] = o->p0[k] - x->t[k]; a1[k] = o->p1[k] - x->t[k]; }
    double cr[3];
    for (int k = 0; k < 3; ++k) rf0[k] = df0[0][k];
    cross3(a0, df0[0], cr);
    for (int k = 0; k < 3; ++k) rf0[3 + k] = cr[k];
    for (int k = 0; k < 3; ++k) rf1[k] = df1[0][k];
    cross3(a1, df1[0], cr);
    for (int k = 0; k < 3; ++k) rf1[3 + k] = cr[k];
    double al = o->alpha, den = f1 - f0;
    double dal[6];
    for (int m = 0; m < 6; ++m) dal[m] = -((1.0 - al) * rf0[m] + al * rf1[m]) / den;
    for (int m = 0; m < 6; ++m) J[0][m] = (o->d1 - o->d0) * dal[m];
    for (int c = 0; c < 3; ++c) {
        double g0[6], g1[6];
        for (int k = 0; k < 3; ++k) { g0[k] = G0[c][k]; g1[k] = G1[c][k]; }
        cross3(a0, G0[c], cr);
        for (int k = 0; k < 3; ++k) g0[3 + k] = cr[k];
        cross3(a1, G1[c], cr);
        for (int k = 0; k < 3; ++k) g1[3 + k] = cr[k];
        for (int m = 0; m < 6; ++m)
            J[1 + c][m] = (c1[c] - c0[c]) * dal[m] + al * g1[m] + (1.0 - al) * g0[m];
    }
}

/* ---------------------------------------------------------------------- */
/* render                                                                  */
/* ---------------------------------------------------------------------- */
void orc_render(const orc_grid *g, const double *mean, const orc_camera *c, const double *pose,
                int decide32, double *depth, double *rgb, uint8_t *mask, int32_t *hit_k) {
    render_ctx x;
    ctx_init(&x, g, mean, c, pose, decide32);
    int W = c->width, H = c->height;
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            ray_out o;
            ray_eval(&x, u, v, &o);
            size_t p = (size_t)v * W + u;
            depth[p] = o.valid ? o.depth : 0.0;
            for (int cc = 0; cc < 3; ++cc) rgb[3 * p + cc] = o.valid ? o.rgb[cc] : 0.0;
            mask[p] = (uint8_t)o.valid;
            if (hit_k) hit_k[p] = o.k;
        }
}

/* normals of a rendered depth image (camera frame of the render) */
void orc_normals(const orc_camera *c, const double *depth, const uint8_t *mask, double disc,
                 double *normals, uint8_t *nmask) {
    int W = c->width, H = c->height;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            normals[3 * p] = normals[3 * p + 1] = normals[3 * p + 2] = 0.0;
            nmask[p] = 0;
            if (u == 0 || v == 0 || u == W - 1 || v == H - 1 || !mask[p]) continue;
            size_t pl = p - 1, pr = p + 1, pu = p - W, pd = p + W;
            if (!mask[pl] || !mask[pr] || !mask[pu] || !mask[pd]) continue;
            double d = depth[p];
            if (fabs(depth[pl] - d) > disc || fabs(depth[pr] - d) > disc ||
                fabs(depth[pu] - d) > disc || fabs(depth[pd] - d) > disc)
                continue;
            double rl[3], rr[3], ru[3], rd[3], r0[3];
            pixel_dir(c, u - 1, v, rl);
            pixel_dir(c, u + 1, v, rr);
            pixel_dir(c, u, v - 1, ru);
            pixel_dir(c, u, v + 1, rd);
            pixel_dir(c, u, v, r0);
            double a[3], b[3], n[3];
            for (int k = 0; k < 3; ++k) {
                a[k] = depth[pr] * rr[k] - depth[pl] * rl[k];
                b[k] = depth[pd] * rd[k] - depth[pu] * ru[k];
            }
            cross3(a, b, n);
            double len = sqrt(dot3(n, n));
            if (!(len > 0.0)) continue;
            double P[3] = {d * r0[0], d * r0[1], d * r0[2]};
            double sgn = dot3(n, P) < 0.0 ? 1.0 : -1.0;
            for (int k = 0; k < 3; ++k) normals[3 * p + k] = sgn * n[k] / len;
            nmask[p] = 1;
        }
}

/* ---------------------------------------------------------------------- */
/* normal-equation accumulation                                            */
/* ---------------------------------------------------------------------- */
static void neq_add_row(double *acc, const double j[6], double r, double w) {
    int q = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b) acc[q++] += w * j[a] * j[b];
    for (int a = 0; a < 6; ++a) acc[21 + a] += w * j[a] * r;
    acc[27] += w * r * r;
}

/* sum per-row partials in row order (deterministic for any thread count) */
static void neq_sum_rows(const double *rows, int H, double *neq) {
    for (int q = 0; q < 29; ++q) neq[q] = 0.0;
    for (int v = 0; v < H; ++v)
        for (int q = 0; q < 29; ++q) neq[q] += rows[(size_t)v * 29 + q];
}

static int depth_ok(double D) { return isfinite(D) && D > 0.0; }

/* Render-through (P1) Jacobian of the emission, residuals against an
 * observed RGB-D frame, gating and the weighted normal equations.
 * J (nullable) receives [H][W][4][6]; resid (nullable) [H][W][4];
 * rowmask (nullable) [H][W] bit0 = depth row used, bit1 = colour rows used. */
void orc_render_jacobian(const orc_grid *g, const double *mean, const orc_camera *c,
                         const double *pose, int decide32, const double *obs_depth,
                         const double *obs_rgb, const orc_weights *wt, double *depth, double *rgb,
                         uint8_t *mask, double *J, double *resid, uint8_t *rowmask, double *neq) {
    render_ctx x;
    ctx_init(&x, g, mean, c, pose, decide32);
    int W = c->width, H = c->height;
    double *rows = (double *)calloc((size_t)H * 29, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v) {
        double *acc = rows + (size_t)v * 29;
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            ray_out o;
            ray_eval(&x, u, v, &o);
            double Jr[4][6] = {{0}};
            double r[4] = {0, 0, 0, 0};
            uint8_t rm = 0;
            if (depth) depth[p] = o.valid ? o.depth : 0.0;
            if (rgb)
                for (int cc = 0; cc < 3; ++cc) rgb[3 * p + cc] = o.valid ? o.rgb[cc] : 0.0;
            if (mask) mask[p] = (uint8_t)o.valid;
            if (o.valid && depth_ok(obs_depth[p])) {
                ray_jacobian(&x, &o, Jr);
                r[0] = o.depth - obs_depth[p];
                for (int cc = 0; cc < 3; ++cc) r[1 + cc] = o.rgb[cc] - obs_rgb[3 * p + cc];
                double l1 = fabs(r[1]) + fabs(r[2]) + fabs(r[3]);
                if (fabs(r[0]) <= wt->gate_depth) {
                    neq_add_row(acc, Jr[0], r[0], wt->w_depth);
                    rm |= 1;
                }
                if (l1 <= wt->gate_rgb) {
                    for (int cc = 0; cc < 3; ++cc) neq_add_row(acc, Jr[1 + cc], r[1 + cc], wt->w_rgb);
                    rm |= 2;
                }
                if (rm) acc[28] += 1.0;
            }
            if (J) memcpy(J + p * 24, Jr, sizeof Jr);
            if (resid) memcpy(resid + p * 4, r, sizeof r);
            if (rowmask) rowmask[p] = rm;
        }
    }
    neq_sum_rows(rows, H, neq);
    free(rows);
}

/* ---------------------------------------------------------------------- */
/* prediction-to-observation tracking against the previous render (P2)     */
/* ---------------------------------------------------------------------- */
/* Per observed pixel: back-project with the observed depth, move it with the
 * current pose iterate into the previous (anchor) camera, associate with the
 * nearest anchor pixel for the point-to-plane term and bilinearly interpolate
 * the anchor colour for the photometric term. */
void orc_track_p2(const orc_camera *c, const double *pose, const double *pose_prev,
                  int decide32, const double *obs_depth, const double *obs_rgb,
                  const double *a_depth, const double *a_rgb, const uint8_t *a_mask,
                  const double *a_normals, const uint8_t *a_nmask, const orc_weights *wt,
                  double *J, double *resid, uint8_t *rowmask, double *neq) {
    double R[3][3], Rp[3][3];
    quat_to_rot(pose, R);
    quat_to_rot(pose_prev, Rp);
    dec32 dc;
    dec32_init(&dc, NULL, c, pose);
    /* relative transform current camera -> anchor camera, formed in double
     * (Rrel = Rp^T R, trel = Rp^T (t - t_prev), sums in index order) and
     * rounded to float for the single-precision association recipe */
    struct { float R[3][3], t[3]; } rel;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            rel.R[a][b] = (float)((Rp[0][a] * R[0][b] + Rp[1][a] * R[1][b]) + Rp[2][a] * R[2][b]);
        double d0 = pose[0] - pose_prev[0], d1 = pose[1] - pose_prev[1], d2 = pose[2] - pose_prev[2];
        rel.t[a] = (float)((Rp[0][a] * d0 + Rp[1][a] * d1) + Rp[2][a] * d2);
    }
    int W = c->width, H = c->height;
    double *rows = (double *)calloc((size_t)H * 29, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v) {
        double *acc = rows + (size_t)v * 29;
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            double Jr[4][6] = {{0}};
            double r[4] = {0, 0, 0, 0};
            uint8_t rm = 0;
            double D = obs_depth[p];
            int geo_ok = 0, pho_ok = 0, giu = 0, giv = 0, bix = 0, biy = 0;
            if (depth_ok(D)) {
                /* integer decisions */
                int front = 0;
                double u_d = 0, v_d = 0;
                if (decide32) {
                    float D32 = (float)D;
                    float rx = ((float)u + 0.5f - dc.cx) * dc.ifx;
                    float ry = ((float)v + 0.5f - dc.cy) * dc.ify;
                    float X[3] = {D32 * rx, D32 * ry, D32};
                    float Y[3];
                    for (int a = 0; a < 3; ++a)
                        Y[a] = ((rel.R[a][0] * X[0] + rel.R[a][1] * X[1]) + rel.R[a][2] * X[2]) + rel.t[a];
                    if (Y[2] > 0.0f) {
                        front = 1;
                        float uu = dc.fx * (Y[0] / Y[2]) + dc.cx;
                        float vv = dc.fy * (Y[1] / Y[2]) + dc.cy;
                        if (uu >= 0.0f && uu < (float)W && vv >= 0.0f && vv < (float)H) {
                            giu = (int)uu; giv = (int)vv; geo_ok = 1;
                        }
                        float bx = uu - 0.5f, by = vv - 0.5f;
                        if (bx >= 0.0f && bx < (float)(W - 1) && by >= 0.0f && by < (float)(H - 1)) {
                            bix = (int)bx; biy = (int)by; pho_ok = 1;
                        }
                    }
                } else {
                    double rc[3], X[3], dW[3], Y[3];
                    pixel_dir(c, u, v, rc);
                    for (int a = 0; a < 3; ++a) X[a] = D * rc[a];
                    for (int a = 0; a < 3; ++a)
                        dW[a] = R[a][0] * X[0] + R[a][1] * X[1] + R[a][2] * X[2] + pose[a] - pose_prev[a];
                    for (int a = 0; a < 3; ++a) Y[a] = Rp[0][a] * dW[0] + Rp[1][a] * dW[1] + Rp[2][a] * dW[2];
                    if (Y[2] > 0.0) {
                        front = 1;
                        u_d = c->fx * Y[0] / Y[2] + c->cx;
                        v_d = c->fy * Y[1] / Y[2] + c->cy;
                        if (u_d >= 0.0 && u_d < W && v_d >= 0.0 && v_d < H) {
                            giu = (int)u_d; giv = (int)v_d; geo_ok = 1;
                        }
                        double bx = u_d - 0.5, by = v_d - 0.5;
                        if (bx >= 0.0 && bx < W - 1 && by >= 0.0 && by < H - 1) {
                            bix = (int)bx; biy = (int)by; pho_ok = 1;
                        }
                    }
                }
                (void)front;
                if (geo_ok) {
                    size_t q = (size_t)giv * W + giu;
                    if (!a_mask[q] || !a_nmask[q]) geo_ok = 0;
                }
                if (pho_ok) {
                    size_t q = (size_t)biy * W + bix;
                    if (!a_mask[q] || !a_mask[q + 1] || !a_mask[q + W] || !a_mask[q + W + 1]) pho_ok = 0;
                }
                if (geo_ok || pho_ok) {
                    /* values in double precision */
                    double rc[3], X[3], RX[3], dW[3], Y[3];
                    pixel_dir(c, u, v, rc);
                    for (int a = 0; a < 3; ++a) X[a] = D * rc[a];
                    for (int a = 0; a < 3; ++a) RX[a] = R[a][0] * X[0] + R[a][1] * X[1] + R[a][2] * X[2];
                    for (int a = 0; a < 3; ++a) dW[a] = RX[a] + pose[a] - pose_prev[a];
                    for (int a = 0; a < 3; ++a) Y[a] = Rp[0][a] * dW[0] + Rp[1][a] * dW[1] + Rp[2][a] * dW[2];
                    /* dY/ddelta = Rp^T [I | -[RX]x]  (3 x 6) */
                    double dY[3][6];
                    for (int a = 0; a < 3; ++a) {
                        double e[3] = {Rp[0][a], Rp[1][a], Rp[2][a]};   /* row a of Rp^T */
                        double cr[3];
                        for (int k = 0; k < 3; ++k) dY[a][k] = e[k];
                        cross3(RX, e, cr);                            /* e . (-[RX]x) = RX x e */
                        for (int k = 0; k < 3; ++k) dY[a][3 + k] = cr[k];
                    }
                    if (geo_ok) {
                        size_t q = (size_t)giv * W + giu;
                        double ra[3], ph[3];
                        pixel_dir(c, giu, giv, ra);
                        for (int a = 0; a < 3; ++a) ph[a] = a_depth[q] * ra[a];
                        const double *nn = a_normals + 3 * q;
                        double diff[3] = {ph[0] - Y[0], ph[1] - Y[1], ph[2] - Y[2]};
                        r[0] = dot3(nn, diff);
                        for (int m = 0; m < 6; ++m)
                            Jr[0][m] = -(nn[0] * dY[0][m] + nn[1] * dY[1][m] + nn[2] * dY[2][m]);
                        if (fabs(r[0]) <= wt->gate_depth) {
                            neq_add_row(acc, Jr[0], r[0], wt->w_depth);
                            rm |= 1;
                        }
                    }
                    if (pho_ok) {
                        double uu = c->fx * Y[0] / Y[2] + c->cx;
                        double vv = c->fy * Y[1] / Y[2] + c->cy;
                        double ax = (uu - 0.5) - bix, ay = (vv - 0.5) - biy;
                        size_t q00 = (size_t)biy * W + bix, q10 = q00 + 1, q01 = q00 + W, q11 = q01 + 1;
                        double dpi[2][3] = {{c->fx / Y[2], 0.0, -c->fx * Y[0] / (Y[2] * Y[2])},
                                            {0.0, c->fy / Y[2], -c->fy * Y[1] / (Y[2] * Y[2])}};
                        double l1 = 0.0;
                        for (int cc = 0; cc < 3; ++cc) {
                            double I00 = a_rgb[3 * q00 + cc], I10 = a_rgb[3 * q10 + cc];
                            double I01 = a_rgb[3 * q01 + cc], I11 = a_rgb[3 * q11 + cc];
                            double Ii = (1 - ax) * (1 - ay) * I00 + ax * (1 - ay) * I10 +
                                        (1 - ax) * ay * I01 + ax * ay * I11;
                            double gu = (1 - ay) * (I10 - I00) + ay * (I11 - I01);
                            double gv = (1 - ax) * (I01 - I00) + ax * (I11 - I10);
                            r[1 + cc] = Ii - obs_rgb[3 * p + cc];
                            l1 += fabs(r[1 + cc]);
                            for (int m = 0; m < 6; ++m) {
                                double du = dpi[0][0] * dY[0][m] + dpi[0][1] * dY[1][m] + dpi[0][2] * dY[2][m];
                                double dv = dpi[1][0] * dY[0][m] + dpi[1][1] * dY[1][m] + dpi[1][2] * dY[2][m];
                                Jr[1 + cc][m] = gu * du + gv * dv;
                            }
                        }
                        if (l1 <= wt->gate_rgb) {
                            for (int cc = 0; cc < 3; ++cc) neq_add_row(acc, Jr[1 + cc], r[1 + cc], wt->w_rgb);
                            rm |= 2;
                        }
                    }
                    if (rm) acc[28] += 1.0;
                }
            }
            if (J) memcpy(J + p * 24, Jr, sizeof Jr);
            if (resid) memcpy(resid + p * 4, r, sizeof r);
            if (rowmask) rowmask[p] = rm;
        }
    }
    neq_sum_rows(rows, H, neq);
    free(rows);
}

/* ---------------------------------------------------------------------- */
/* closed-form map update (App. D)                                         */
/* ---------------------------------------------------------------------- */
/* For every voxel whose centre projects into the image in front of the
 * camera, onto a valid observed depth D, with camera z <= D + trunc:
 *   f = (max(z - D, -trunc), rgb_obs)      (negative SDF, then colour)
 *   Lambda' = Lambda + lam_u,  mu' = (Lambda')^-1 (Lambda mu + lam_u f)
 * (the product written with the inverse of the new precision, as App. D
 * prints it; the stored variance is that inverse), applied per channel in
 * place on mean/var ([4][N^3] each).
 * upd (nullable) receives a 0/1 flag per voxel.  Returns the update count. */
int64_t orc_map_update(const orc_grid *g, double *mean, double *var, const orc_camera *c,
                       const double *pose, int decide32, const double *obs_depth,
                       const double *obs_rgb, double trunc, double lam_u, uint8_t *upd) {
    double R[3][3];
    quat_to_rot(pose, R);
    dec32 d;
    dec32_init(&d, g, c, pose);
    float trunc32 = (float)trunc;
    int n = g->n, W = c->width, H = c->height;
    size_t NV = (size_t)n * n * n;
    int64_t count = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : count)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t idx = ((size_t)k * n + j) * n + i;
                if (upd) upd[idx] = 0;
                int iu, iv, ok = 0;
                if (decide32) {
                    float xw[3] = {d.o[0] + d.s * ((float)i + 0.5f), d.o[1] + d.s * ((float)j + 0.5f),
                                   d.o[2] + d.s * ((float)k + 0.5f)};
                    float dd[3] = {xw[0] - d.t[0], xw[1] - d.t[1], xw[2] - d.t[2]};
                    float X[3];
                    for (int a = 0; a < 3; ++a) X[a] = (d.R[0][a] * dd[0] + d.R[1][a] * dd[1]) + d.R[2][a] * dd[2];
                    if (X[2] > 0.0f) {
                        float uu = d.fx * (X[0] / X[2]) + d.cx;
                        float vv = d.fy * (X[1] / X[2]) + d.cy;
                        if (uu >= 0.0f && uu < (float)W && vv >= 0.0f && vv < (float)H) {
                            iu = (int)uu; iv = (int)vv;
                            float D = (float)obs_depth[(size_t)iv * W + iu];
                            if (D > 0.0f && isfinite(D) && X[2] <= D + trunc32) ok = 1;
                        }
                    }
                } else {
                    double xw[3] = {g->origin[0] + g->voxel * (i + 0.5), g->origin[1] + g->voxel * (j + 0.5),
                                    g->origin[2] + g->voxel * (k + 0.5)};
                    double dd[3] = {xw[0] - pose[0], xw[1] - pose[1], xw[2] - pose[2]};
                    double X[3];
                    for (int a = 0; a < 3; ++a) X[a] = R[0][a] * dd[0] + R[1][a] * dd[1] + R[2][a] * dd[2];
                    if (X[2] > 0.0) {
                        double uu = c->fx * X[0] / X[2] + c->cx;
                        double vv = c->fy * X[1] / X[2] + c->cy;
                        if (uu >= 0.0 && uu < W && vv >= 0.0 && vv < H) {
                            iu = (int)uu; iv = (int)vv;
                            double D = obs_depth[(size_t)iv * W + iu];
                            if (depth_ok(D) && X[2] <= D + trunc) ok = 1;
                        }
                    }
                }
                if (!ok) continue;
                /* update values in double precision */
                double xw[3] = {g->origin[0] + g->voxel * (i + 0.5), g->origin[1] + g->voxel * (j + 0.5),
                                g->origin[2] + g->voxel * (k + 0.5)};
                double dd[3] = {xw[0] - pose[0], xw[1] - pose[1], xw[2] - pose[2]};
                double z = R[0][2] * dd[0] + R[1][2] * dd[1] + R[2][2] * dd[2];
                size_t pix = (size_t)iv * W + iu;
                double D = obs_depth[pix];
                double f[4];
                f[0] = z - D;
                if (f[0] < -trunc) f[0] = -trunc;
                for (int cc = 0; cc < 3; ++cc) f[1 + cc] = obs_rgb[3 * pix + cc];
                for (int ch = 0; ch < 4; ++ch) {
                    size_t q = (size_t)ch * NV + idx;
                    double lam = 1.0 / var[q];
                    double lam2 = lam + lam_u;
                    double var2 = 1.0 / lam2;
                    mean[q] = var2 * (lam * mean[q] + lam_u * f[ch]);
                    var[q] = var2;
                }
                if (upd) upd[idx] = 1;
                count += 1;
            }
    return count;
}

/* ---------------------------------------------------------------------- */
/* adjoint of render                                                       */
/* ---------------------------------------------------------------------- */
/* Given the hit sample k* of every ray (held fixed) and upstream gradients
 * of the rendered depth and colour, accumulate dL/dmean ([4][N^3]) and
 * dL/ddelta (6).  Recomputes the two bracketing samples of each ray. */
void orc_render_vjp(const orc_grid *g, const double *mean, const orc_camera *c, const double *pose,
                    int decide32, const double *g_depth, const double *g_rgb, double *grad_mean,
                    double *grad_pose) {
    render_ctx x;
    ctx_init(&x, g, mean, c, pose, decide32);
    int W = c->width, H = c->height, n = g->n;
    size_t NV = (size_t)n * n * n;
    double gp[6] = {0, 0, 0, 0, 0, 0};
    /* serial on purpose: scatter-adds into grad_mean in a fixed order */
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            ray_out o;
            ray_eval(&x, u, v, &o);
            if (!o.valid) continue;
            double gd = g_depth[p];
            const double *gc = g_rgb + 3 * p;
            double Jr[4][6];
            ray_jacobian(&x, &o, Jr);
            for (int m = 0; m < 6; ++m)
                gp[m] += gd * Jr[0][m] + gc[0] * Jr[1][m] + gc[1] * Jr[2][m] + gc[2] * Jr[3][m];
            double al = o.alpha, den = o.f1 - o.f0;
            double g_alpha = gd * (o.d1 - o.d0);
            for (int cc = 0; cc < 3; ++cc) g_alpha += gc[cc] * (o.c1[cc] - o.c0[cc]);
            double g_f0 = g_alpha * (-(1.0 - al) / den);
            double g_f1 = g_alpha * (-al / den);
            for (int s = 0; s < 2; ++s) {
                const double *pt = s ? o.p1 : o.p0;
                const int *cell = s ? o.cell1 : o.cell0;
                double gcd[3], w[3];
                grid_coord(g, pt, gcd);
                for (int a = 0; a < 3; ++a) w[a] = gcd[a] - cell[a];
                double g_occ = s ? g_f1 : g_f0;
                double crgb = s ? al : 1.0 - al;
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx) {
                            int i = cell[0] + cx, j = cell[1] + cy, k = cell[2] + cz;
                            if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) continue;
                            double h = (cx ? w[0] : 1 - w[0]) * (cy ? w[1] : 1 - w[1]) * (cz ? w[2] : 1 - w[2]);
                            size_t idx = ((size_t)k * n + j) * n + i;
                            grad_mean[idx] += g_occ * h;
                            for (int cc = 0; cc < 3; ++cc) grad_mean[(size_t)(1 + cc) * NV + idx] += gc[cc] * crgb * h;
                        }
            }
        }
    for (int m = 0; m < 6; ++m) grad_pose[m] = gp[m];
}
