"""Pins of the oracle's paper-literal modes (the forms the paper prints where
the default takes another reading): the (dt)^2 transition (App. E.1), the
factor of the Laplace covariance (Sec. 5.1), the L1 objective of App. E.3
minimised by iteratively reweighted least squares, and the App. B / App. G
sample spacing.  Each is pinned to something other than the oracle itself:
a closed form, a library routine or a textbook property."""
import math

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.spatial.transform import Rotation

import synth


def _state(rng):
    q = Rotation.from_rotvec(rng.normal(size=3)).as_quat()
    return dict(t=rng.normal(size=3), q=np.array([q[3], q[0], q[1], q[2]]),
                v=rng.normal(size=3), w=rng.normal(size=3))


def _rot(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def test_dt2_transition_is_the_printed_form(orc):
    """App. E.1 as printed: v' = v + u dt^2, w' = w + u_w dt^2, then the pose
    with the new velocities; written out here with scipy's rotations."""
    rng = np.random.default_rng(31)
    x, u, dt = _state(rng), rng.normal(size=6), 0.07
    xn = orc.transition_mean(x, u, dt, dt2=True)
    v = x["v"] + u[:3] * dt ** 2
    w = x["w"] + u[3:] * dt ** 2
    np.testing.assert_allclose(xn["v"], v, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(xn["w"], w, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(xn["t"], x["t"] + v * dt, rtol=1e-14, atol=1e-15)
    R = Rotation.from_rotvec(w * dt).as_matrix() @ _rot(x["q"])
    np.testing.assert_allclose(_rot(xn["q"]), R, atol=1e-14)
    # at dt = 1 the two forms coincide; elsewhere they differ by the control
    one = orc.transition_mean(x, u, 1.0, dt2=True)
    ref = orc.transition_mean(x, u, 1.0)
    for k in one:
        np.testing.assert_allclose(one[k], ref[k], rtol=1e-15, atol=1e-15)
    assert np.linalg.norm(xn["v"] - orc.transition_mean(x, u, dt)["v"]) > 1e-3


def test_dt2_transition_reaches_prediction_and_rollouts(orc):
    """The prediction's mean and a rollout's noise-free draw both follow the
    printed form when the mode is on; the covariance propagation does not
    depend on the control (the control enters additively)."""
    rng = np.random.default_rng(32)
    x, u = _state(rng), rng.normal(size=6)
    P = np.diag(rng.uniform(1e-4, 1e-3, 12))
    p = orc.Params(dt=0.05, transition_dt2=True)
    xn, Pn = orc.predict(x, P, u, p)
    ref = orc.transition_mean(x, u, p.dt, dt2=True)
    for k in ("t", "v", "w", "q"):
        np.testing.assert_array_equal(xn[k], ref[k])
    # the covariance depends on the control only through the new angular
    # velocity (Exp(w' dt) and its Jacobian): the default form started from
    # the angular velocity that gives the same w' propagates the same one
    x2 = dict(x)
    x2["w"] = x["w"] + u[3:] * (p.dt ** 2 - p.dt)
    _, Pd2 = orc.predict(x2, P, u, orc.Params(dt=0.05))
    np.testing.assert_allclose(Pn, Pd2, rtol=1e-12, atol=1e-18)
    s = orc.transition_sample(x, u, np.zeros(12), p.dt, dt2=True)
    for k in ("t", "v", "w"):
        np.testing.assert_allclose(s[k], ref[k], rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("factor", [1.0, 2.0])
def test_laplace_factor_is_the_gaussian_posterior(orc, factor):
    """Sec. 5.1 prints Sigma = (2 J^T J)^-1 for the squared objective
    sum w r^2; with factor f the Laplace covariance (f H + Lp)^-1 is the
    Kalman posterior covariance of a linear measurement with noise variance
    1/(f w) (factor 1: the Gaussian likelihood of precision w)."""
    rng = np.random.default_rng(33)
    m = 30
    Jm = rng.normal(size=(m, 6))
    w = rng.uniform(0.5, 3.0, m)
    neq = np.zeros(29)
    q = 0
    for a in range(6):
        for b in range(a, 6):
            neq[q] = np.sum(w * Jm[:, a] * Jm[:, b])
            q += 1
    A = rng.normal(size=(6, 6))
    P0 = (A @ A.T + 6 * np.eye(6)) * 0.01
    S = orc.laplace(neq, np.linalg.inv(P0), factor)
    Rm = np.diag(1.0 / (factor * w))
    K = P0 @ Jm.T @ np.linalg.inv(Jm @ P0 @ Jm.T + Rm)
    np.testing.assert_allclose(S, P0 - K @ Jm @ P0, rtol=1e-9, atol=1e-14)


def test_irls_weights_find_the_median(orc):
    """A location problem under the L1 objective sum |x - y_i| / b is solved
    by the median (textbook); iterating the weighted least-squares solution
    with the oracle's IRLS weights converges to it."""
    rng = np.random.default_rng(34)
    y = rng.laplace(0.3, 0.05, 101)
    b = 0.02
    x = float(np.mean(y))
    for _ in range(300):
        w = orc.irls_weight(x - y, b, 1e-9)
        x = float(np.sum(w * y) / np.sum(w))
    assert abs(x - np.median(y)) < 1e-7
    # the weight is that of the majoriser r^2 / (2 b |r0|) of |r| / b
    r0 = np.array([0.3, -0.02, 1e-12])
    np.testing.assert_allclose(orc.irls_weight(r0, b, 0.01), 1.0 / (2 * b * np.array([0.3, 0.02, 0.01 * b])))


def test_neq_from_rows_equals_the_accumulated_normal_equations(orc):
    """The numpy normal equations from a frame's rows, with the weights
    1/b^2 of the squared form, equal the ones the C objective accumulates
    pixel by pixel (two independent sums of the same rows)."""
    c = synth.single_frame_case(0)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    pt = synth.pose7(c["t_gt"], c["q_gt"])
    p0 = synth.pose7(c["t_init"], c["q_init"])
    D, C = synth.raycast(c["scene"], c["cam"], c["t_gt"], c["q_gt"])
    anchor = orc.render(g, mean, cam, pt, normals=True)
    p = orc.Params()
    out = orc.track_p2(cam, p0, pt, D, C, anchor, p, want_J=True)
    r = out["resid"].reshape(-1, 4)
    w = np.empty_like(r)
    w[:, 0] = 1.0 / p.b_geo ** 2
    w[:, 1:] = 1.0 / p.b_rgb ** 2
    neq = orc.neq_from_rows(out["J"], r, out["rowmask"], w)
    assert out["neq"][28] > 500
    np.testing.assert_allclose(neq, out["neq"], rtol=1e-10, atol=1e-9 * np.abs(out["neq"][:21]).max())


def test_irls_gauss_newton_reaches_the_l1_minimum(orc):
    """Linear rows r = r0 + J delta (four per pixel, as the objective's
    pixels have) and a negligible prior: Gauss-Newton iterations on the IRLS
    normal equations reach the minimum of sum |r_d| / b_geo + sum |r_c| /
    b_rgb that a linear program (scipy's HiGHS) finds."""
    rng = np.random.default_rng(35)
    npx = 60
    J = rng.normal(size=(npx, 4, 6))
    d_true = rng.normal(0, 0.1, 6)
    r0 = rng.laplace(0, 0.05, size=(npx, 4)) - J @ d_true
    p = orc.Params(irls=True, irls_floor=1e-9)
    scale = np.array([p.b_geo, p.b_rgb, p.b_rgb, p.b_rgb])
    Lp = 1e-12 * np.eye(6)
    rows = dict(J=J, rowmask=np.full(npx, 3, np.uint8))
    delta = np.zeros(6)
    for _ in range(200):
        rows["resid"] = r0 + J @ delta
        neq = orc.irls_neq(rows, p)
        delta = delta + orc.gn_solve(neq, Lp, delta)

    def l1(d):
        return float(np.sum(np.abs(r0 + J @ d) / scale))

    # min sum t_i  s.t.  -t <= (r0 + J d) / b <= t
    A = (J / scale[None, :, None]).reshape(-1, 6)
    b0 = (r0 / scale).reshape(-1)
    m = len(b0)
    cost = np.concatenate([np.zeros(6), np.ones(m)])
    A_ub = np.block([[A, -np.eye(m)], [-A, -np.eye(m)]])
    b_ub = np.concatenate([-b0, b0])
    lp = linprog(cost, A_ub=A_ub, b_ub=b_ub, bounds=[(None, None)] * 6 + [(0, None)] * m, method="highs")
    assert lp.status == 0
    assert l1(delta) <= lp.fun * (1 + 1e-6) + 1e-9
    assert l1(np.zeros(6)) > 2 * lp.fun


def test_paper_sample_camera_spacing(orc):
    """App. B samples at depth offsets eps, 2 eps, 3 eps, ...; App. G sets
    eps = 0.4 voxel and the maximum camera depth: the camera's k-th sample
    depth is (k + 1) eps and the last one is the largest multiple of eps not
    beyond the maximum depth."""
    for voxel, dmax in ((0.025, 8.0), (0.05, 7.0), (0.1, 20.0), (0.03, 5.0)):
        cam = orc.paper_sample_camera(64, 48, 50.0, 50.0, 32.0, 24.0, voxel, dmax)
        eps = 0.4 * voxel
        K = cam.n_samples
        assert K * eps <= dmax * (1 + 1e-12) and (K + 1) * eps > dmax
        step = (cam.d_far - cam.d_near) / (K - 1)
        d = cam.d_near + np.arange(K) * step
        np.testing.assert_allclose(d, eps * (np.arange(K) + 1), rtol=1e-12)
        assert math.isclose(cam.d_near, eps)
