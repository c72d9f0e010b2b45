"""Pins of the oracle's 15-D state (pose, velocities and an accelerometer
bias, the state the simulated IMU trajectories call for; the paper's own
state is 12-D, App. E): the transition with the body-frame specific force as
the linear control, its linearisation, and the filter's split and
combination over the larger velocity block.  Each is pinned to something
other than the oracle: an independent write-out of the transition with
scipy's rotations, central differences, the 12-D prediction it reduces to,
and Monte Carlo over the transition."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

G = np.array([0.0, 0.0, -9.81])


def _state(rng, bias=True):
    q = Rotation.from_rotvec(rng.normal(size=3)).as_quat()
    x = dict(t=rng.normal(size=3), q=np.array([q[3], q[0], q[1], q[2]]),
             v=rng.normal(size=3), w=rng.normal(0, 0.5, size=3))
    x["b"] = rng.normal(0, 0.05, size=3) if bias else np.zeros(3)
    return x


def _rot(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]])


def _step(x, u, dt, n, du=None):
    """The biased-IMU transition written out with scipy's rotations: the
    acceleration R (f - b) + g, velocities first (+ n_v, n_w), the position
    with the new velocity (+ n_t), the rotation by Exp(w' dt) with the noise
    on the left, the bias a random walk (+ n_b); the controls enter over du
    (dt, or dt^2 in the printed form).  Returns (t, R, v, w, b)."""
    du = dt if du is None else du
    R = _rot(x["q"])
    a = R.apply(u[:3] - x["b"]) + G
    v = x["v"] + a * du + n[6:9]
    w = x["w"] + u[3:] * du + n[9:12]
    t = x["t"] + v * dt + n[0:3]
    R2 = Rotation.from_rotvec(n[3:6]) * Rotation.from_rotvec(w * dt) * R
    return t, R2.as_matrix(), v, w, x["b"] + n[12:15]


def _err(a, b):
    return np.concatenate([a[0] - b[0], Rotation.from_matrix(a[1] @ b[1].T).as_rotvec(), a[2] - b[2], a[3] - b[3],
                           a[4] - b[4]])


def test_bias_transition_mean_is_the_written_out_step(orc):
    rng = np.random.default_rng(41)
    x, u, dt = _state(rng), rng.normal(size=6) + np.array([0, 0, 9.81, 0, 0, 0]), 0.1
    xn = orc.transition_mean_bias(x, u, dt, G)
    t, R, v, w, b = _step(x, u, dt, np.zeros(15))
    np.testing.assert_allclose(xn["t"], t, rtol=0, atol=1e-13)
    np.testing.assert_allclose(xn["v"], v, rtol=0, atol=1e-13)
    np.testing.assert_allclose(xn["w"], w, rtol=0, atol=1e-14)
    np.testing.assert_allclose(orc.quat_to_rot(xn["q"]), R, rtol=0, atol=1e-13)
    np.testing.assert_array_equal(xn["b"], b)


@pytest.mark.parametrize("dt2", [False, True])
def test_bias_transition_linearisation_matches_fd(orc, dt2):
    """M and G of the 15-D linearised transition (tangent dt, dtheta, dv, dw,
    db; left perturbations) against central differences of the written-out
    transition in the error state and in the noise; also with the controls
    entering over dt^2 (the printed form)."""
    rng = np.random.default_rng(42)
    x, u, dt = _state(rng), rng.normal(size=6) + np.array([0, 0, 9.81, 0, 0, 0]), 0.1
    du = dt * dt if dt2 else dt
    xn = orc.transition_mean_bias(x, u, dt, G, dt2)
    M, Gn = orc.transition_jacobians_bias(x, xn, u, dt, dt2)
    base = _step(x, u, dt, np.zeros(15), du)
    eps = 1e-6
    Mfd = np.zeros((15, 15))
    Gfd = np.zeros((15, 15))
    for i in range(15):
        for sgn in (1, -1):
            d = np.zeros(15)
            d[i] = sgn * eps
            R2 = (Rotation.from_rotvec(d[3:6]) * _rot(x["q"])).as_quat()
            xp = dict(t=x["t"] + d[0:3], q=np.array([R2[3], R2[0], R2[1], R2[2]]), v=x["v"] + d[6:9],
                      w=x["w"] + d[9:12], b=x["b"] + d[12:15])
            Mfd[:, i] += sgn * _err(_step(xp, u, dt, np.zeros(15), du), base) / (2 * eps)
            Gfd[:, i] += sgn * _err(_step(x, u, dt, d, du), base) / (2 * eps)
    np.testing.assert_allclose(M, Mfd, atol=2e-7)
    np.testing.assert_allclose(Gn, Gfd, atol=2e-7)
    # the new blocks are really exercised
    assert np.abs(M[6:9, 3:6]).max() > 0.1 * du / dt and np.abs(M[6:9, 12:15]).max() > 0.05 * du / dt


def test_bias_prediction_reduces_to_the_12d_one(orc):
    """With no bias, no bias noise and a certain rotation and bias, feeding
    the body-frame force f = R^T (a - g) predicts the same mean and the same
    pose-velocity covariance as the 12-D filter fed the world acceleration a
    (the rotation's uncertainty is what the extra coupling acts on)."""
    rng = np.random.default_rng(43)
    x = _state(rng, bias=False)
    a = rng.normal(size=3)
    alpha = rng.normal(size=3)
    R = _rot(x["q"])
    u_body = np.concatenate([R.inv().apply(a - G), alpha])
    u_world = np.concatenate([a, alpha])
    A = rng.normal(size=(15, 15))
    P = (A @ A.T + 15 * np.eye(15)) * 1e-3
    P[3:6, :] = 0.0
    P[:, 3:6] = 0.0
    P[12:15, :] = 0.0
    P[:, 12:15] = 0.0
    p15 = orc.Params(accel_bias=True, sigma_bias=0.0, gravity=tuple(G))
    x15, P15 = orc.predict(x, P, u_body, p15)
    x12, P12 = orc.predict({k: x[k] for k in ("t", "q", "v", "w")}, P[:12, :12], u_world, orc.Params())
    for k in ("t", "v", "w"):
        np.testing.assert_allclose(x15[k], x12[k], rtol=0, atol=1e-12)
    assert np.linalg.norm(orc.pose_error(np.concatenate([x15["t"], x15["q"]]),
                                         np.concatenate([x12["t"], x12["q"]]))) < 1e-12
    np.testing.assert_allclose(P15[:12, :12], P12, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(P15[12:, 12:], np.zeros((3, 3)))


def test_bias_prediction_matches_monte_carlo(orc):
    """3000 draws from the 15-D belief pushed through the written-out
    transition with its process noise: sample mean and covariance (tangent
    at the predicted mean) agree with the linearised prediction within
    sampling error."""
    rng = np.random.default_rng(44)
    x = _state(rng)
    u = np.array([0.3, -0.2, 9.6, 0.1, -0.2, 0.05])
    s = np.array([0.01] * 3 + [0.01] * 3 + [0.02] * 3 + [0.02] * 3 + [0.01] * 3)
    A = rng.normal(size=(15, 15)) * 0.2
    C = np.diag(s) @ (A @ A.T + np.eye(15)) @ np.diag(s)
    p = orc.Params(accel_bias=True, sigma_bias=0.002, gravity=tuple(G))
    xn, Pn = orc.predict(x, C, u, p)
    L = np.linalg.cholesky(C)
    q = np.sqrt([p.sigma_pose_t ** 2] * 3 + [p.sigma_pose_r ** 2] * 3 + [p.sigma_vel_t ** 2] * 3 +
                [p.sigma_vel_r ** 2] * 3 + [p.sigma_bias ** 2] * 3)
    S = 3000
    base = (xn["t"], orc.quat_to_rot(xn["q"]), xn["v"], xn["w"], xn["b"])
    E = np.zeros((S, 15))
    for k in range(S):
        e = L @ rng.normal(size=15)
        R0 = (Rotation.from_rotvec(e[3:6]) * _rot(x["q"])).as_quat()
        xs = dict(t=x["t"] + e[0:3], q=np.array([R0[3], R0[0], R0[1], R0[2]]), v=x["v"] + e[6:9],
                  w=x["w"] + e[9:12], b=x["b"] + e[12:15])
        E[k] = _err(_step(xs, u, p.dt, q * rng.normal(size=15)), base)
    sd = np.sqrt(np.diag(Pn))
    assert np.all(np.abs(E.mean(0)) < 4 * sd / np.sqrt(S) + 2e-2 * sd)
    Ce = np.cov(E.T)
    assert np.linalg.norm(Ce - Pn) < 0.1 * np.linalg.norm(Pn), np.linalg.norm(Ce - Pn) / np.linalg.norm(Pn)


def test_bias_split_and_combine_round_trip(orc):
    """Split of a 15-D joint covariance into the pose marginal and the
    9-D velocity-and-bias conditional, and the combination with the same
    pose marginal, give the joint back."""
    rng = np.random.default_rng(45)
    A = rng.normal(size=(15, 15))
    P = A @ A.T + 15 * np.eye(15)
    Spp, D, Sv = orc.split(P)
    assert D.shape == (9, 6) and Sv.shape == (9, 9)
    prior = np.array([0.1, 0.2, 0.3, 1.0, 0.0, 0.0, 0.0])
    mu = rng.normal(size=9)
    vm, Pj = orc.combine(prior, Spp, prior, mu, D, Sv)
    np.testing.assert_allclose(Pj, 0.5 * (P + P.T), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(vm, mu, rtol=0, atol=0)


def test_bias_filter_follows_the_trajectory(orc):
    """Sanity (not parity): the 15-D oracle filter on a short trajectory,
    fed the accelerometer's body-frame force, keeps the position error at
    the centimetre level."""
    import synth
    c = synth.trajectory_case(seed=1, n=64, width=80, height=60, n_samples=32, n_frames=6)
    tr = c["traj"]
    mean = np.zeros((4, 64, 64, 64))
    mean[0] = np.float32(-0.001)
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6 + [1e-4] * 3)
    of = orc.Filter(orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"]),
                    orc.Params(accel_bias=True, gravity=tuple(G), n_gn=3),
                    dict(t=tr.t[0], q=tr.q[0], v=tr.v[0], w=tr.w[0], b=np.zeros(3)), P0, mean,
                    np.full_like(mean, 1e4))
    for i in range(6):
        of.step(c["depth"][i].astype(np.float64), c["rgb"][i].astype(np.float64), tr.u_body[i - 1] if i else None)
        assert of.s.P.shape == (15, 15) and of.s.b.shape == (3,)
    assert np.linalg.norm(of.s.t - tr.t[5]) < 0.05


def _rollout_belief15(rng):
    x = dict(t=np.array([1.0, 2.0, 1.5]), q=np.array([0.9, 0.1, -0.2, 0.3]) / np.linalg.norm([0.9, 0.1, -0.2, 0.3]),
             v=np.array([0.3, -0.1, 0.05]), w=np.array([0.2, 0.4, -0.3]), b=np.array([0.02, -0.03, 0.01]))
    A = rng.normal(size=(15, 15)) * 0.01
    P = A @ A.T + np.diag([1e-5] * 6 + [1e-4] * 6 + [1e-5] * 3)
    u = rng.normal(size=(5, 6)) + np.array([0.0, 0.0, 9.81, 0.0, 0.0, 0.0])
    return x, P, u


def test_bias_rollout_without_noise_follows_the_predicted_mean(orc):
    """Zero draws from the 15-D belief: every sampled trajectory is the
    noise-free transition of the mean, i.e. the closed-form predicted means
    (the bias stays at its mean)."""
    rng = np.random.default_rng(46)
    x, P, u = _rollout_belief15(rng)
    p = orc.Params(accel_bias=True, gravity=tuple(G))
    out = orc.rollout(None, None, None, x, P, u, np.zeros((2, 6, 15)), p, frames=False)
    assert out["mean"].shape == (5, 16) and out["cov"].shape == (5, 15, 15)
    for s in range(2):
        np.testing.assert_allclose(out["poses"][s, :, :3], out["mean"][:, :3], rtol=0, atol=1e-12)
        for j in range(5):
            assert np.linalg.norm(orc.pose_error(out["poses"][s, j], out["mean"][j, :7])) < 1e-12
    np.testing.assert_allclose(out["mean"][:, 13:16], np.tile(x["b"], (5, 1)), rtol=0, atol=0)


def test_bias_rollout_samples_match_the_linearised_moments(orc):
    """Monte Carlo over the 15-D generative transition (bias walk included):
    the sampled poses' mean and covariance agree with the closed-form
    linearised prediction within sampling error."""
    rng = np.random.default_rng(47)
    x, P, u = _rollout_belief15(rng)
    p = orc.Params(accel_bias=True, gravity=tuple(G), sigma_bias=0.01)
    S = 3000
    out = orc.rollout(None, None, None, x, P, u, rng.normal(size=(S, 6, 15)), p, frames=False)
    for j in (0, 4):
        e = np.array([orc.pose_error(out["poses"][s, j], out["mean"][j, :7]) for s in range(S)])
        C = out["cov"][j][:6, :6]
        sd = np.sqrt(np.diag(C))
        assert np.all(np.abs(e.mean(0)) < 4 * sd / np.sqrt(S) + 1e-3 * sd)
        Ce = np.cov(e.T)
        assert np.linalg.norm(Ce - C) < 0.1 * np.linalg.norm(C), (j, np.linalg.norm(Ce - C) / np.linalg.norm(C))
