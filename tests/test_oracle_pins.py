"""Pins of the FP64 oracle against things other than itself: closed forms,
library routines, brute force on tiny inputs and finite differences.

Each test names the passage of the paper (Mirchev et al., PRISM, CoRL 2022)
whose statement it pins.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
from scipy.spatial.transform import Rotation

import synth


def _pose(t, R):
    q = Rotation.from_matrix(R).as_quat()        # (x, y, z, w)
    return np.array([t[0], t[1], t[2], q[3], q[0], q[1], q[2]])


def _look_rot(fwd, up=(0, 0, 1)):
    """Camera->world rotation (x right, y down, z forward)."""
    f = np.asarray(fwd, float) / np.linalg.norm(fwd)
    r = np.cross(f, np.asarray(up, float))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    return np.stack([r, d, f], axis=1)


def _affine_map(n, voxel, nrm, p0, A, b, occ_out=-0.001):
    """Dense [4][n][n][n] map with occupancy n.(p - p0) and colour A p + b."""
    ax = (np.arange(n) + 0.5) * voxel
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    P = np.stack([x, y, z], -1)
    m = np.empty((4, n, n, n))
    m[0] = (P - p0) @ nrm
    m[1:] = np.moveaxis(P @ A.T + b, -1, 0)
    return m


# ---------------------------------------------------------------------------
# App. B emission
# ---------------------------------------------------------------------------
def test_render_affine_plane_is_exact(orc):
    """Trilinear interpolation reproduces affine fields, and along a ray an
    affine occupancy is affine in depth, so the interpolated crossing
    (App. B depth-interpolation eq.) is the exact ray/plane intersection and
    the blended colour is the colour field at that point."""
    rng = np.random.default_rng(3)
    n, s = 24, 0.1
    nrm = np.array([0.9, 0.3, -0.2]); nrm /= np.linalg.norm(nrm)
    cam_t = np.array([1.0, 1.2, 1.1])
    p0 = cam_t + 0.55 * nrm
    A = rng.normal(size=(3, 3)) * 0.3
    b = rng.normal(size=3)
    mean = _affine_map(n, s, nrm, p0, A, b)
    R = _look_rot(nrm + np.array([0.1, -0.2, 0.05]))
    pose = _pose(cam_t, R)
    cam = orc.Cam(16, 12, 12.0, 12.0, 8.0, 6.0, 0.05, 0.95, 24)
    grid = orc.Grid(n, s)
    out = orc.render(grid, mean, cam, pose, decide32=False)
    checked = 0
    for v in range(cam.height):
        for u in range(cam.width):
            rc = np.array([(u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy, 1.0])
            d = R @ rc
            dex = nrm @ (p0 - cam_t) / (nrm @ d)
            ds = cam.d_near + np.arange(cam.n_samples) * (cam.d_far - cam.d_near) / (cam.n_samples - 1)
            kx = int(np.argmax(ds > dex))
            pts = cam_t + ds[:kx + 1, None] * d
            g = pts / s - 0.5
            if not (np.all(g >= 0) and np.all(g <= n - 1) and kx >= 1 and ds[-1] > dex):
                continue
            checked += 1
            assert out["mask"][v, u] == 1
            assert out["hit_k"][v, u] == kx
            assert abs(out["depth"][v, u] - dex) < 1e-12
            np.testing.assert_allclose(out["rgb"][v, u], A @ (cam_t + dex * d) + b, atol=1e-12)
    assert checked > 100


def _brute_render(mean, n, s, occ_out, rgb_out, cam, t, R, tau=0.0):
    """Independent first-crossing search with scipy's linear interpolation
    (map_coordinates order 1, constant padding)."""
    H, W, K = cam.height, cam.width, cam.n_samples
    ds = cam.d_near + np.arange(K) * (cam.d_far - cam.d_near) / (K - 1)
    depth = np.zeros((H, W)); rgb = np.zeros((H, W, 3)); mask = np.zeros((H, W), np.uint8)
    hit = np.full((H, W), -1)
    for v in range(H):
        for u in range(W):
            rc = np.array([(u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy, 1.0])
            pts = t + ds[:, None] * (R @ rc)
            coords = (pts / s - 0.5)[:, ::-1].T           # (k, j, i) order
            f = ndi.map_coordinates(mean[0], coords, order=1, mode="grid-constant", cval=occ_out)
            above = np.nonzero(f > tau)[0]
            if len(above) == 0:
                continue
            k = above[0]
            hit[v, u] = k
            if k == 0:
                continue
            col = np.stack([ndi.map_coordinates(mean[c], coords[:, k - 1:k + 1], order=1,
                                                mode="grid-constant", cval=rgb_out) for c in (1, 2, 3)], -1)
            a = (tau - f[k - 1]) / (f[k] - f[k - 1])
            depth[v, u] = a * ds[k] + (1 - a) * ds[k - 1]
            rgb[v, u] = a * col[1] + (1 - a) * col[0]
            mask[v, u] = 1
    return depth, rgb, mask, hit


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_render_matches_bruteforce_tiny(orc, seed):
    """First sample whose occupancy exceeds tau, strict (App. B); checked on
    random 4^3 and 6^3 grids against an independent search."""
    rng = np.random.default_rng(seed)
    n = 4 + 2 * (seed % 2)
    s = 0.25
    mean = rng.uniform(-1, 1, size=(4, n, n, n))
    mean[0] -= 0.3
    t = np.array([0.5, 0.5, -0.3]) + rng.normal(0, 0.05, 3)
    R = Rotation.from_rotvec(rng.normal(0, 0.2, 3)).as_matrix()
    cam = orc.Cam(7, 5, 5.0, 5.0, 3.5, 2.5, 0.1, 1.6, 12)
    out = orc.render(orc.Grid(n, s), mean, cam, _pose(t, R), decide32=False)
    d, c, m, k = _brute_render(mean, n, s, -0.001, 0.0, cam, t, R)
    np.testing.assert_array_equal(out["hit_k"], k)
    np.testing.assert_array_equal(out["mask"], m)
    np.testing.assert_allclose(out["depth"], d, atol=1e-12)
    np.testing.assert_allclose(out["rgb"], c, atol=1e-12)
    assert m.sum() > 5


def test_render_tie_is_not_a_hit(orc):
    """Occupancy equal to tau does not exceed it: an all-zero map has no hit,
    in both decision precisions."""
    n = 8
    mean = np.zeros((4, n, n, n))
    cam = orc.Cam(6, 4, 4.0, 4.0, 3.0, 2.0, 0.1, 1.5, 10)
    g = orc.Grid(n, 0.25, occ_out=0.0)
    pose = _pose(np.array([1.0, 1.0, 0.2]), np.eye(3))
    for d32 in (False, True):
        out = orc.render(g, mean, cam, pose, decide32=d32)
        assert out["mask"].sum() == 0 and np.all(out["hit_k"] == -1)


def test_render_room_matches_raycast(orc):
    """On the synthetic room (axis-aligned walls, clamped SDF map) the render
    equals the analytic ray cast wherever the crossing lies in a single
    wall's affine band; elsewhere (edges) it is within two voxels."""
    c = synth.single_frame_case(0)
    scene = c["scene"]
    mean, _ = synth.gt_map(scene)
    g = orc.grid_from_scene(scene)
    cam = orc.cam_from(c["cam"])
    pose = synth.pose7(c["t_gt"], c["q_gt"])
    out = orc.render(g, mean, cam, pose, decide32=False)
    d_ex, _ = synth.raycast(scene, c["cam"], c["t_gt"], c["q_gt"])
    err = np.abs(out["depth"] - d_ex)[out["mask"] == 1]
    assert out["mask"].mean() > 0.99
    assert np.mean(err < 1e-9) > 0.7
    assert err.max() < 2 * scene.voxel


def test_decide32_agrees_with_decide64(orc):
    """Single-precision decisions change hit samples only where the FP64
    occupancy is within rounding of tau; depth stays continuous."""
    c = synth.single_frame_case(1)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    pose = synth.pose7(c["t_init"], c["q_init"])
    a = orc.render(g, mean, cam, pose, decide32=True)
    b = orc.render(g, mean, cam, pose, decide32=False)
    assert np.mean(a["hit_k"] != b["hit_k"]) < 1e-3
    both = (a["mask"] == 1) & (b["mask"] == 1)
    np.testing.assert_allclose(a["depth"][both], b["depth"][both], rtol=1e-6)


# ---------------------------------------------------------------------------
# pose Jacobian of the emission (P1) and normal equations
# ---------------------------------------------------------------------------
def _retract_np(pose, delta):
    R = Rotation.from_quat([pose[4], pose[5], pose[6], pose[3]]).as_matrix()
    R2 = Rotation.from_rotvec(delta[3:]).as_matrix() @ R
    return _pose(pose[:3] + delta[:3], R2)


def test_render_jacobian_finite_differences(orc):
    """Per-ray d(depth, rgb)/d(delta) against central differences of the
    render (eps 1e-6, FP64 decisions); rays whose hit sample changes are
    excluded."""
    c = synth.single_frame_case(0)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    pose = synth.pose7(c["t_init"], c["q_init"])
    p = orc.Params()
    obs = orc.render(g, mean, cam, pose)
    out = orc.render_jacobian(g, mean, cam, pose, obs["depth"], obs["rgb"], p, decide32=False,
                              want_J=True)
    J = out["J"]
    eps = 1e-6
    good = 0
    total = 0
    for m in range(6):
        e = np.zeros(6); e[m] = eps
        a = orc.render(g, mean, cam, _retract_np(pose, e), decide32=False)
        b = orc.render(g, mean, cam, _retract_np(pose, -e), decide32=False)
        ok = (a["hit_k"] == b["hit_k"]) & (a["mask"] == 1) & (b["mask"] == 1) & (out["mask"] == 1)
        fd = np.concatenate([(a["depth"] - b["depth"])[..., None], a["rgb"] - b["rgb"]], -1) / (2 * eps)
        err = np.abs(fd - J[..., m])[ok]
        scale = np.maximum(np.abs(J[..., m][ok]), 1e-2)
        good += np.sum(np.all(err / scale < 1e-4, axis=-1))
        total += ok.sum()
    assert total > 0.9 * 6 * cam.width * cam.height
    assert good / total > 0.99


def test_neq_packing(orc):
    """The 29-vector holds sum w J^T J (upper triangle), sum w J^T r, cost
    and the contributing-pixel count of the rows that pass the gates."""
    c = synth.single_frame_case(2)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    p = orc.Params()
    obs_d, obs_c = synth.raycast(c["scene"], c["cam"], c["t_gt"], c["q_gt"],
                                 np.random.default_rng(0), 0.01, 0.02)
    out = orc.render_jacobian(g, mean, cam, synth.pose7(c["t_init"], c["q_init"]), obs_d, obs_c, p,
                              want_J=True)
    J, r, rm = out["J"], out["resid"], out["rowmask"]
    w = np.zeros(r.shape)
    w[..., 0] = np.where(rm & 1, 1 / p.b_geo ** 2, 0)
    w[..., 1:] = np.where((rm & 2)[..., None], 1 / p.b_rgb ** 2, 0)
    Hm = np.einsum("hwr,hwra,hwrb->ab", w, J, J)
    gv = np.einsum("hwr,hwra,hwr->a", w, J, r)
    H, gg, cost, cnt = orc.neq_unpack(out["neq"])
    np.testing.assert_allclose(H, Hm, rtol=1e-10, atol=1e-6)
    np.testing.assert_allclose(gg, gv, rtol=1e-10, atol=1e-8)
    assert abs(cost - np.sum(w * r * r)) < 1e-8 * max(1, cost)
    assert cnt == np.sum(rm > 0)
    # gating: the rows kept are exactly those within the App. G thresholds
    valid = (out["mask"] == 1) & (obs_d > 0)
    np.testing.assert_array_equal((rm & 1) > 0, valid & (np.abs(r[..., 0]) <= p.gate_geo))
    np.testing.assert_array_equal((rm & 2) > 0, valid & (np.abs(r[..., 1:]).sum(-1) <= p.gate_rgb))


def test_known_pose_gives_zero_step(orc):
    """Observation rendered at the true pose, prior centred there: every
    residual vanishes, g = 0 and the Gauss-Newton step is 0."""
    c = synth.single_frame_case(0)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    pose = synth.pose7(c["t_gt"], c["q_gt"])
    p = orc.Params()
    obs = orc.render(g, mean, cam, pose)
    out = orc.render_jacobian(g, mean, cam, pose, obs["depth"], obs["rgb"], p)
    H, gg, cost, cnt = orc.neq_unpack(out["neq"])
    assert cnt > 0.9 * cam.width * cam.height
    assert cost == 0.0 and np.all(gg == 0.0)
    Lp = np.diag([1 / 0.05 ** 2] * 3 + [1 / 0.02 ** 2] * 3)
    delta = orc.gn_solve(out["neq"], Lp, np.zeros(6))
    assert np.all(np.abs(delta) < 1e-15)


def test_gn_step_converges_from_perturbation(orc):
    """From a 2 cm / 1 degree perturbation a few Gauss-Newton steps on the
    render-through objective recover the pose (expected behaviour)."""
    c = synth.single_frame_case(0)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    gt = synth.pose7(c["t_gt"], c["q_gt"])
    p = orc.Params()
    obs = orc.render(g, mean, cam, gt)
    prior = synth.pose7(c["t_init"], c["q_init"])
    Lp = np.diag([1 / 0.05 ** 2] * 3 + [1 / 0.02 ** 2] * 3) * 1e-3
    it = prior.copy()
    for _ in range(5):
        out = orc.render_jacobian(g, mean, cam, it, obs["depth"], obs["rgb"], p)
        it = orc.retract(it, orc.gn_solve(out["neq"], Lp, orc.pose_error(it, prior)))
    e0 = np.linalg.norm(orc.pose_error(prior, gt))
    e1 = np.linalg.norm(orc.pose_error(it, gt))
    assert e1 < 0.1 * e0


# ---------------------------------------------------------------------------
# P2 surrogate (App. E.3)
# ---------------------------------------------------------------------------
def _plane_anchor(orc):
    n, s = 24, 0.1
    nrm = np.array([0.2, -0.1, 1.0]); nrm /= np.linalg.norm(nrm)
    cam_t = np.array([1.2, 1.2, 0.6])
    p0 = cam_t + 0.9 * nrm
    mean = _affine_map(n, s, nrm, p0, np.zeros((3, 3)), np.zeros(3))
    # smooth colour so the photometric term has a gradient
    ax = (np.arange(n) + 0.5) * s
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    mean[1] = 0.5 + 0.3 * np.sin(3 * x) * np.cos(2 * y)
    mean[2] = 0.4 + 0.2 * np.cos(4 * y + z)
    mean[3] = 0.3 + 0.1 * x
    R = _look_rot(nrm + np.array([0.05, 0.1, 0.0]), up=(0, 1, 0))
    pose = _pose(cam_t, R)
    cam = orc.Cam(40, 30, 30.0, 30.0, 20.0, 15.0, 0.1, 1.8, 48)
    g = orc.Grid(n, s)
    a = orc.render(g, mean, cam, pose, decide32=False, normals=True)
    return g, mean, cam, pose, a, nrm, p0


def test_p2_identity_has_zero_residuals(orc):
    """Observation equal to the anchor, current pose equal to the anchor
    pose: every pixel associates with itself and all residuals vanish."""
    g, mean, cam, pose, a, _, _ = _plane_anchor(orc)
    p = orc.Params()
    for d32 in (False, True):
        out = orc.track_p2(cam, pose, pose, a["depth"], a["rgb"], a, p, decide32=d32)
        used = out["rowmask"] > 0
        assert used.sum() > 0.5 * cam.width * cam.height
        assert np.max(np.abs(out["resid"][used])) < 1e-12


def test_p2_point_to_plane_is_plane_distance(orc):
    """Against a rendered plane, the point-to-plane residual n.(p_hat - Y)
    equals the analytic signed distance of the moved point to that plane."""
    g, mean, cam, pose, a, nrm, p0 = _plane_anchor(orc)
    p = orc.Params(gate_geo=10.0, gate_rgb=10.0)
    cur = _retract_np(pose, np.array([0.01, -0.02, 0.015, 0.01, -0.005, 0.008]))
    rng = np.random.default_rng(0)
    obs_d = rng.uniform(0.6, 1.2, size=(cam.height, cam.width))
    obs_c = np.zeros((cam.height, cam.width, 3))
    out = orc.track_p2(cam, cur, pose, obs_d, obs_c, a, p, decide32=False)
    Rc = Rotation.from_quat([cur[4], cur[5], cur[6], cur[3]]).as_matrix()
    Ra = Rotation.from_quat([pose[4], pose[5], pose[6], pose[3]]).as_matrix()
    n_a = Ra.T @ nrm             # plane normal in the anchor camera frame (towards camera)
    n_a = -n_a if n_a @ (Ra.T @ (p0 - pose[:3])) > 0 else n_a
    p0_a = Ra.T @ (p0 - pose[:3])
    checked = 0
    for v in range(cam.height):
        for u in range(cam.width):
            if not out["rowmask"][v, u] & 1:
                continue
            rc = np.array([(u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy, 1.0])
            Y = Ra.T @ (Rc @ (obs_d[v, u] * rc) + cur[:3] - pose[:3])
            assert abs(out["resid"][v, u, 0] - n_a @ (p0_a - Y)) < 1e-9
            checked += 1
    assert checked > 200


def test_p2_jacobian_finite_differences(orc):
    """P2 residual Jacobian against central differences (eps 1e-7); pixels
    whose association or gating changes are excluded."""
    g, mean, cam, pose, a, _, _ = _plane_anchor(orc)
    p = orc.Params()
    cur = _retract_np(pose, np.array([0.004, -0.003, 0.002, 0.003, -0.002, 0.002]))
    obs_d = a["depth"] * 1.001
    obs_c = a["rgb"] + 0.01
    out = orc.track_p2(cam, cur, pose, obs_d, obs_c, a, p, decide32=False, want_J=True)
    eps = 1e-7
    tot = good = 0
    for m in range(6):
        e = np.zeros(6); e[m] = eps
        A_ = orc.track_p2(cam, _retract_np(cur, e), pose, obs_d, obs_c, a, p, decide32=False)
        B_ = orc.track_p2(cam, _retract_np(cur, -e), pose, obs_d, obs_c, a, p, decide32=False)
        ok = (A_["rowmask"] == out["rowmask"]) & (B_["rowmask"] == out["rowmask"])
        fd = (A_["resid"] - B_["resid"]) / (2 * eps)
        for row, bit in ((slice(0, 1), 1), (slice(1, 4), 2)):
            sel = ok & ((out["rowmask"] & bit) > 0)
            err = np.abs(fd[..., row] - out["J"][..., row, m])[sel]
            scale = np.maximum(np.abs(out["J"][..., row, m][sel]), 1e-2)
            good += np.sum(np.all(err / scale < 1e-4, axis=-1))
            tot += sel.sum()
    assert tot > 1000 and good / tot > 0.98


# ---------------------------------------------------------------------------
# map update (App. D)
# ---------------------------------------------------------------------------
def _frontal_wall(orc, n=16, s=0.1):
    """Camera looking along +x at a wall x = xw, exact constant z-depth."""
    cam = orc.Cam(20, 16, 15.0, 15.0, 10.0, 8.0, 0.1, 2.0, 20)
    t = np.array([0.33, 0.81, 0.79])
    R = _look_rot([1.0, 0.0, 0.0])
    xw = 1.17
    depth = np.full((cam.height, cam.width), xw - t[0])
    return orc.Grid(n, s), cam, _pose(t, R), depth, t, R


def test_map_update_frontal_wall_closed_form(orc):
    """With an uninformative prior (precision ~0) one update sets each voxel
    in the update region to max(z - D, -trunc) and the observed colour;
    voxels outside the region are bitwise unchanged."""
    g, cam, pose, depth, t, R = _frontal_wall(orc)
    p = orc.Params()
    n = g.n
    rng = np.random.default_rng(0)
    mean = rng.normal(size=(4, n, n, n))
    var = np.full((4, n, n, n), 1e300)
    rgb = np.broadcast_to(np.array([0.2, 0.5, 0.7]), (cam.height, cam.width, 3)).copy()
    m0, v0 = mean.copy(), var.copy()
    cnt, upd = orc.map_update(g, mean, var, cam, pose, depth, rgb, p, decide32=False, want_mask=True)
    trunc = p.trunc_voxels * g.voxel
    ax = (np.arange(n) + 0.5) * g.voxel
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    Pc = (np.stack([X, Y, Z], -1) - t) @ R      # camera-frame coordinates
    z = Pc[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        uu = cam.fx * Pc[..., 0] / z + cam.cx
        vv = cam.fy * Pc[..., 1] / z + cam.cy
    inside = (z > 0) & (uu >= 0) & (uu < cam.width) & (vv >= 0) & (vv < cam.height)
    expect = inside & (z <= depth[0, 0] + trunc)
    np.testing.assert_array_equal(upd.astype(bool), expect)
    assert cnt == expect.sum() > 100
    f = np.maximum(z - depth[0, 0], -trunc)
    np.testing.assert_allclose(mean[0][expect], f[expect], rtol=0, atol=1e-12)
    for c in range(3):
        np.testing.assert_allclose(mean[1 + c][expect], rgb[0, 0, c], atol=1e-12)
    np.testing.assert_array_equal(mean[:, ~expect], m0[:, ~expect])
    np.testing.assert_array_equal(var[:, ~expect], v0[:, ~expect])


def test_map_update_curless_levoy(orc):
    """Precision-form product = Curless-Levoy running average (App. D): from
    a flat prior, after n unit-precision updates the mean is the arithmetic
    mean of the updates and the precision is n."""
    g, cam, pose, depth0, t, R = _frontal_wall(orc)
    p = orc.Params()
    n = g.n
    mean = np.zeros((4, n, n, n))
    var = np.full((4, n, n, n), 1e300)
    rng = np.random.default_rng(1)
    fs = []
    masks = []
    for i in range(5):
        dd = depth0 + rng.uniform(-0.02, 0.02)
        col = rng.uniform(0, 1, 3)
        rgb = np.broadcast_to(col, (cam.height, cam.width, 3)).copy()
        _, upd = orc.map_update(g, mean, var, cam, pose, dd, rgb, p, decide32=False, want_mask=True)
        masks.append(upd.astype(bool))
        fs.append((dd[0, 0], col))
    allm = np.logical_and.reduce(masks)
    assert allm.sum() > 100
    trunc = p.trunc_voxels * g.voxel
    ax = (np.arange(n) + 0.5) * g.voxel
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    z = ((np.stack([X, Y, Z], -1) - t) @ R)[..., 2]
    f_mean = np.mean([np.maximum(z - D, -trunc) for D, _ in fs], axis=0)
    np.testing.assert_allclose(mean[0][allm], f_mean[allm], atol=1e-12)
    np.testing.assert_allclose(mean[1][allm], np.mean([c[0] for _, c in fs]), atol=1e-12)
    np.testing.assert_allclose(1.0 / var[:, allm], 5.0, rtol=1e-12)


def test_map_update_precision_sum(orc):
    """Two Gaussians multiply to precision Lambda + Lambda_u and a precision-
    weighted mean (App. D); checked against the covariance form of the
    product, sigma'^2 = s1 s2 / (s1 + s2), mu' = (s2 mu1 + s1 mu2)/(s1+s2)."""
    g, cam, pose, depth, t, R = _frontal_wall(orc)
    p = orc.Params(sigma_update=0.7)
    n = g.n
    rng = np.random.default_rng(5)
    mean = rng.normal(size=(4, n, n, n))
    var = rng.uniform(0.1, 3.0, size=(4, n, n, n))
    m0, v0 = mean.copy(), var.copy()
    rgb = rng.uniform(0, 1, size=(cam.height, cam.width, 3))
    _, upd = orc.map_update(g, mean, var, cam, pose, depth, rgb, p, decide32=False, want_mask=True)
    u = upd.astype(bool)
    s2 = p.sigma_update ** 2
    trunc = p.trunc_voxels * g.voxel
    ax = (np.arange(n) + 0.5) * g.voxel
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    z = ((np.stack([X, Y, Z], -1) - t) @ R)[..., 2]
    f0 = np.maximum(z - depth[0, 0], -trunc)
    np.testing.assert_allclose(var[:, u], v0[:, u] * s2 / (v0[:, u] + s2), rtol=1e-12)
    np.testing.assert_allclose(mean[0][u], (s2 * m0[0][u] + v0[0][u] * f0[u]) / (v0[0][u] + s2),
                               rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# adjoint of the emission
# ---------------------------------------------------------------------------
def test_render_vjp_finite_differences(orc):
    """dL/dmean and dL/ddelta of L = sum(gd * depth + gc . rgb), against
    central differences on a small case (hit samples held; rays whose hit
    changes under the perturbation are rare and excluded via tolerance)."""
    rng = np.random.default_rng(0)
    n, s = 12, 0.2
    mean = np.empty((4, n, n, n))
    ax = (np.arange(n) + 0.5) * s
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    mean[0] = 0.3 * np.sin(2.1 * X) + 0.25 * np.cos(1.7 * Y + 0.5 * Z) + 0.2 * Z - 0.2
    mean[1:] = rng.uniform(0, 1, size=(3, n, n, n))
    t = np.array([1.2, 1.1, 0.3])
    R = _look_rot([0.1, 0.05, 1.0], up=(0, 1, 0))
    pose = _pose(t, R)
    cam = orc.Cam(10, 8, 8.0, 8.0, 5.0, 4.0, 0.1, 1.9, 24)
    g = orc.Grid(n, s)
    gd = rng.normal(size=(cam.height, cam.width))
    gc = rng.normal(size=(cam.height, cam.width, 3))
    gm, gp = orc.render_vjp(g, mean, cam, pose, gd, gc, decide32=False)
    base = orc.render(g, mean, cam, pose, decide32=False)
    assert base["mask"].sum() > 40

    def L(mm, pp):
        o = orc.render(g, mm, cam, pp, decide32=False)
        return np.sum(gd * o["depth"]) + np.sum(gc * o["rgb"]), o["hit_k"]

    eps = 1e-6
    for m in range(6):
        e = np.zeros(6); e[m] = eps
        la, ka = L(mean, _retract_np(pose, e))
        lb, kb = L(mean, _retract_np(pose, -e))
        assert np.array_equal(ka, kb)
        assert abs((la - lb) / (2 * eps) - gp[m]) < 1e-5 * max(1.0, abs(gp[m]))
    idx = np.argwhere(np.abs(gm).sum(0) > 0)
    assert len(idx) > 50
    pick = idx[rng.choice(len(idx), size=40, replace=False)]
    for (k, j, i) in pick:
        for ch in range(4):
            mp = mean.copy(); mp[ch, k, j, i] += eps
            mq = mean.copy(); mq[ch, k, j, i] -= eps
            la, ka = L(mp, pose)
            lb, kb = L(mq, pose)
            if not np.array_equal(ka, kb):
                continue
            assert abs((la - lb) / (2 * eps) - gm[ch, k, j, i]) < 1e-6 * max(1.0, abs(gm[ch, k, j, i]))


def test_render_vjp_pose_is_jacobian_transpose(orc):
    """The pose part of the adjoint is J^T g for the per-ray P1 Jacobian."""
    c = synth.single_frame_case(0)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    pose = synth.pose7(c["t_init"], c["q_init"])
    p = orc.Params()
    rng = np.random.default_rng(1)
    gd = rng.normal(size=(cam.height, cam.width))
    gc = rng.normal(size=(cam.height, cam.width, 3))
    out = orc.render_jacobian(g, mean, cam, pose, np.ones((cam.height, cam.width)),
                              np.zeros((cam.height, cam.width, 3)), p, want_J=True)
    _, gp = orc.render_vjp(g, mean, cam, pose, gd, gc)
    ug = np.concatenate([gd[..., None], gc], -1) * (out["mask"][..., None] == 1)
    np.testing.assert_allclose(gp, np.einsum("hwr,hwrm->m", ug, out["J"]), rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------------------
# map inference by gradient descent through the renderer (Sec. 4.3.1, Sec. 5.3)
# ---------------------------------------------------------------------------
def _gd_case(orc, seed=0):
    rng = np.random.default_rng(seed)
    n, s = 12, 0.2
    ax = (np.arange(n) + 0.5) * s
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    mean0 = np.empty((4, n, n, n))
    mean0[0] = 0.3 * np.sin(2.1 * X) + 0.25 * np.cos(1.7 * Y + 0.5 * Z) + 0.2 * Z - 0.2
    mean0[1:] = rng.uniform(0, 1, size=(3, n, n, n))
    var0 = rng.uniform(0.5, 2.0, size=(4, n, n, n))
    pose = _pose(np.array([1.2, 1.1, 0.3]), _look_rot([0.1, 0.05, 1.0], up=(0, 1, 0)))
    cam = orc.Cam(10, 8, 8.0, 8.0, 5.0, 4.0, 0.1, 1.9, 24)
    g = orc.Grid(n, s)
    ref = orc.render(g, mean0, cam, pose, decide32=False)
    obs_d = np.where(ref["mask"] == 1, ref["depth"] + rng.normal(0, 0.05, ref["depth"].shape), 0.0)
    obs_c = np.clip(ref["rgb"] + rng.normal(0, 0.05, ref["rgb"].shape), 0, 1)
    return rng, g, cam, pose, mean0, var0, obs_d, obs_c


def test_map_gd_gradient_finite_differences(orc):
    """dE/dmu of the map-filter objective (data rows through the adjoint plus
    the quadratic previous-belief term) against central differences of E,
    at a point away from the previous mean so the prior term is live; rays
    whose hit or kept rows change under the perturbation are skipped."""
    rng, g, cam, pose, mean0, var0, obs_d, obs_c = _gd_case(orc)
    p = orc.Params(gate_rgb=0.3)
    mean = mean0 + rng.normal(0, 0.01, mean0.shape)
    E, grad = orc.map_gd_objective(g, mean, mean0, var0, cam, pose, obs_d, obs_c, p, decide32=False)
    rj = orc.render_jacobian(g, mean, cam, pose, obs_d, obs_c, p, decide32=False)
    assert rj["neq"][28] > 30 and 0 < np.count_nonzero(rj["rowmask"] == 1) < rj["neq"][28]

    def ev(mm):
        e, _ = orc.map_gd_objective(g, mm, mean0, var0, cam, pose, obs_d, obs_c, p, decide32=False)
        o = orc.render_jacobian(g, mm, cam, pose, obs_d, obs_c, p, decide32=False)
        return e, (o["rowmask"].tobytes(), orc.render(g, mm, cam, pose, decide32=False)["hit_k"].tobytes())

    eps = 1e-6
    touched = np.argwhere(np.abs(grad - (mean - mean0) / var0).sum(0) > 1e-9)
    assert len(touched) > 50
    pick = touched[rng.choice(len(touched), size=30, replace=False)]
    checked = 0
    for (k, j, i) in pick:
        for ch in range(4):
            mp = mean.copy(); mp[ch, k, j, i] += eps
            mq = mean.copy(); mq[ch, k, j, i] -= eps
            ea, ka = ev(mp)
            eb, kb = ev(mq)
            if ka != kb:
                continue
            fd = (ea - eb) / (2 * eps)
            assert abs(fd - grad[ch, k, j, i]) < 1e-5 * max(1.0, abs(grad[ch, k, j, i])), (ch, k, j, i)
            checked += 1
    assert checked > 80
    # a voxel no ray touches: central differences of E see only the
    # previous-belief term (mu - mu0) / var0
    far = np.argwhere(np.abs(grad - (mean - mean0) / var0).sum(0) == 0)
    assert len(far) > 100
    for (k, j, i) in far[rng.choice(len(far), size=5, replace=False)]:
        for ch in range(4):
            mp = mean.copy(); mp[ch, k, j, i] += 1e-4
            mq = mean.copy(); mq[ch, k, j, i] -= 1e-4
            fd = (ev(mp)[0] - ev(mq)[0]) / 2e-4
            exp = (mean[ch, k, j, i] - mean0[ch, k, j, i]) / var0[ch, k, j, i]
            assert abs(fd - exp) < 1e-8 and abs(grad[ch, k, j, i] - exp) < 1e-15


def test_map_gd_without_data_keeps_the_previous_belief(orc):
    """No valid observed depth: the data term is empty and the previous mean
    is the minimiser, so descent stays there with zero objective."""
    _, g, cam, pose, mean0, var0, obs_d, obs_c = _gd_case(orc)
    mean, costs = orc.map_gd(g, mean0.astype(np.float32), var0, cam, pose, np.zeros_like(obs_d), obs_c,
                             orc.Params(), 0.01, 0.01, 3)
    assert costs == [0.0, 0.0, 0.0]
    assert np.array_equal(mean, mean0.astype(np.float32).astype(np.float64))


def test_map_gd_descends(orc):
    """With a small step the objective decreases at every step, and the
    first decrease matches the first-order prediction lr * |grad|^2."""
    _, g, cam, pose, mean0, var0, obs_d, obs_c = _gd_case(orc, seed=1)
    p = orc.Params(gate_geo=10.0, gate_rgb=10.0)
    lr_occ, lr_rgb = 2e-7, 1e-4
    mean, costs = orc.map_gd(g, mean0, var0, cam, pose, obs_d, obs_c, p, lr_occ, lr_rgb, 5, decide32=False,
                             store32=False)
    assert all(b < a for a, b in zip(costs, costs[1:])), costs
    _, g0 = orc.map_gd_objective(g, mean0, mean0, var0, cam, pose, obs_d, obs_c, p, decide32=False)
    pred = lr_occ * float(np.sum(g0[0] ** 2)) + lr_rgb * float(np.sum(g0[1:] ** 2))
    assert abs((costs[0] - costs[1]) - pred) < 0.05 * pred


# ---------------------------------------------------------------------------
# linear-Gaussian state filter (App. E)
# ---------------------------------------------------------------------------
def _transition_with_noise(orc, x, u, dt, n):
    """The generative transition of App. B with explicit noise: velocity
    integration (+ n_v), then pose integration with the new velocity
    (+ n_t on position, rotation perturbed by Exp(n_theta))."""
    v = x["v"] + u[:3] * dt + n[6:9]
    w = x["w"] + u[3:] * dt + n[9:12]
    t = x["t"] + v * dt + n[0:3]
    R = (Rotation.from_rotvec(n[3:6]) * Rotation.from_rotvec(w * dt) *
         Rotation.from_quat([x["q"][1], x["q"][2], x["q"][3], x["q"][0]])).as_matrix()
    return dict(t=t, R=R, v=v, w=w)


def _err(a, b):
    return np.concatenate([a["t"] - b["t"], Rotation.from_matrix(a["R"] @ b["R"].T).as_rotvec(),
                           a["v"] - b["v"], a["w"] - b["w"]])


def test_transition_linearisation_matches_fd(orc):
    """M and G of the linearised transition (App. E.1) against central
    differences of the generative transition in the error state."""
    rng = np.random.default_rng(2)
    q = Rotation.from_rotvec(rng.normal(size=3)).as_quat()
    x = dict(t=rng.normal(size=3), q=np.array([q[3], q[0], q[1], q[2]]),
             v=rng.normal(size=3), w=rng.normal(size=3))
    u = rng.normal(size=6)
    dt = 0.1
    xn = orc.transition_mean(x, u, dt)
    M, G = orc.transition_jacobians(xn, dt)
    base = _transition_with_noise(orc, x, u, dt, np.zeros(12))
    np.testing.assert_allclose(base["t"], xn["t"], atol=1e-14)
    np.testing.assert_allclose(base["R"], orc.quat_to_rot(xn["q"]), atol=1e-14)
    eps = 1e-6
    Mfd = np.zeros((12, 12)); Gfd = np.zeros((12, 12))
    Rx = Rotation.from_quat([q[0], q[1], q[2], q[3]])
    for i in range(12):
        for sgn in (1, -1):
            d = np.zeros(12); d[i] = sgn * eps
            R2 = (Rotation.from_rotvec(d[3:6]) * Rx).as_quat()
            xp = dict(t=x["t"] + d[0:3], q=np.array([R2[3], R2[0], R2[1], R2[2]]),
                      v=x["v"] + d[6:9], w=x["w"] + d[9:12])
            Mfd[:, i] += sgn * _err(_transition_with_noise(orc, xp, u, dt, np.zeros(12)), base) / (2 * eps)
            Gfd[:, i] += sgn * _err(_transition_with_noise(orc, x, u, dt, d), base) / (2 * eps)
    np.testing.assert_allclose(M, Mfd, atol=1e-7)
    np.testing.assert_allclose(G, Gfd, atol=1e-7)


def _rand_spd(rng, n):
    A = rng.normal(size=(n, n))
    return A @ A.T + n * np.eye(n)


def _adam_case(orc):
    c = synth.single_frame_case(0)
    mean, _ = synth.gt_map(c["scene"])
    g = orc.grid_from_scene(c["scene"])
    cam = orc.cam_from(c["cam"])
    pt = synth.pose7(c["t_gt"], c["q_gt"])
    p0 = synth.pose7(c["t_init"], c["q_init"])
    D, C = synth.raycast(c["scene"], c["cam"], c["t_gt"], c["q_gt"])
    anchor = orc.render(g, mean, cam, pt, normals=True)
    return cam, pt, p0, D, C, anchor


def test_adam_gradient_finite_differences(orc):
    """The optimiser's gradient (App. G sampled-pixel objective of Sec. 4.3.2)
    against central differences of
        scale * sum over sampled kept rows w r^2 + 1/2 e^T Lp e,
    with repeated and out-of-image indices in the sample; rows and decisions
    held.  The prior term is differenced along translation, where the pose
    error is exactly linear in the perturbation."""
    cam, pt, p0, D, C, anchor = _adam_case(orc)
    p = orc.Params()
    H, W = cam.height, cam.width
    rng = np.random.default_rng(4)
    pix = rng.integers(0, H * W, size=200).astype(np.int32)
    pix[:5] = pix[5:10]                     # repeats count twice
    pix[10] = H * W + 7                     # outside the image: no rows
    pix[11] = -3
    A = rng.normal(size=(6, 6))
    Lp = A @ A.T + 6 * np.eye(6)
    prior = _retract_np(p0, np.array([0.004, -0.002, 0.003, 0.0, 0.0, 0.0]))
    g = orc.adam_gradient(cam, p0, prior, Lp, pt, D, C, anchor, p, pix, decide32=False)
    wg, wc = 1 / p.b_geo ** 2, 1 / p.b_rgb ** 2
    valid = pix[(pix >= 0) & (pix < H * W)]
    scale = H * W / len(pix)

    def E(pose):
        o = orc.track_p2(cam, pose, pt, D, C, anchor, p, decide32=False)
        r = o["resid"].reshape(-1, 4)
        rm = o["rowmask"].reshape(-1)
        data = wg * np.sum((rm[valid] & 1 != 0) * r[valid, 0] ** 2)
        data += wc * np.sum((rm[valid] & 2 != 0)[:, None] * r[valid, 1:] ** 2)
        e = orc.pose_error(pose, prior)
        return scale * data + 0.5 * e @ Lp @ e, rm[valid].tobytes()

    eps = 1e-6
    for m in range(6):
        d = np.zeros(6); d[m] = eps
        ea, ka = E(_retract_np(p0, d))
        eb, kb = E(_retract_np(p0, -d))
        assert ka == kb
        fd = (ea - eb) / (2 * eps)
        if m < 3:
            assert abs(fd - g[m]) < 1e-4 * max(1.0, abs(g[m])), (m, fd, g[m])
        else:
            # rotation: the prior's pose error is linear only to first order
            e0 = orc.pose_error(p0, prior)
            assert abs(fd - g[m]) < 1e-4 * max(1.0, abs(g[m])) + np.abs(Lp @ e0).max() * 1e-2, (m, fd, g[m])


def test_adam_first_step_has_the_step_size(orc):
    """With bias correction and no momentum, the first step moves every
    component by its step size against the sign of its gradient."""
    cam, pt, p0, D, C, anchor = _adam_case(orc)
    p = orc.Params()
    pix = synth.sample_pixels(2, 1, 200, cam.height, cam.width)
    Lp = np.eye(6) * 1e-3
    g = orc.adam_gradient(cam, p0, p0, Lp, pt, D, C, anchor, p, pix[0])
    it = orc.adam_pose(cam, p0, Lp, pt, D, C, anchor, p, pix, 1e-3, 3.6e-4)
    d = orc.pose_error(it, p0)
    # a direction the sampled rows do not constrain (here vertical
    # translation in front of vertical walls) has a gradient at rounding
    # level, where the floor eps dominates the step
    live = np.abs(g) > 1e-6 * np.abs(g).max()
    assert live.sum() >= 5
    lr = np.array([1e-3] * 3 + [3.6e-4] * 3)
    np.testing.assert_allclose(d[live], (-np.sign(g) * lr)[live], rtol=1e-6)
    assert np.all(np.abs(d[~live]) < 1e-2 * lr[~live])


def test_adam_recovers_the_pose(orc):
    """App. G optimiser (200 pixels per step, step sizes 0.001 / 0.00036)
    from a 1.3 cm / 1.5 degree perturbation against an anchor rendered at the
    true pose: 300 steps bring the pose to within a few millimetres."""
    cam, pt, p0, D, C, anchor = _adam_case(orc)
    pix = synth.sample_pixels(1, 300, 200, cam.height, cam.width)
    it = orc.adam_pose(cam, p0, np.eye(6) * 1e-6, pt, D, C, anchor, orc.Params(), pix, 1e-3, 3.6e-4)
    e0, e = orc.pose_error(p0, pt), orc.pose_error(it, pt)
    assert np.linalg.norm(e0[:3]) > 0.01 and np.linalg.norm(e0[3:]) > 0.02
    assert np.linalg.norm(e[:3]) < 0.005 and np.linalg.norm(e[3:]) < 0.002, e


def test_split_and_combine_are_gaussian_identities(orc):
    """Marginal x conditional of a joint Gaussian reproduce the joint; the
    product of a pose posterior with the conditional has that posterior as
    its pose marginal and the conditional's (D, S) (Sec. 4.3.2, App. E.2)."""
    rng = np.random.default_rng(4)
    P = _rand_spd(rng, 12)
    Spp, D, Sv = orc.split(P)
    J = np.zeros((12, 12))
    J[:6, :6] = Spp
    J[:6, 6:] = Spp @ D.T
    J[6:, :6] = D @ Spp
    J[6:, 6:] = Sv + D @ Spp @ D.T
    np.testing.assert_allclose(J, P, rtol=1e-12, atol=1e-12)
    # conditional by the Schur complement of the precision matrix
    Lam = np.linalg.inv(P)
    np.testing.assert_allclose(Sv, np.linalg.inv(Lam[6:, 6:]), rtol=1e-10)
    np.testing.assert_allclose(D, -np.linalg.solve(Lam[6:, 6:], Lam[6:, :6]), rtol=1e-10, atol=1e-12)
    prior = np.array([0.1, 0.2, 0.3, 1.0, 0.0, 0.0, 0.0])
    post = orc.retract(prior, rng.normal(0, 0.01, 6))
    S_post = _rand_spd(rng, 6) * 1e-3
    mu_v = rng.normal(size=6)
    vm, Pj = orc.combine(post, S_post, prior, mu_v, D, Sv)
    np.testing.assert_allclose(Pj[:6, :6], S_post, rtol=1e-12)
    Sv2, D2 = orc.split(Pj)[2], orc.split(Pj)[1]
    np.testing.assert_allclose(D2, D, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(Sv2, Sv, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(vm, mu_v + D @ orc.pose_error(post, prior), rtol=1e-12)


def test_gn_and_laplace_equal_kalman_for_linear_measurements(orc):
    """For a linear-Gaussian measurement one Gauss-Newton step is the Kalman
    posterior mean and the Laplace covariance its covariance (Sec. 4.3.2;
    objective sum w r^2 = Gaussian with variance 1/(2w))."""
    rng = np.random.default_rng(6)
    m = 40
    Jm = rng.normal(size=(m, 6))
    r0 = rng.normal(size=m)
    w = rng.uniform(0.5, 3.0, m)
    neq = np.zeros(29)
    q = 0
    for a in range(6):
        for b in range(a, 6):
            neq[q] = np.sum(w * Jm[:, a] * Jm[:, b]); q += 1
    neq[21:27] = (w * r0) @ Jm
    P0 = _rand_spd(rng, 6) * 0.01
    Lp = np.linalg.inv(P0)
    e0 = rng.normal(0, 0.01, 6)
    delta = orc.gn_solve(neq, Lp, e0)
    S = orc.laplace(neq, Lp)
    # Kalman gain form: state x = prior offset, measurement 0 = r0 + J x, R = diag(1/(2w))
    Rm = np.diag(1.0 / (2 * w))
    x0 = -e0
    K = P0 @ Jm.T @ np.linalg.inv(Jm @ P0 @ Jm.T + Rm)
    x_post = x0 + K @ (-(r0 + Jm @ np.zeros(6)) - Jm @ x0)
    P_post = P0 - K @ Jm @ P0
    np.testing.assert_allclose(delta, x_post, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(S, P_post, rtol=1e-9, atol=1e-14)


@pytest.mark.slow
def test_filter_tracks_small_trajectory(orc):
    """Sanity (not parity): on a short synthetic trajectory (128^3 room,
    160x120 textured frames) the filter keeps the position error at the
    centimetre level."""
    case = synth.trajectory_case(seed=1, n=128, width=160, height=120, n_samples=64, n_frames=12)
    tr = case["traj"]
    g = orc.grid_from_scene(case["scene"])
    cam = orc.cam_from(case["cam"])
    n = g.n
    mean = np.zeros((4, n, n, n)); mean[0] = -0.001
    var = np.full((4, n, n, n), 1e4)
    x0 = dict(t=tr.t[0], q=tr.q[0], v=tr.v[0], w=tr.w[0])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    f = orc.Filter(g, cam, orc.Params(), x0, P0, mean, var)
    errs = []
    for i in range(len(tr.t)):
        f.step(case["depth"][i], case["rgb"][i], tr.u[i - 1] if i else None)
        errs.append(np.linalg.norm(f.s.t - tr.t[i]))
    assert max(errs) < 0.05


def _small_filter(orc, P0, n_frames=3):
    case = synth.trajectory_case(seed=3, n=32, width=40, height=30, n_samples=16, n_frames=n_frames)
    tr = case["traj"]
    g = orc.grid_from_scene(case["scene"])
    n = g.n
    mean = np.zeros((4, n, n, n)); mean[0] = -0.001
    var = np.full((4, n, n, n), 1e4)
    x0 = dict(t=tr.t[0], q=tr.q[0], v=tr.v[0], w=tr.w[0])
    f = orc.Filter(g, orc.cam_from(case["cam"]), orc.Params(), x0, P0, mean, var)
    return case, tr, f


def test_filter_without_data_is_pure_prediction(orc):
    """A frame with no valid depth carries no likelihood: the MAP pose is the
    prior mean, the Laplace covariance is the prior pose covariance, and the
    product with the velocity conditional rebuilds the predicted joint
    covariance exactly (Gaussian marginal/conditional identity)."""
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    case, tr, f = _small_filter(orc, P0)
    f.step(case["depth"][0], case["rgb"][0], None)
    s = f.s
    xn, Pm = orc.predict(dict(t=s.t, q=s.q, v=s.v, w=s.w), s.P, tr.u[0], f.p)
    mean_before = f.mean.copy()
    f.step(np.zeros_like(case["depth"][1]), case["rgb"][1], tr.u[0])
    assert f.s.last["n_updated"] == 0
    assert np.array_equal(f.mean, mean_before)
    assert np.all(f.s.last["neq"] == 0.0)
    np.testing.assert_allclose(f.s.t, xn["t"], rtol=0, atol=1e-15)
    assert orc.pose_error(f.s.pose, np.concatenate([xn["t"], xn["q"]])) == pytest.approx(np.zeros(6), abs=1e-15)
    np.testing.assert_allclose(np.concatenate([f.s.v, f.s.w]), np.concatenate([xn["v"], xn["w"]]), atol=1e-15)
    np.testing.assert_allclose(f.s.P, Pm, rtol=1e-9, atol=1e-18)


def test_filter_keeps_prediction_for_improper_covariance(orc):
    """A covariance whose predicted pose block is not positive definite
    defines no MAP problem: the step keeps the transition mean and the
    predicted covariance, and the map is still updated at that pose."""
    case, tr, f = _small_filter(orc, -np.eye(12))
    f.step(case["depth"][0], case["rgb"][0], None)
    s = f.s
    xn, Pm = orc.predict(dict(t=s.t, q=s.q, v=s.v, w=s.w), s.P, tr.u[0], f.p)
    assert np.all(np.linalg.eigvalsh(Pm[:6, :6]) < 0)
    f.step(case["depth"][1], case["rgb"][1], tr.u[0])
    assert f.s.last["prior_not_pd"]
    assert f.s.last["n_updated"] > 0
    for k in "tqvw":
        assert np.array_equal(getattr(f.s, k), xn[k])
    assert np.array_equal(f.s.P, Pm)
    assert np.array_equal(f.s.anchor_pose, np.concatenate([xn["t"], xn["q"]]))


# ---------------------------------------------------------------------------
# predictive rollouts (App. J)
# ---------------------------------------------------------------------------
def _rollout_belief(rng):
    x = dict(t=np.array([1.0, 2.0, 1.5]), q=np.array([0.9, 0.1, -0.2, 0.3]) / np.linalg.norm([0.9, 0.1, -0.2, 0.3]),
             v=np.array([0.3, -0.1, 0.05]), w=np.array([0.2, 0.4, -0.3]))
    A = rng.normal(size=(12, 12)) * 0.01
    P = A @ A.T + np.diag([1e-5] * 6 + [1e-4] * 6)
    u = rng.normal(size=(5, 6))
    return x, P, u


def test_rollout_without_noise_follows_the_predicted_mean(orc):
    """Zero draws: every sampled trajectory is the noise-free transition of
    the mean, i.e. the closed-form predicted means."""
    rng = np.random.default_rng(0)
    x, P, u = _rollout_belief(rng)
    out = orc.rollout(None, None, None, x, P, u, np.zeros((2, 6, 12)), orc.Params(), frames=False)
    for s in range(2):
        np.testing.assert_allclose(out["poses"][s, :, :3], out["mean"][:, :3], rtol=0, atol=1e-12)
        for j in range(5):
            assert np.linalg.norm(orc.pose_error(out["poses"][s, j], out["mean"][j, :7])) < 1e-12


def test_rollout_samples_match_the_linearised_moments(orc):
    """Monte Carlo over the generative transition: the sampled poses' mean
    and covariance (tangent at the predicted mean) agree with the closed-form
    linearised prediction within sampling error."""
    rng = np.random.default_rng(1)
    x, P, u = _rollout_belief(rng)
    S = 3000
    out = orc.rollout(None, None, None, x, P, u, rng.normal(size=(S, 6, 12)), orc.Params(), frames=False)
    for j in (0, 4):
        e = np.array([orc.pose_error(out["poses"][s, j], out["mean"][j, :7]) for s in range(S)])
        C = out["cov"][j][:6, :6]
        sd = np.sqrt(np.diag(C))
        assert np.all(np.abs(e.mean(0)) < 4 * sd / np.sqrt(S) + 1e-3 * sd)
        Ce = np.cov(e.T)
        assert np.linalg.norm(Ce - C) < 0.1 * np.linalg.norm(C), (j, np.linalg.norm(Ce - C) / np.linalg.norm(C))


def test_rollout_improper_covariance_starts_at_the_mean(orc):
    rng = np.random.default_rng(2)
    x, _, u = _rollout_belief(rng)
    z = rng.normal(size=(1, 6, 12))
    z[:, 1:] = 0.0
    out = orc.rollout(None, None, None, x, -np.eye(12), u, z, orc.Params(), frames=False)
    assert not out["ok"]
    assert np.linalg.norm(orc.pose_error(out["poses"][0, 0], out["mean"][0, :7])) < 1e-12


# ---------------------------------------------------------------------------
# App. G.2 Laplace average and App. E.3 / G.3 anchor normals
# ---------------------------------------------------------------------------
def test_laplace_average_enters_the_state_covariance(orc):
    """App. G: the Laplace pose covariances are smoothed by an exponential
    moving average with coefficient 0.8 on the previous average, the first
    average being the first Laplace covariance; the averaged covariance is
    the pose block of the combined state belief (Sec. 4.3.2 product with
    the velocity conditional).  Each Laplace covariance is formed here from
    the recorded normal equations and the predicted pose precision,
    (2 H + Lp)^-1, independently of the filter's own code path."""
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    case, tr, f = _small_filter(orc, P0, n_frames=4)
    f.step(case["depth"][0], case["rgb"][0], None)
    assert f.s.Sbar is None                      # the first frame has no pose update
    laps = []
    for i in (1, 2, 3):
        s = f.s
        _, Pm = orc.predict(dict(t=s.t, q=s.q, v=s.v, w=s.w), s.P, tr.u[i - 1], f.p)
        Lp = np.linalg.inv(Pm[:6, :6])
        f.step(case["depth"][i], case["rgb"][i], tr.u[i - 1])
        neq = f.s.last["neq"]
        assert neq[28] > 100
        H = np.zeros((6, 6))
        H[np.triu_indices(6)] = neq[:21]
        H = H + np.triu(H, 1).T
        laps.append(np.linalg.inv(2.0 * H + Lp))
        if i == 1:
            expect = laps[0]
        else:
            expect = 0.8 * prev + 0.2 * laps[-1]
            swapped = 0.2 * prev + 0.8 * laps[-1]
            # the two weightings differ well beyond the tolerance below
            assert np.linalg.norm(swapped - expect) > 1e-4 * np.linalg.norm(expect)
        np.testing.assert_allclose(f.s.Sbar, expect, rtol=1e-8, atol=1e-8 * np.abs(expect).max())
        np.testing.assert_allclose(f.s.P[:6, :6], expect, rtol=1e-8, atol=1e-8 * np.abs(expect).max())
        prev = expect


def _plane_depth(cam, nrm, c):
    """z-depth image of the plane nrm . X = c seen from the camera origin."""
    u = (np.arange(cam.width) + 0.5 - cam.cx) / cam.fx
    v = (np.arange(cam.height) + 0.5 - cam.cy) / cam.fy
    rx, ry = np.meshgrid(u, v)
    return c / (nrm[0] * rx + nrm[1] * ry + nrm[2])


def test_anchor_normals_validity_and_plane_normal(orc):
    """App. E.3: the anchor normal is the normal of the rendered depth image;
    App. G: depth discontinuities are ignored.  On a constructed image of
    two tilted planes with a 0.5 m step between the left and right halves,
    a 0.05 m step inside the left half, and two invalid pixels, the valid
    set is known from the construction: not the border, not an invalid pixel
    or one of its four neighbours, not a pixel next to the 0.5 m step (the
    0.05 m step stays below the 0.1 m threshold).  Away from both steps the
    normal is the plane's unit normal, oriented towards the camera."""
    W, H = 40, 30
    cam = orc.Cam(W, H, 30.0, 30.0, 20.0, 15.0, 0.1, 5.0, 16)
    nrm = np.array([0.3, -0.2, -1.0])
    nrm /= np.linalg.norm(nrm)
    cA = -1.5                                      # plane nrm . X = c, about 1.5 m away
    dA = _plane_depth(cam, nrm, cA)
    dB = _plane_depth(cam, nrm, cA - 0.5)          # 0.5 m further along the normal
    dS = _plane_depth(cam, nrm, cA - 0.05)         # 0.05 m further
    depth = dA.copy()
    depth[:, 20:] = dB[:, 20:]
    depth[22:, :20] = dS[22:, :20]
    mask = np.ones((H, W), np.uint8)
    holes = [(10, 5), (20, 30)]                    # (v, u)
    for v, u in holes:
        mask[v, u] = 0
        depth[v, u] = 0.0
    assert np.all(np.abs(depth[:, 20] - depth[:, 19]) > 0.1)
    assert np.all(np.abs(depth[22, :20] - depth[21, :20]) < 0.1)
    expect = np.ones((H, W), np.uint8)
    expect[0, :] = expect[-1, :] = 0
    expect[:, 0] = expect[:, -1] = 0
    expect[:, 19:21] = 0                           # a neighbour across the 0.5 m step
    for v, u in holes:
        for dv, du in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
            expect[v + dv, u + du] = 0
    n_out, nmask = orc.normals_of(cam, depth, mask, 0.1)
    np.testing.assert_array_equal(nmask, expect)
    # the camera (origin) lies where nrm . X - c has the sign of -c, so the
    # plane normal pointing to the camera's side is sign(-c) nrm
    facing = nrm if cA < 0 else -nrm
    flat = expect.astype(bool).copy()
    flat[20:24, :20] = False                       # stencils straddling the small step
    err = np.abs(n_out[flat] - facing).max()
    assert err < 1e-9, err
    # facing the camera: the normal opposes the back-projected point
    rx = (np.arange(W) + 0.5 - cam.cx) / cam.fx
    ry = (np.arange(H) + 0.5 - cam.cy) / cam.fy
    Pt = depth[..., None] * np.stack([*np.meshgrid(rx, ry), np.ones((H, W))], -1)
    assert np.all(np.einsum("ij,ij->i", n_out[flat], Pt[flat]) < 0)
    assert np.all(n_out[~expect.astype(bool)] == 0.0)
