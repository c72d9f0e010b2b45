"""HIP library against the FP64 oracle, element by element, at the sizes the
throughput figures are measured on, plus the parity tier with double-
precision decisions.

* Render Jacobian (P1) and tracking (P2): row masks exactly, every Jacobian
  entry against its row, residuals, and the 29 normal-equation entries one by
  one (scales in gpu_util.neq_check), at 80x60 and at the 8-frame
  256^3 / 320x240 / K = 128 call of the render+Jacobian throughput figure.
* Anchor normals: the GPU normals kernel and the oracle's normals on the same
  rendered depth image, mask bit for bit.
* Adjoint: every component of the pose gradient and every voxel of the map
  gradient, at 80x60 and at the 8-frame 256^3 / 320x240 / K = 128 call of
  the adjoint throughput figure.
* Double-precision decisions: the oracle with every decision in FP64 (not
  the kernels' single-precision recipe); a hit sample, updated voxel or
  tracking row may differ only where the FP64 decision margin is below 1e-4
  relative, and such flips are counted and printed.
* The FP32 filter at the single-stream trajectory size (256^3, 320x240,
  K = 128) for 6 frames, and brick-pool maps smaller than the grid against
  the oracle.
* Descent mapping (one step), the rollout (16 x 10, sampled frames) and
  filter steps with the paper's optimiser (1000 x 200 pixels) at 256^3 /
  320x240 / K = 128.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import oracle as orc
import synth
from gpu_util import (DEV, banner, cam_of, depth_close, gpu_map, grid_of, neq_check, oracle_map_values, rgb_close,
                      rot_angle, rows_check, t, P)

pytestmark = pytest.mark.gpu

MARGIN = 1e-4    # FP64 decision margin (relative) above which no flip is allowed


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P().lib()
    yield


@pytest.fixture(scope="module")
def small():
    c = synth.single_frame_case(0)
    mean, var = synth.gt_map(c["scene"])
    return c, mean, var


@pytest.fixture(scope="module")
def big():
    """The single-stream trajectory room: 256^3 (2.5 cm), 320x240, K = 128,
    8 frames of the trajectory with depth noise 1 cm and colour noise 0.02;
    the map holds the ground-truth means (FP32)."""
    c = synth.trajectory_case(seed=1, n=256, width=320, height=240, n_samples=128, n_frames=8)
    mean, var = synth.gt_map(c["scene"], dtype=np.float32)
    return c, mean, var


def _np_anchor(a):
    a32 = {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in a.items()}
    a64 = {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in a32.items()}
    dev = {k: t(v, torch.uint8 if v.dtype == np.uint8 else torch.float32) for k, v in a32.items()
           if k in ("depth", "rgb", "mask", "normals", "nmask")}
    return a64, dev


# ---------------------------------------------------------------------------
# P1: render Jacobian
# ---------------------------------------------------------------------------
def _p1_compare(out, ref, i, label):
    rm = out["rowmask"][i].cpu().numpy()
    np.testing.assert_array_equal(out["mask"][i].cpu().numpy(), ref["mask"], err_msg=label)
    np.testing.assert_array_equal(rm, ref["rowmask"], err_msg=f"{label}: row masks")
    use = rm > 0
    J = out["J"][i].cpu().numpy()
    rows_check(J[use], ref["J"][use], label)
    assert np.all(J[~use] == 0)
    r = out["resid"][i].cpu().numpy()
    # residuals: single-precision roundings of the double-precision values
    assert np.all(np.abs(r[use] - ref["resid"][use]) <= 1e-6 * np.maximum(np.abs(ref["resid"][use]), 1.0)), label
    neq_check(out["neq"][i].cpu().numpy(), ref["neq"], label)


@pytest.mark.parametrize("dtype", [0, 1])
def test_render_jacobian_per_element(small, dtype):
    banner(f"render_jacobian per element, 64^3 80x60, dtype {dtype}")
    c, mean, _ = small
    g = grid_of(c["scene"], dtype)
    cam = cam_of(c["cam"])
    vm = gpu_map(g, mean, np.full_like(mean, 1e-2))
    od, oc = synth.raycast(c["scene"], c["cam"], c["t_gt"], c["q_gt"], np.random.default_rng(3), 0.01, 0.02)
    od = od.astype(np.float32); oc = oc.astype(np.float32)
    pose = synth.pose7(c["t_init"], c["q_init"])
    out = P().render_jacobian(g, vm, cam, P().poses_tensor(pose), t(od)[None], t(oc)[None], P().Weights.make(),
                              want_J=True, want_resid=True)
    torch.cuda.synchronize()
    ref = orc.render_jacobian(orc.grid_from_scene(c["scene"]), oracle_map_values(mean, dtype),
                              orc.cam_from(c["cam"]), pose, od, oc, orc.Params(), want_J=True)
    _p1_compare(out, ref, 0, f"P1 80x60 dtype {dtype}")


def test_render_jacobian_8_frames_full_size(big):
    """The call behind the render+Jacobian throughput figure: 8 frames in one
    launch, 256^3 FP32, 320x240, K = 128 (1200 workgroups per frame, so the
    final sum of partials takes two rounds)."""
    banner("render_jacobian per element, 8 frames 256^3 320x240 K=128")
    c, mean, _ = big
    tr = c["traj"]
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    vm = gpu_map(g, mean, np.full_like(mean, 1e-2))
    rng = np.random.default_rng(21)
    poses = np.stack([synth.pose7(*synth.perturb_pose(rng, tr.t[i], tr.q[i], 0.01, 0.01)) for i in range(8)])
    od = c["depth"][:8]; oc = c["rgb"][:8]
    out = P().render_jacobian(g, vm, cam, P().poses_tensor(poses), t(od), t(oc), P().Weights.make(),
                              want_J=True, want_resid=True)
    torch.cuda.synchronize()
    og, ocm, m64 = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"]), mean.astype(np.float64)
    for i in range(8):
        ref = orc.render_jacobian(og, m64, ocm, poses[i], od[i], oc[i], orc.Params(), want_J=True)
        assert ref["neq"][28] > 30000
        _p1_compare(out, ref, i, f"P1 frame {i} of 8")


# ---------------------------------------------------------------------------
# P2: tracking
# ---------------------------------------------------------------------------
def _p2_case(c, mean, prev, rng, obs=None):
    a64, adev = _np_anchor(orc.render(orc.grid_from_scene(c["scene"]), mean, orc.cam_from(c["cam"]), prev,
                                      normals=True))
    if obs is None:
        tt, qq = synth.perturb_pose(rng, prev[:3], prev[3:], 0.03, 0.03)
        od, oc = synth.raycast(c["scene"], c["cam"], tt, qq, rng, 0.01, 0.02)
    else:
        tt, qq = obs[2], obs[3]
        od, oc = obs[0], obs[1]
    od = od.astype(np.float32); oc = oc.astype(np.float32)
    cur = synth.pose7(*synth.perturb_pose(rng, tt, qq, 0.01, 0.01))
    return a64, adev, od, oc, cur


@pytest.mark.parametrize("size", ["80x60", "320x240"])
def test_track_p2_per_element(small, big, size):
    banner(f"track_p2 per element, {size}")
    c, mean, _ = small if size == "80x60" else big
    rng = np.random.default_rng(4)
    if size == "80x60":
        prev = synth.pose7(c["t_gt"], c["q_gt"])
        a64, adev, od, oc, cur = _p2_case(c, mean.astype(np.float32).astype(np.float64), prev, rng)
    else:
        tr = c["traj"]
        prev = synth.pose7(tr.t[2], tr.q[2])
        a64, adev, od, oc, cur = _p2_case(c, mean.astype(np.float64), prev, rng,
                                          obs=(c["depth"][3], c["rgb"][3], tr.t[3], tr.q[3]))
    cam = cam_of(c["cam"])
    out = P().track_p2(cam, P().poses_tensor(cur), P().poses_tensor(prev), t(od), t(oc), adev, P().Weights.make(),
                       want_J=True, want_resid=True)
    torch.cuda.synchronize()
    ref = orc.track_p2(orc.cam_from(c["cam"]), cur, prev, od, oc, a64, orc.Params(), want_J=True)
    rm = out["rowmask"].cpu().numpy()
    np.testing.assert_array_equal(rm, ref["rowmask"], err_msg="P2 row masks")
    use = rm > 0
    assert use.sum() > 1000
    J = out["J"].cpu().numpy()
    rows_check(J[use], ref["J"][use], f"P2 {size}")
    r = out["resid"].cpu().numpy()
    assert np.all(np.abs(r[use] - ref["resid"][use]) <= 1e-6 * np.maximum(np.abs(ref["resid"][use]), 1.0))
    neq_check(out["neq"][0].cpu().numpy(), ref["neq"], f"P2 {size}")


# ---------------------------------------------------------------------------
# anchor normals
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("size", ["80x60", "320x240"])
def test_anchor_normals_bit_exact_mask(small, big, size):
    """The normals kernel against the oracle's normals on the same rendered
    depth image and mask.  The kernel tests |d(nbr) - d| > 0.1 in single
    precision: a pixel whose double-precision difference lies within 1e-6 of
    the threshold may go either way (counted; none is expected)."""
    banner(f"anchor normals, mask bit for bit, {size}")
    c, mean, _ = small if size == "80x60" else big
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    vm = gpu_map(g, mean, np.full_like(mean, 1e-2))
    if size == "80x60":
        poses = [synth.pose7(c["t_gt"], c["q_gt"]), synth.pose7(c["t_init"], c["q_init"])]
    else:
        poses = [synth.pose7(c["traj"].t[i], c["traj"].q[i]) for i in (0, 5)]
    out = P().render(g, vm, cam, P().poses_tensor(np.stack(poses)), normals=True)
    torch.cuda.synchronize()
    ocm = orc.cam_from(c["cam"])
    for i in range(len(poses)):
        d = out["depth"][i].cpu().numpy().astype(np.float64)
        m = out["mask"][i].cpu().numpy()
        nref, mref = orc.normals_of(ocm, d, m, 0.1)
        nm = out["nmask"][i].cpu().numpy()
        # pixels with a neighbour difference within 1e-6 of the threshold
        H, W = d.shape
        near = np.zeros((H, W), bool)
        for dv, du in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            sh = np.roll(np.roll(d, -dv, 0), -du, 1)
            near |= np.abs(np.abs(sh - d) - 0.1) <= 1e-6
        diff = nm != mref
        print(f"[normals {size} pose {i}] valid {int(mref.sum())}, mask flips {int(diff.sum())} "
              f"(near the threshold {int((diff & near).sum())})", flush=True)
        assert not np.any(diff & ~near), f"normal mask differs away from the threshold ({int((diff & ~near).sum())})"
        both = (nm == 1) & (mref == 1)
        assert both.sum() > 0.3 * m.sum()
        nrm = out["normals"][i].cpu().numpy()
        err = np.abs(nrm[both] - nref[both]).max()
        print(f"[normals {size} pose {i}] max normal error {err:.2e}", flush=True)
        assert err <= 1e-4, err
        assert np.all(nrm[nm == 0] == 0)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def test_render_vjp_per_element(small):
    """Pose gradient: each component against its accumulation scale, the sum
    over rays and rows of |J row| |upstream| (the rows are single precision,
    so a component that cancels is judged against the rows it sums), with
    the rows from the oracle's Jacobian.  Map gradient: each voxel and
    channel relatively, with a floor of 1e-3 of the channel's largest
    gradient for entries that cancel."""
    banner("render_vjp per element, 64^3 80x60")
    c, mean, _ = small
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    m32 = mean.astype(np.float32).astype(np.float64)
    vm = gpu_map(g, mean, np.full_like(mean, 1e-2))
    pose = synth.pose7(c["t_init"], c["q_init"])
    pt = P().poses_tensor(pose)
    fwd = P().render(g, vm, cam, pt, hit_k=True)
    rng = np.random.default_rng(6)
    H, W = cam.height, cam.width
    gd = rng.normal(size=(1, H, W)).astype(np.float32)
    gc = rng.normal(size=(1, H, W, 3)).astype(np.float32)
    gm, gp = P().render_vjp(g, vm, cam, pt, fwd["hit_k"], t(gd), t(gc))
    gm = P().bricks_to_dense(g.n, gm).cpu().numpy().astype(np.float64)
    gp = gp[0].cpu().numpy()
    torch.cuda.synchronize()
    og, ocm = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
    rgm, rgp = orc.render_vjp(og, m32, ocm, pose, gd[0], gc[0])
    # every valid ray's Jacobian: observations equal to the render keep every row
    r = orc.render(og, m32, ocm, pose)
    full = orc.render_jacobian(og, m32, ocm, pose, np.where(r["mask"] == 1, r["depth"], 0.0), r["rgb"],
                               orc.Params(), want_J=True)
    assert int(full["neq"][28]) == int(r["mask"].sum())
    up = np.concatenate([gd[0][..., None], gc[0]], -1).astype(np.float64)        # [H, W, 4]
    scale = float(np.sum(np.linalg.norm(full["J"], axis=-1) * np.abs(up)))
    # the oracle's own J^T g equals its adjoint (identity pinned on the CPU)
    np.testing.assert_allclose(np.einsum("hwrc,hwr->c", full["J"], up), rgp, rtol=0, atol=1e-12 * scale)
    ep = np.abs(gp - rgp) / scale
    print(f"[vjp pose] max error / accumulation scale {ep.max():.2e} (scale {scale:.3e}; |grad| "
          f"{np.abs(rgp).round(4).tolist()})", flush=True)
    assert ep.max() <= 1e-6, ep
    nz = (rgm != 0) | (gm != 0)
    assert nz.sum() > 1000
    cmax = np.abs(rgm).reshape(4, -1).max(1)[:, None, None, None]
    em = np.abs(gm - rgm) / np.maximum(np.abs(rgm), 1e-2 * cmax)
    e3 = np.abs(gm - rgm) / np.maximum(np.abs(rgm), 1e-3 * cmax)
    w = np.unravel_index(np.argmax(np.where(nz, em, 0)), em.shape)
    print(f"[vjp map] {int(nz.sum())} entries, max scaled error {em[nz].max():.2e} (floor 1e-2 of the channel "
          f"maximum; with 1e-3: {e3[nz].max():.2e}, 99.9% {np.quantile(e3[nz], 0.999):.2e}); worst: channel "
          f"{w[0]}, |grad| / channel max {abs(rgm[w]) / cmax[w[0], 0, 0, 0]:.2e}", flush=True)
    assert em[nz].max() <= 1e-4, em[nz].max()


def test_render_vjp_8_frames_full_size(big):
    """The call behind the adjoint throughput figure: 8 frames in one launch,
    256^3 FP32 (ground-truth means), 320x240, K = 128, upstream gradients
    N(0, 1) on every output.  Pose gradient of each frame against its
    accumulation scale; the map gradient, summed over the 8 frames, voxel by
    voxel with a floor of 1e-2 of the channel's largest gradient."""
    banner("render_vjp per element, 8 frames 256^3 320x240 K=128")
    c, mean, _ = big
    tr = c["traj"]
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    vm = gpu_map(g, mean, np.full_like(mean, 1e-2))
    rng = np.random.default_rng(22)
    poses = np.stack([synth.pose7(*synth.perturb_pose(rng, tr.t[i], tr.q[i], 0.01, 0.01)) for i in range(8)])
    pt = P().poses_tensor(poses)
    H, W = cam.height, cam.width
    gd = rng.normal(size=(8, H, W)).astype(np.float32)
    gc = rng.normal(size=(8, H, W, 3)).astype(np.float32)
    fwd = P().render(g, vm, cam, pt, hit_k=True)
    gm, gp = P().render_vjp(g, vm, cam, pt, fwd["hit_k"], t(gd), t(gc))
    gm = P().bricks_to_dense(g.n, gm).cpu().numpy().reshape(4, -1)
    gp = gp.cpu().numpy()
    torch.cuda.synchronize()
    og, ocm, m64 = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"]), mean.astype(np.float64)
    rgm = np.zeros((4, g.n ** 3))
    for i in range(8):
        fm, fp = orc.render_vjp(og, m64, ocm, poses[i], gd[i], gc[i])
        rgm += fm.reshape(4, -1)
        del fm
        r = orc.render(og, m64, ocm, poses[i])
        full = orc.render_jacobian(og, m64, ocm, poses[i], np.where(r["mask"] == 1, r["depth"], 0.0), r["rgb"],
                                   orc.Params(), want_J=True)
        assert int(full["neq"][28]) == int(r["mask"].sum()) > 30000
        up = np.concatenate([gd[i][..., None], gc[i]], -1).astype(np.float64)
        scale = float(np.sum(np.linalg.norm(full["J"], axis=-1) * np.abs(up)))
        ep = np.abs(gp[i] - fp) / scale
        print(f"[vjp pose, frame {i}] max error / accumulation scale {ep.max():.2e}", flush=True)
        assert ep.max() <= 1e-6, (i, ep)
    nz = np.nonzero((rgm != 0) | (gm != 0))
    assert nz[0].size > 100000
    cmax = np.abs(rgm).max(1)
    a, b = rgm[nz], gm[nz].astype(np.float64)
    em = np.abs(b - a) / np.maximum(np.abs(a), 1e-2 * cmax[nz[0]])
    print(f"[vjp map, 8 frames] {nz[0].size} entries, max scaled error {em.max():.2e}", flush=True)
    assert em.max() <= 1e-4, em.max()


def test_map_gd_full_size(big):
    """Descent mapping at the size of the closed-form comparison: 256^3 FP32,
    320x240, K = 128, one step from a perturbed previous belief (means of
    the ground truth plus noise, variances U[0.5, 2]); the objective and every
    mean after the step against the oracle (the same decisions on both
    sides)."""
    banner("map_gd 256^3 320x240 K=128, 1 step")
    c, mean, _ = big
    tr = c["traj"]
    rng = np.random.default_rng(23)
    m0 = (mean + np.concatenate([rng.normal(0, 0.01, (1,) + mean.shape[1:]),
                                 rng.normal(0, 0.05, (3,) + mean.shape[1:])]).astype(np.float32)).astype(np.float32)
    v0 = rng.uniform(0.5, 2.0, m0.shape).astype(np.float32)
    pose = synth.pose7(tr.t[3], tr.q[3])
    od, oc = c["depth"][3], c["rgb"][3]
    g = grid_of(c["scene"], 0)
    cam = cam_of(c["cam"])
    p = orc.Params()
    w = P().Weights.make(p.b_geo, p.b_rgb, p.gate_geo, p.gate_rgb)
    lro, lrc = 3e-6, 3e-3
    vm = gpu_map(g, m0, v0)
    ws = P().map_gd_workspace(g, cam)
    cost = torch.zeros(1, dtype=torch.float64, device=DEV)
    P().map_gd(g, vm, cam, P().poses_tensor(pose), t(od), t(oc), w, lro, lrc, 1, ws, cost)
    mg, _ = vm.to_dense()
    mg = mg.cpu().numpy()
    cg = float(cost.cpu().numpy()[0])
    torch.cuda.synchronize()
    ref, rcost = orc.map_gd(orc.grid_from_scene(c["scene"]), m0.astype(np.float64), v0.astype(np.float64),
                            orc.cam_from(c["cam"]), pose, od, oc, p, lro, lrc, 1)
    print(f"cost gpu {cg} oracle {rcost[0]}", flush=True)
    assert abs(cg - rcost[0]) <= 1e-5 * abs(rcost[0])
    moved = ref != m0
    err = np.abs(mg.astype(np.float64) - ref)
    print(f"voxels moved {int(moved.sum())}, max err {err.max():.3e}", flush=True)
    assert moved.sum() > 100000
    assert np.all(err <= 1e-6 * np.maximum(np.abs(ref), 1e-2))
    assert np.array_equal(mg[~moved], m0[~moved])


def test_rollout_full_size(big):
    """The rollout of the throughput figure: 16 sampled trajectories x 10
    steps with moments and every predicted frame, 256^3 FP32 (ground-truth
    means), 320x240, K = 128.  Every sampled pose and the moments against the
    oracle; four of the 160 frames (first and last steps of two
    trajectories) against the oracle's render at its own sampled pose, mask
    bit for bit."""
    banner("rollout 256^3 320x240 K=128, 16 samples x 10 steps")
    c, mean, var = big
    tr = c["traj"]
    g = grid_of(c["scene"], 0)
    cam = cam_of(c["cam"])
    f = P().Filter(g, cam, P().FilterParams(objective=0), vmap=gpu_map(g, mean, var))
    rng = np.random.default_rng(24)
    A = rng.normal(size=(12, 12)) * 0.01
    Pb = A @ A.T + np.diag([1e-5] * 6 + [1e-4] * 6)
    x = dict(t=tr.t[2], q=tr.q[2], v=tr.v[2], w=tr.w[2])
    f.reset(np.concatenate([x["t"], x["q"], x["v"], x["w"]]), Pb)
    k, S = 10, 16
    u = rng.normal(size=(k, 6))
    z = rng.normal(size=(S, k + 1, 12))
    out = f.rollout(t(u, torch.float64), t(z, torch.float64), moments=True, frames=True)
    torch.cuda.synchronize()
    og, ocm = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
    ref = orc.rollout(og, None, ocm, x, Pb, u, z, orc.Params(), frames=False)
    assert int(out["flags"].item()) == 0 and ref["ok"]
    pg = out["poses"].cpu().numpy()
    err = max(np.linalg.norm(orc.pose_error(pg[s, j], ref["poses"][s, j])) for s in range(S) for j in range(k))
    print(f"[rollout] max pose error over {S * k} poses {err:.2e}", flush=True)
    assert err < 1e-9
    np.testing.assert_allclose(out["mean"].cpu().numpy(), ref["mean"], rtol=0, atol=1e-12)
    cg = out["cov"].cpu().numpy()
    assert np.linalg.norm(cg - ref["cov"]) <= 1e-10 * np.linalg.norm(ref["cov"])
    m64 = mean.astype(np.float64)
    for s, j in ((0, 0), (0, k - 1), (S - 1, 0), (S - 1, k - 1)):
        n = s * k + j
        r = orc.render(og, m64, ocm, ref["poses"][s, j])
        mk = out["mask"][n].cpu().numpy()
        np.testing.assert_array_equal(mk, r["mask"], err_msg=f"frame of sample {s}, step {j}")
        v = mk == 1
        assert v.sum() > 1000
        assert np.all(depth_close(out["depth"][n].cpu().numpy()[v], r["depth"][v]))
        assert np.all(rgb_close(out["rgb"][n].cpu().numpy()[v], r["rgb"][v]))


def test_filter_adam_full_size(big):
    """The paper's optimiser at its own settings (1000 steps of 200 sampled
    pixels) in filter steps at 256^3 FP32, 320x240, K = 128: two steps from
    the prior map against the oracle filter on the same frames and samples."""
    banner("filter adam 256^3 320x240 K=128, 2 steps x 1000 Adam steps")
    c, _, _ = big
    tr = c["traj"]
    n = c["scene"].n
    g = grid_of(c["scene"], 0)
    f = P().Filter(g, cam_of(c["cam"]), P().FilterParams(objective=0))
    f.map.init()
    x0 = np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    f.reset(x0, P0)
    mean = np.zeros((4, n, n, n)); mean[0] = np.float32(-0.001)
    of = orc.Filter(orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"]), orc.Params(objective="p2"),
                    dict(t=tr.t[0], q=tr.q[0], v=tr.v[0], w=tr.w[0]), P0, mean, np.full_like(mean, 1e4))
    del mean
    ap = P().AdamParams.make(n_steps=1000, n_pixels=200)
    H, W = c["cam"].height, c["cam"].width
    for i in range(3):
        pix = synth.sample_pixels(30 + i, ap.n_steps, ap.n_pixels, H, W)
        u = tr.u[i - 1] if i else None
        f.step_adam(t(c["depth"][i]), t(c["rgb"][i]), t(u, torch.float64) if i else None, ap,
                    t(pix, torch.int32))
        of.step(c["depth"][i].astype(np.float64), c["rgb"][i].astype(np.float64), u,
                adam=dict(pixels=pix, lr_t=ap.lr_t, lr_r=ap.lr_r, beta2=ap.beta2, eps=ap.eps))
        s = f.state()
        dt_ = np.linalg.norm(np.array(s.pose.t) - of.s.t)
        dr = rot_angle(np.array(s.pose.q), of.s.q)
        print(f"step {i}: flags {s.flags} |dt| {dt_:.3e} dR {dr:.3e}", flush=True)
        assert s.flags == 0
        assert dt_ <= 1e-5 and dr <= 1e-5
        Pg = np.array(s.P).reshape(12, 12)
        assert np.linalg.norm(Pg - of.s.P) <= 1e-4 * np.linalg.norm(of.s.P)


# ---------------------------------------------------------------------------
# double-precision decisions (tier ii)
# ---------------------------------------------------------------------------
def _sample_occupancy(mean0, og, cam, pose, vs, us):
    """FP64 occupancy at every sample of the given rays: scipy's linear
    interpolation with the outside value as constant padding."""
    K = cam.n_samples
    ds = cam.d_near + np.arange(K) * (cam.d_far - cam.d_near) / (K - 1)
    R = orc.quat_to_rot(pose[3:])
    rc = np.stack([(us + 0.5 - cam.cx) / cam.fx, (vs + 0.5 - cam.cy) / cam.fy, np.ones(len(us))], -1)
    dirs = rc @ R.T
    pts = pose[:3] + ds[None, :, None] * dirs[:, None, :]                      # [rays, K, 3]
    gcrd = (pts - np.asarray(og.origin)) / og.voxel - 0.5
    coords = gcrd.reshape(-1, 3)[:, ::-1].T
    f = ndi.map_coordinates(mean0, coords, order=1, mode="grid-constant", cval=og.occ_out)
    return f.reshape(len(us), K)


def _render_flips(og, ocm, mean, pose, out_hit, label):
    ref = orc.render(og, mean, ocm, pose, decide32=False)
    hk = ref["hit_k"]
    flip = out_hit != hk
    vs, us = np.nonzero(flip)
    scale = np.abs(mean[0]).max()
    margins = []
    if len(us):
        f = _sample_occupancy(mean[0], og, ocm, pose, vs, us)
        for j in range(len(us)):
            a, b = int(out_hit[vs[j], us[j]]), int(hk[vs[j], us[j]])
            last = max(a, b) if min(a, b) >= 0 else ocm.n_samples - 1
            margins.append(np.abs(f[j, :last + 1] - ocm.tau).min() / scale)
    margins = np.array(margins)
    print(f"[tier ii render {label}] {hk.size} rays, hit flips {len(margins)}, largest flip margin "
          f"{margins.max() if len(margins) else 0.0:.1e}", flush=True)
    assert np.all(margins <= MARGIN), margins
    return ref, flip


def test_fp64_decisions_render(small, big):
    banner("tier ii: render hit samples with FP64 decisions")
    for name, (c, mean, _), idx in (("64^3 80x60", small, None), ("256^3 320x240", big, (0, 3, 6))):
        g = grid_of(c["scene"])
        cam = cam_of(c["cam"])
        vm = gpu_map(g, mean, np.full_like(mean, 1e-2))
        if idx is None:
            poses = [synth.pose7(c["t_gt"], c["q_gt"]), synth.pose7(c["t_init"], c["q_init"])]
        else:
            poses = [synth.pose7(c["traj"].t[i], c["traj"].q[i]) for i in idx]
        out = P().render(g, vm, cam, P().poses_tensor(np.stack(poses)), hit_k=True)
        torch.cuda.synchronize()
        og, ocm, m64 = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"]), mean.astype(np.float32).astype(float)
        for i, pose in enumerate(poses):
            hit = out["hit_k"][i].cpu().numpy()
            ref, flip = _render_flips(og, ocm, m64, pose, hit, f"{name} pose {i}")
            v = (ref["mask"] == 1) & (out["mask"][i].cpu().numpy() == 1) & ~flip
            assert np.all(depth_close(out["depth"][i].cpu().numpy()[v], ref["depth"][v]))
            assert np.all(rgb_close(out["rgb"][i].cpu().numpy()[v], ref["rgb"][v]))


def _voxel_margins(og, ocm, pose, od, trunc, idx):
    """FP64 margins of the map-update decisions of voxels idx (k, j, i):
    pixel coordinates to the nearest integer (relative to max(|u|, 1)), the
    camera depth to 0 and to D + trunc (relative to max(z, 1 mm))."""
    k, j, i = idx
    x = np.asarray(og.origin) + og.voxel * (np.stack([i, j, k], -1) + 0.5)
    R = orc.quat_to_rot(pose[3:])
    Xc = (x - pose[:3]) @ R
    z = Xc[:, 2]
    u = ocm.fx * Xc[:, 0] / z + ocm.cx
    v = ocm.fy * Xc[:, 1] / z + ocm.cy
    mu = np.abs(u - np.round(u)) / np.maximum(np.abs(u), 1.0)
    mv = np.abs(v - np.round(v)) / np.maximum(np.abs(v), 1.0)
    mz = np.abs(z) / 1e-3
    iu = np.clip(np.floor(u).astype(int), 0, ocm.width - 1)
    iv = np.clip(np.floor(v).astype(int), 0, ocm.height - 1)
    D = od[iv, iu].astype(np.float64)
    md = np.abs(z - (D + trunc)) / np.maximum(np.abs(z), 1e-3)
    return np.minimum(np.minimum(mu, mv), np.minimum(mz, md))


def test_fp64_decisions_map_update(small, big):
    banner("tier ii: updated voxel set with FP64 decisions")
    for name, (c, mean_gt, _) in (("64^3 80x60", small), ("256^3 320x240", big)):
        n = c["scene"].n
        g = grid_of(c["scene"])
        cam = cam_of(c["cam"])
        og, ocm = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
        p = orc.Params()
        trunc = p.trunc_voxels * g.voxel
        if "traj" in c:
            tr = c["traj"]
            pose = synth.pose7(tr.t[4], tr.q[4])
            od, oc = c["depth"][4], c["rgb"][4]
        else:
            pose = synth.pose7(c["t_init"], c["q_init"])
            od, oc = synth.raycast(c["scene"], c["cam"], c["t_gt"], c["q_gt"], np.random.default_rng(5), 0.01, 0.02)
            od = od.astype(np.float32); oc = oc.astype(np.float32)
        var = np.full((4, n, n, n), 0.25, np.float32)
        vm = gpu_map(g, mean_gt, var)
        P().map_update(g, vm, cam, P().poses_tensor(pose), t(od), t(oc), trunc, 1.0)
        m2, v2 = vm.to_dense()
        torch.cuda.synchronize()
        gpu_upd = v2[0].cpu().numpy() != np.float32(0.25)
        del v2
        om = mean_gt.astype(np.float32).astype(np.float64)
        ov = var.astype(np.float64)
        cnt, upd = orc.map_update(og, om, ov, ocm, pose, od, oc, p, decide32=False, want_mask=True)
        # a voxel flips if its update decision differs, or if both update it
        # from different pixels (the stored means differ)
        same_val = np.all(m2.cpu().numpy() == om.astype(np.float32), axis=0)
        del m2
        flip = (gpu_upd != upd.astype(bool)) | (gpu_upd & ~same_val)
        idx = np.nonzero(flip)
        m = _voxel_margins(og, ocm, pose, od, trunc, idx) if len(idx[0]) else np.zeros(0)
        print(f"[tier ii map update {name}] {cnt} voxels updated, flips {len(m)}, largest flip margin "
              f"{m.max() if len(m) else 0.0:.1e}", flush=True)
        assert cnt > 1000
        assert np.all(m <= MARGIN), m


def test_fp64_decisions_track_p2(small, big):
    """Tracking rows with FP64 association and gating decisions: a pixel's
    rows may differ only where the projected coordinate is within 1e-4
    (relative) of a pixel edge or a bilinear tap edge, or the depth /
    colour residual within 1e-4 (relative) of its gate."""
    banner("tier ii: tracking rows with FP64 decisions")
    for name, (c, mean, _) in (("80x60", small), ("320x240", big)):
        rng = np.random.default_rng(8)
        if "traj" in c:
            tr = c["traj"]
            prev = synth.pose7(tr.t[2], tr.q[2])
            a64, adev, od, oc, cur = _p2_case(c, mean.astype(np.float64), prev, rng,
                                              obs=(c["depth"][3], c["rgb"][3], tr.t[3], tr.q[3]))
        else:
            prev = synth.pose7(c["t_gt"], c["q_gt"])
            a64, adev, od, oc, cur = _p2_case(c, mean.astype(np.float32).astype(np.float64), prev, rng)
        cam = cam_of(c["cam"])
        out = P().track_p2(cam, P().poses_tensor(cur), P().poses_tensor(prev), t(od), t(oc), adev,
                           P().Weights.make(), want_resid=True)
        torch.cuda.synchronize()
        ocm = orc.cam_from(c["cam"])
        ref = orc.track_p2(ocm, cur, prev, od, oc, a64, orc.Params(), decide32=False)
        rm = out["rowmask"].cpu().numpy()
        r = out["resid"].cpu().numpy().astype(np.float64)
        flip = (rm != ref["rowmask"]) | np.any(np.abs(r - ref["resid"]) > 1e-6 * np.maximum(np.abs(ref["resid"]), 1.0),
                                               axis=-1)
        vs, us = np.nonzero(flip)
        margins = []
        if len(us):
            H, W = od.shape
            Rc, Rp = orc.quat_to_rot(cur[3:]), orc.quat_to_rot(prev[3:])
            X = od[vs, us].astype(np.float64)[:, None] * np.stack(
                [(us + 0.5 - ocm.cx) / ocm.fx, (vs + 0.5 - ocm.cy) / ocm.fy, np.ones(len(us))], -1)
            Y = (X @ Rc.T + cur[:3] - prev[:3]) @ Rp
            up = ocm.fx * Y[:, 0] / Y[:, 2] + ocm.cx
            vp = ocm.fy * Y[:, 1] / Y[:, 2] + ocm.cy
            rel = lambda a, b: np.abs(a - b) / np.maximum(np.abs(a), 1.0)
            m = np.minimum.reduce([rel(up, np.round(up)), rel(vp, np.round(vp)),
                                   rel(up - 0.5, np.round(up - 0.5)), rel(vp - 0.5, np.round(vp - 0.5)),
                                   np.abs(Y[:, 2]) / 1e-3])
            rr = ref["resid"][vs, us]
            mg = np.abs(np.abs(rr[:, 0]) - 0.45) / 0.45
            mc = np.abs(np.abs(rr[:, 1:]).sum(-1) - 0.15) / 0.15
            margins = np.minimum(m, np.minimum(mg, mc))
        margins = np.asarray(margins)
        print(f"[tier ii track {name}] {int((ref['rowmask'] > 0).sum())} pixels with rows, flips {len(margins)}, "
              f"largest flip margin {margins.max() if len(margins) else 0.0:.1e}", flush=True)
        assert np.all(margins <= MARGIN), margins


# ---------------------------------------------------------------------------
# FP32 filter at the single-stream trajectory size
# ---------------------------------------------------------------------------
def test_filter_fp32_full_size_matches_oracle():
    """256^3 (2.5 cm) room, 320x240, K = 128, FP32 map, P2 with 3 Gauss-Newton
    iterations, 7 frames (the first frame and 6 full filter steps).  The
    closed loop (pose -> map update -> anchor -> next pose) amplifies any
    difference: the oracle run with FP64 decisions parts from its own FP32-
    decision run the same way.  So every step is compared from the same
    start: before step i the oracle takes the GPU filter's state (mean,
    covariance, Laplace average) and map, renders its anchor from them, and
    both take one step on frame i."""
    banner("filter FP32 256^3 320x240 K=128, 7 frames, one step at a time from the GPU state")
    n_frames = 7
    c = synth.trajectory_case(seed=1, n=256, width=320, height=240, n_samples=128, n_frames=n_frames)
    tr = c["traj"]
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    f = P().Filter(g, cam, P().FilterParams(objective=P().OBJ_P2))
    f.map.init()
    x0 = np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    f.reset(x0, P0)
    og, ocm = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
    D = t(c["depth"]); C = t(c["rgb"]); U = t(tr.u, torch.float64)
    for i in range(n_frames):
        s0 = f.state()
        m0, v0 = f.map.to_dense()
        pose0 = np.concatenate([np.array(s0.pose.t), np.array(s0.pose.q)])
        of = orc.Filter(og, ocm, orc.Params(), dict(t=pose0[:3], q=pose0[3:], v=np.array(s0.v), w=np.array(s0.w)),
                        np.array(s0.P).reshape(12, 12), m0.cpu().numpy().astype(np.float64),
                        v0.cpu().numpy().astype(np.float64))
        del m0, v0
        if i:
            of.s.step = i
            of.s.Sbar = np.array(s0.Sbar).reshape(6, 6) if s0.has_sbar else None
            of.s.anchor = orc.render(og, of.mean, ocm, pose0, normals=True)
            of.s.anchor_pose = pose0.copy()
        f.step(D[i], C[i], U[i - 1] if i else None)
        of.step(c["depth"][i].astype(np.float64), c["rgb"][i].astype(np.float64), tr.u[i - 1] if i else None)
        s = f.state()
        tg, qg = np.array(s.pose.t), np.array(s.pose.q)
        Pg = np.array(s.P).reshape(12, 12)
        dt_, dr_ = np.linalg.norm(tg - of.s.t), rot_angle(qg, of.s.q)
        eP = np.linalg.norm(Pg - of.s.P) / np.linalg.norm(of.s.P)
        print(f"step {i}: |dt| {dt_:.2e} m, dR {dr_:.2e} rad, P {eP:.2e}, updated {int(s.n_updated)} vs "
              f"{of.s.last['n_updated']}, position error to the truth {np.linalg.norm(tg - tr.t[i]):.4f} m",
              flush=True)
        assert s.flags == 0
        assert dt_ <= 1e-5 and dr_ <= 1e-5, (i, dt_, dr_)
        assert np.linalg.norm(np.array(s.v) - of.s.v) <= 1e-4
        assert eP <= 1e-4, (i, eP)
        # the map update runs at the two posterior means, which agree to ~1e-9,
        # and decides in single precision from the pose rounded to float: a
        # voxel whose decision margin is below that rounding may take the
        # neighbouring pixel or flip (at most 1e-4 of the updated voxels)
        nu = of.s.last["n_updated"]
        assert abs(int(s.n_updated) - nu) <= max(10, 1e-4 * nu), i
        m1, _ = f.map.to_dense()
        dm = np.abs(m1.cpu().numpy().astype(np.float64) - of.mean)
        nd = int((dm > 1e-6).any(0).sum())
        print(f"  map means: max |difference| {dm.max():.2e}, voxels differing by more than 1e-6: {nd}", flush=True)
        assert nd <= max(10, 1e-4 * nu), (i, nd)
        del m1, dm, of


# ---------------------------------------------------------------------------
# brick-pool maps smaller than the grid
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [0, 1])
def test_pool_smaller_than_grid_matches_oracle(big, dtype):
    """A brick-pool map with room for 40 % of the grid's bricks, fused from
    four frames of the trajectory: no brick update is dropped, the updated
    means and variances equal the oracle's bit for bit (rounded to the
    storage type), and renders match the oracle's hit samples exactly."""
    banner(f"brick pool at 40 % of the grid against the oracle, dtype {dtype}")
    c, _, _ = big
    tr = c["traj"]
    n = c["scene"].n
    nb3 = (n // 8) ** 3
    cap = int(0.4 * nb3)
    sc = c["scene"]
    g = P().Grid.make(n, sc.voxel, tuple(float(v) for v in sc.origin), dtype, capacity=cap)
    assert P().map_bytes(g) < 0.45 * P().map_bytes(grid_of(sc, dtype))
    cam = cam_of(c["cam"])
    vm = P().VoxelMap(g).init()
    og, ocm, p = orc.grid_from_scene(sc), orc.cam_from(c["cam"]), orc.Params()
    cast = (lambda a: a.astype(np.float32)) if dtype == 0 else synth.bf16_round
    om = np.zeros((4, n, n, n)); om[0] = -0.001
    ov = np.full_like(om, 1e4)
    om, ov = cast(om).astype(np.float64), cast(ov).astype(np.float64)
    for i in (0, 2, 4, 6):
        pose = synth.pose7(tr.t[i], tr.q[i])
        nu = P().map_update(g, vm, cam, P().poses_tensor(pose), t(c["depth"][i]), t(c["rgb"][i]),
                            p.trunc_voxels * sc.voxel, 1.0)
        cnt = orc.map_update(og, om, ov, ocm, pose, c["depth"][i], c["rgb"][i], p)
        # the GPU map holds its storage type: the oracle continues from the stored values
        om, ov = cast(om).astype(np.float64), cast(ov).astype(np.float64)
        assert int(nu.item()) == cnt > 100000
    usage = vm.pool_usage().cpu().numpy()
    print(f"[pool] {int(usage[0])} of {cap} slots used ({nb3} bricks in the grid), dropped {int(usage[1])}",
          flush=True)
    assert usage[1] == 0 and 0 < usage[0] <= cap
    m2, v2 = vm.to_dense()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m2.cpu().numpy(), cast(om))
    np.testing.assert_array_equal(v2.cpu().numpy(), cast(ov))
    del v2
    poses = [synth.pose7(tr.t[i], tr.q[i]) for i in (1, 5)]
    out = P().render(g, vm, cam, P().poses_tensor(np.stack(poses)), hit_k=True)
    torch.cuda.synchronize()
    mref = m2.cpu().numpy().astype(np.float64)
    for i, pose in enumerate(poses):
        ref = orc.render(og, mref, ocm, pose)
        np.testing.assert_array_equal(out["hit_k"][i].cpu().numpy(), ref["hit_k"])
        v = ref["mask"] == 1
        assert v.sum() > 10000
        assert np.all(depth_close(out["depth"][i].cpu().numpy()[v], ref["depth"][v]))
        assert np.all(rgb_close(out["rgb"][i].cpu().numpy()[v], ref["rgb"][v]))
