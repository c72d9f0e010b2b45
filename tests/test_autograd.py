"""RenderFn: the renderer's hand-written adjoint behind torch.autograd."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth


@pytest.mark.gpu
def test_retract_matches_oracle():
    """prism_pose_retract (through the C ABI): t + dt, Exp(dtheta) R, against
    the oracle's retraction, for rotations from small to large."""
    from gpu_util import P
    rng = np.random.default_rng(0)
    n = 8
    t, q = rng.normal(size=(n, 3)), rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    d = rng.normal(0, 0.3, (n, 6))
    d[0] = 0.0
    d[1, 3:] = 1e-9                       # below the series switch of Exp
    poses = np.concatenate([t, q], 1)
    got = P().pose_retract(P().poses_tensor(poses), torch.tensor(d, device="cuda")).cpu().numpy()
    for i in range(n):
        ref = orc.retract(poses[i], d[i])
        g = got[i].copy()
        if g[3] * ref[3] < 0:
            g[3:] = -g[3:]
        np.testing.assert_allclose(g, ref, atol=1e-12)


def _subcase():
    """32^3 grid over a 6.4 m room (20 cm voxels), 40x30 camera, 16 samples."""
    c = synth.trajectory_case(seed=3, n=32, width=40, height=30, n_samples=16, n_frames=3, frames=False)
    mean, var = synth.gt_map(c["scene"])
    return c, mean, var


@pytest.mark.gpu
def test_autograd_matches_oracle_adjoint():
    from gpu_util import banner, cam_of, gpu_map, grid_of, P
    from paper_2212_02988_amd.autograd import render as drender
    banner("autograd 32^3 40x30")
    c, mean, var = _subcase()
    tr = c["traj"]
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    vm = gpu_map(g, mean, var)
    poses = P().poses_tensor(np.stack([np.concatenate([tr.t[i], tr.q[i]]) for i in range(2)]))
    rng = np.random.default_rng(1)
    od = np.stack([synth.raycast(c["scene"], c["cam"], tr.t[i] + 0.01, tr.q[i])[0] for i in range(2)])
    oc = np.stack([synth.raycast(c["scene"], c["cam"], tr.t[i] + 0.01, tr.q[i])[1] for i in range(2)])
    od_t = torch.tensor(od, dtype=torch.float32, device="cuda")
    oc_t = torch.tensor(oc, dtype=torch.float32, device="cuda")
    wd, wc = 1.0 / 0.02 ** 2, 1.0 / 0.1 ** 2
    mp = vm.mean_planes().requires_grad_(True)
    delta = torch.zeros((2, 6), dtype=torch.float64, device="cuda", requires_grad=True)
    d, rgb, mask = drender(vm, cam, poses, delta, mp)
    m = mask.float()
    L = (wd * m * (d - od_t) ** 2).sum() + (wc * m[..., None] * (rgb - oc_t) ** 2).sum()
    L.backward()
    gm = P().bricks_to_dense(g.n, mp.grad).cpu().numpy()
    gp = delta.grad.cpu().numpy()
    # oracle adjoint with the same upstream gradients (from the oracle's own render)
    og, ocm = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
    m32 = mean.astype(np.float32).astype(np.float64)
    gm_ref = np.zeros_like(m32)
    for i in range(2):
        pose = np.concatenate([tr.t[i], tr.q[i]])
        r = orc.render(og, m32, ocm, pose)
        mk = r["mask"] == 1
        gd = 2 * wd * mk * (r["depth"] - od[i])
        gc = 2 * wc * mk[..., None] * (r["rgb"] - oc[i])
        gmi, gpi = orc.render_vjp(og, m32, ocm, pose, gd, gc)
        gm_ref += gmi
        # each pose component against its accumulation scale: the sum over
        # rays and rows of |J row| |upstream gradient| (oracle rows; an
        # observation equal to the render keeps every row)
        full = orc.render_jacobian(og, m32, ocm, pose, np.where(mk, r["depth"], 0.0), r["rgb"], orc.Params(),
                                   want_J=True)
        up = np.concatenate([gd[..., None], gc], -1)
        scale = float(np.sum(np.linalg.norm(full["J"], axis=-1) * np.abs(up)))
        ep = np.abs(gp[i] - gpi) / scale
        print(f"[autograd pose {i}] max error / accumulation scale {ep.max():.2e}", flush=True)
        assert ep.max() <= 1e-5, (gp[i], gpi, scale)
    nz = (gm != 0) | (gm_ref != 0)
    assert nz.sum() > 1000
    # every voxel and channel, relative, with a floor of 1e-3 of the channel's
    # largest gradient for entries that cancel
    floor = 1e-3 * np.abs(gm_ref).reshape(4, -1).max(1)[:, None, None, None]
    em = np.abs(gm - gm_ref) / np.maximum(np.abs(gm_ref), floor)
    print(f"[autograd map] {int(nz.sum())} entries, max scaled error {em[nz].max():.2e}", flush=True)
    assert em[nz].max() <= 1e-4, em[nz].max()


@pytest.mark.gpu
def test_autograd_finite_differences():
    """Central differences (eps = 1e-3) of the GPU render against the
    adjoint, for all 6 pose components and 64 random touched voxel means.
    Per perturbation, only rays whose hit sample is the same at -eps, 0 and
    +eps, and whose two bracketing samples stay in the same trilinear cells,
    enter the loss (the render is smooth there: the trilinear field has
    gradient kinks on cell faces); the adjoint is run with the same ray mask
    on its upstream gradients."""
    from gpu_util import banner, cam_of, gpu_map, grid_of, P
    from paper_2212_02988_amd.autograd import render as drender
    banner("autograd finite differences")
    c, mean, var = _subcase()
    tr = c["traj"]
    g = grid_of(c["scene"])
    cam = cam_of(c["cam"])
    vm = gpu_map(g, mean, var)
    poses = P().poses_tensor(np.concatenate([tr.t[0], tr.q[0]]))
    rng = np.random.default_rng(2)
    H, W = cam.height, cam.width
    gd_up = torch.tensor(rng.normal(size=(1, H, W)), dtype=torch.float64, device="cuda")
    gc_up = torch.tensor(rng.normal(size=(1, H, W, 3)), dtype=torch.float64, device="cuda")
    zero = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
    eps = 1e-3

    def fwd(p):
        o = P().render(g, vm, cam, p, hit_k=True)
        return o["depth"].double(), o["rgb"].double(), o["hit_k"].clone()

    def loss(d, rgb, S):
        return float((S * gd_up * d).sum() + (S[..., None] * gc_up * rgb).sum())

    def adjoint(S):
        mp = vm.mean_planes().requires_grad_(True)
        delta = zero.clone().requires_grad_(True)
        d, rgb, _ = drender(vm, cam, poses, delta, mp)
        (((S * gd_up).float() * d).sum() + ((S[..., None] * gc_up).float() * rgb).sum()).backward()
        return mp.grad.clone(), delta.grad[0].cpu().numpy()

    _, _, k0 = fwd(poses)
    sc, cm = c["scene"], c["cam"]
    dirs = synth.pixel_dirs(cm)
    k0n = k0[0].cpu().numpy().astype(np.int64)
    step = (cm.d_far - cm.d_near) / (cm.n_samples - 1)

    def cells(p7):
        """Trilinear cells of samples k*-1 and k* of every ray (host, float64)."""
        p7 = p7[0].cpu().numpy()
        R = orc.quat_to_rot(p7[3:])
        out = []
        for k in (k0n - 1, k0n):
            pts = p7[:3] + (dirs * (cm.d_near + np.maximum(k, 0) * step)[..., None]) @ R.T
            out.append(np.floor((pts - sc.origin) / sc.voxel - 0.5))
        return np.concatenate(out, -1)

    c_base = cells(poses)
    checked = 0
    for m in range(6):
        e = zero.clone()
        e[0, m] = eps
        pa, pb = P().pose_retract(poses, e), P().pose_retract(poses, -e)
        da, ca, ka = fwd(pa)
        db, cb, kb = fwd(pb)
        same = np.all((cells(pa) == c_base) & (cells(pb) == c_base), -1)
        S = ((ka == k0) & (kb == k0) & (k0 >= 1)).double() * torch.tensor(same[None], device="cuda")
        assert S.sum() > 0.8 * H * W * 0.5
        fd = (loss(da, ca, S) - loss(db, cb, S)) / (2 * eps)
        _, gp = adjoint(S)
        assert abs(fd - gp[m]) <= 1e-2 * max(1.0, abs(gp[m])), (m, fd, gp[m])
        checked += 1
    assert checked == 6
    S_all = (k0 >= 1).double()
    gm, _ = adjoint(S_all)
    planes = vm.mean_planes()
    idx = torch.nonzero(gm.abs().sum(0) > 0).flatten().cpu().numpy()
    pick = rng.choice(idx, size=min(64, len(idx)), replace=False)
    ok = 0
    with torch.no_grad():
        for v in pick:
            ch = int(rng.integers(0, 4))
            old = planes[ch, v].item()
            planes[ch, v] = old + eps
            vm.refresh()
            da, ca, ka = fwd(poses)
            planes[ch, v] = old - eps
            vm.refresh()
            db, cb, kb = fwd(poses)
            planes[ch, v] = old
            vm.refresh()
            S = ((ka == k0) & (kb == k0) & (k0 >= 1)).double()
            if not torch.equal(S, S_all):
                continue        # a hit moved: the render is not smooth in this direction
            fd = (loss(da, ca, S) - loss(db, cb, S)) / (2 * eps)
            an = gm[ch, v].item()
            assert abs(fd - an) <= 1e-2 * max(1.0, abs(an)), (ch, v, fd, an)
            ok += 1
    assert ok >= 32
