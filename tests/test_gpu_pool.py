"""Brick-pool maps on the GPU against dense maps (the dense path is itself
checked against the oracle): with room for every brick every result is the
dense map's bit for bit; with a small pool, the bricks that got a slot hold
exactly the dense values and every other brick reads as the prior."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, P, banner, cam_of, t

pytestmark = pytest.mark.gpu


def _case():
    c = synth.trajectory_case(seed=3, n=128, width=160, height=120, n_samples=64, n_frames=6)
    tr = c["traj"]
    poses = [P().poses_tensor(np.concatenate([tr.t[i], tr.q[i]])) for i in range(6)]
    return c, poses


def _grid(c, dtype, capacity):
    sc = c["scene"]
    return P().Grid.make(sc.n, sc.voxel, tuple(float(v) for v in sc.origin), dtype, capacity=capacity)


@pytest.mark.parametrize("dtype", [0, 1])
def test_pool_map_equals_dense_map(dtype):
    banner(f"brick-pool map vs dense 128^3 160x120 dtype={dtype}")
    c, poses = _case()
    cam = cam_of(c["cam"])
    nb3 = (c["scene"].n // 8) ** 3
    gd, gp = _grid(c, dtype, 0), _grid(c, dtype, nb3)
    md, mp = P().VoxelMap(gd).init(), P().VoxelMap(gp).init()
    trunc = 4 * gd.voxel
    for i in range(6):
        D, C = t(c["depth"][i]), t(c["rgb"][i])
        nd = P().map_update(gd, md, cam, poses[i], D, C, trunc)
        npl = P().map_update(gp, mp, cam, poses[i], D, C, trunc)
        rd = P().render(gd, md, cam, poses[(i + 1) % 6], normals=True, hit_k=True)
        rp = P().render(gp, mp, cam, poses[(i + 1) % 6], normals=True, hit_k=True)
        torch.cuda.synchronize()
        assert int(nd.item()) == int(npl.item())
        for k in ("depth", "rgb", "mask", "hit_k", "normals", "nmask"):
            assert torch.equal(rd[k], rp[k]), (i, k)
    a, b = md.to_dense(), mp.to_dense()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    usage = mp.pool_usage().cpu().numpy()
    # bricks holding any voxel that differs from the initial values
    mean, var = a
    n = c["scene"].n
    shape = (4, n // 8, 8, n // 8, 8, n // 8, 8)
    m0, v0 = (x.cpu().numpy().reshape(shape) for x in P().VoxelMap(gd).init().to_dense())
    m, v = mean.cpu().numpy().reshape(shape), var.cpu().numpy().reshape(shape)
    changed = ((m != m0) | (v != v0)).any(axis=(0, 2, 4, 6))
    print(f"slots used {usage[0]} of {nb3}, dropped {usage[1]}, bricks changed {changed.sum()}", flush=True)
    assert usage[1] == 0 and usage[0] >= changed.sum() and usage[0] < nb3


def test_small_pool_keeps_what_fits():
    banner("brick-pool map with a small pool")
    c, poses = _case()
    cam = cam_of(c["cam"])
    cap = 150
    gd, gp = _grid(c, 0, 0), _grid(c, 0, cap)
    md, mp = P().VoxelMap(gd).init(), P().VoxelMap(gp).init()
    trunc = 4 * gd.voxel
    for i in range(6):
        D, C = t(c["depth"][i]), t(c["rgb"][i])
        P().map_update(gd, md, cam, poses[i], D, C, trunc)
        P().map_update(gp, mp, cam, poses[i], D, C, trunc)
        rp = P().render(gp, mp, cam, poses[i])
    torch.cuda.synchronize()
    usage = mp.pool_usage().cpu().numpy()
    assert usage[0] == cap and usage[1] > 0
    n = c["scene"].n
    shape = (4, n // 8, 8, n // 8, 8, n // 8, 8)
    (dm, dv), (pm, pv) = md.to_dense(), mp.to_dense()
    m0, v0 = P().VoxelMap(gd).init().to_dense()
    dm, dv, pm, pv, m0, v0 = (x.cpu().numpy().reshape(shape) for x in (dm, dv, pm, pv, m0, v0))
    same = ((dm == pm).all(axis=(0, 2, 4, 6)) & (dv == pv).all(axis=(0, 2, 4, 6)))
    prior = ((pm == m0).all(axis=(0, 2, 4, 6)) & (pv == v0).all(axis=(0, 2, 4, 6)))
    assert np.all(same | prior)
    kept = same & ~prior
    print(f"bricks kept {kept.sum()} (pool {cap}), dropped updates {usage[1]}", flush=True)
    assert 0 < kept.sum() <= cap
    assert rp["mask"].any()


def test_filter_with_pool_map_equals_dense():
    """Filter steps on brick-pool maps, single and batched (a batch mixing
    dense and brick-pool maps of both storage types), give exactly the states,
    maps and anchors of dense single steps."""
    banner("filter with brick-pool maps (single and batched)")
    c, _ = _case()
    tr = c["traj"]
    cam = cam_of(c["cam"])
    nb3 = (c["scene"].n // 8) ** 3
    H, W = c["cam"].height, c["cam"].width
    x0 = np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    s = torch.cuda.Stream()

    def make(dtype, cap, slots=False):
        f = P().Filter(_grid(c, dtype, cap), cam, P().FilterParams(objective=0))
        with torch.cuda.stream(s):
            f.map.init(stream=s)
            f.reset(x0, P0, stream=s)
        if slots:
            f.set_slots([(torch.empty((H, W), device=DEV), torch.empty((H, W, 3), device=DEV),
                          torch.zeros(6, dtype=torch.float64, device=DEV)) for _ in range(2)])
        return f

    ref = {0: make(0, 0), 1: make(1, 0)}                 # dense, single steps
    single = {0: make(0, nb3), 1: make(1, nb3)}          # brick pool, single steps
    batch = [make(0, nb3, True), make(1, nb3, True), make(1, 0, True)]
    with torch.cuda.stream(s):
        for i in range(6):
            D, C = t(c["depth"][i]), t(c["rgb"][i])
            U = t(tr.u[i - 1], torch.float64) if i else None
            for f in list(ref.values()) + list(single.values()):
                f.step(D, C, U, stream=s)
            assert P().filter_step_batch(batch, [(D, C, U)] * 3, stream=s)
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    pairs = [(ref[0], single[0]), (ref[1], single[1]), (ref[0], batch[0]), (ref[1], batch[1]), (ref[1], batch[2])]
    for k, (fa, fb) in enumerate(pairs):
        assert bytes(fa.state()) == bytes(fb.state()), k
        ma, va = fa.map.to_dense()
        mb, vb = fb.map.to_dense()
        assert torch.equal(ma, mb) and torch.equal(va, vb), k
        aa, ab = fa.anchor(), fb.anchor()
        for key in aa:
            assert torch.equal(aa[key], ab[key]), (k, key)
    for f in (single[0], single[1], batch[0], batch[1]):
        assert int(f.map.pool_usage()[1].item()) == 0
