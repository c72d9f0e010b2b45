"""The renderer's free-space bits on the GPU.  After every call that writes
a map (initialisation, dense upload, closed-form update, filter steps single
and batched, descent steps) the brick summary's sign must be exact (a brick
is summarised by a value <= 0 exactly when every occupancy mean in its
planes is <= 0; a positive summary is the brick's largest occupancy), the
plain bits must equal "brick summary <= 0"
and the dilated bits must equal the AND over each brick's 2x2x2 block of
bricks, both recomputed here in numpy from the map's own brick maxima.  A
wrong bit would let the renderer skip a sample whose occupancy can exceed
0 (the render parity tests would catch most such cases, this catches all)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, P, banner, cam_of, gpu_map, t

pytestmark = pytest.mark.gpu


def _r256(x):
    return (x + 255) // 256 * 256


def _aux(grid, vm):
    """(brick maxima, plain words, dilated words) read from the map buffer:
    the planes, then the brick maxima, then the two bitmaps."""
    n, nb = grid.n, grid.n // 8
    nb3, nw = nb ** 3, (nb ** 3 + 31) // 32
    elem = 2 if grid.dtype == P().PRISM_BF16 else 4
    plane = grid.capacity * 512 if grid.capacity > 0 else n ** 3
    off_bmax = _r256(8 * plane * elem)
    off_bits = off_bmax + _r256(4 * nb3)
    raw = vm.buf.cpu().numpy()
    bmax = raw[off_bmax:off_bmax + 4 * nb3].view(np.float32)
    words = raw[off_bits:off_bits + 8 * nw].view(np.uint32)
    return bmax, words[:nw], words[nw:]


def _unpack(words, count):
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:count].astype(bool)


def _check(grid, vm, what):
    nb = grid.n // 8
    nb3 = nb ** 3
    nw = (nb3 + 31) // 32
    bmax, plain, dil = _aux(grid, vm)
    free = bmax <= 0.0
    bits = _unpack(plain, 32 * nw)
    assert np.array_equal(bits[:nb3], free), what
    # the summary's sign is exact: a brick is free exactly when every
    # occupancy mean stored in its planes is <= 0
    occ = vm.to_dense()[0][0].cpu().numpy()
    true_max = occ.reshape(nb, 8, nb, 8, nb, 8).max(axis=(1, 3, 5)).ravel()
    assert np.array_equal(true_max <= 0.0, free), (what, "summary sign", int(((true_max <= 0) != free).sum()))
    pos = true_max > 0
    assert np.array_equal(bmax[pos], true_max[pos].astype(np.float32)), (what, "positive maxima are exact")
    assert not bits[nb3:].any(), what
    # dilated bit b: bits b + {0, 1} + {0, nb} + {0, nb^2}, zero past the last brick
    ext = np.zeros(32 * nw + nb * nb + nb + 2, dtype=bool)
    ext[:nb3] = free
    idx = np.arange(32 * nw)
    want = np.ones(32 * nw, dtype=bool)
    for o in (0, 1, nb, nb + 1, nb * nb, nb * nb + 1, nb * nb + nb, nb * nb + nb + 1):
        want &= ext[idx + o]
    got = _unpack(dil, 32 * nw)
    assert np.array_equal(got, want), (what, int((got != want).sum()))
    # what the renderer relies on: off the last layers, a set dilated bit
    # means every brick of the 2x2x2 block is free, and the converse
    f3 = free.reshape(nb, nb, nb)                      # [bz, by, bx]
    block = np.ones((nb - 1, nb - 1, nb - 1), dtype=bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                block &= f3[dz:nb - 1 + dz, dy:nb - 1 + dy, dx:nb - 1 + dx]
    g3 = got[:nb3].reshape(nb, nb, nb)[:nb - 1, :nb - 1, :nb - 1]
    assert np.array_equal(g3, block), what
    return int(free.sum()), int(got[:nb3].sum())


@pytest.mark.parametrize("n", [48, 64])
def test_free_bits_after_init_and_upload(n):
    """48^3: 216 bricks, the last bitmap word only partly used."""
    banner(f"free-space bits after init / from_dense {n}^3")
    for dtype in (0, 1):
        g = P().Grid.make(n, 0.05, dtype=dtype)
        vm = P().VoxelMap(g).init()
        torch.cuda.synchronize()
        _check(g, vm, f"init dtype={dtype}")
        rng = np.random.default_rng(7 + dtype)
        # sparse positive occupancy: a few bricks with one positive voxel each
        mean = np.full((4, n, n, n), -0.001, np.float32)
        for _ in range(12):
            z, y, x = rng.integers(0, n, 3)
            mean[0, z, y, x] = 0.3
        var = np.ones((4, n, n, n), np.float32)
        vm = gpu_map(g, mean, var)
        torch.cuda.synchronize()
        nf, nd = _check(g, vm, f"from_dense dtype={dtype}")
        print(f"n={n} dtype={dtype}: {nf} free bricks, {nd} dilated bits set", flush=True)


def _traj():
    c = synth.trajectory_case(seed=3, n=128, width=160, height=120, n_samples=64, n_frames=6)
    tr = c["traj"]
    return c, tr


@pytest.mark.parametrize("dtype,pool", [(0, False), (1, False), (1, True)])
def test_free_bits_after_map_updates(dtype, pool):
    banner(f"free-space bits after closed-form updates dtype={dtype} pool={pool}")
    c, tr = _traj()
    sc = c["scene"]
    nb3 = (sc.n // 8) ** 3
    g = P().Grid.make(sc.n, sc.voxel, tuple(float(v) for v in sc.origin), dtype, capacity=nb3 if pool else 0)
    cam = cam_of(c["cam"])
    vm = P().VoxelMap(g).init()
    for i in range(6):
        pose = P().poses_tensor(np.concatenate([tr.t[i], tr.q[i]]))
        P().map_update(g, vm, cam, pose, t(c["depth"][i]), t(c["rgb"][i]), 4 * g.voxel)
        torch.cuda.synchronize()
        nf, nd = _check(g, vm, f"after update {i}")
    print(f"{nf} of {nb3} bricks free, {nd} dilated bits set", flush=True)
    assert nf < nb3 and nd < nf


def test_free_bits_after_filter_steps_and_descent():
    banner("free-space bits after filter steps (single, batched) and descent steps")
    c, tr = _traj()
    sc = c["scene"]
    cam = cam_of(c["cam"])
    H, W = c["cam"].height, c["cam"].width
    x0 = np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    s = torch.cuda.Stream()

    def make(dtype, slots):
        g = P().Grid.make(sc.n, sc.voxel, tuple(float(v) for v in sc.origin), dtype)
        f = P().Filter(g, cam, P().FilterParams(objective=0))
        with torch.cuda.stream(s):
            f.map.init(stream=s)
            f.reset(x0, P0, stream=s)
        if slots:
            f.set_slots([(torch.empty((H, W), device=DEV), torch.empty((H, W, 3), device=DEV),
                          torch.zeros(6, dtype=torch.float64, device=DEV)) for _ in range(2)])
        return f

    single, batch = make(0, False), [make(0, True), make(1, True)]
    with torch.cuda.stream(s):
        for i in range(5):
            D, C = t(c["depth"][i]), t(c["rgb"][i])
            U = t(tr.u[i - 1], torch.float64) if i else None
            single.step(D, C, U, stream=s)
            assert P().filter_step_batch(batch, [(D, C, U)] * 2, stream=s)
    torch.cuda.synchronize()
    for k, f in enumerate([single] + batch):
        _check(f.grid, f.map, f"filter {k}")
    # descent steps on the single filter's (FP32) map
    g = single.grid
    ws = P().map_gd_workspace(g, cam)
    pose = P().poses_tensor(np.concatenate([tr.t[5], tr.q[5]]))
    P().map_gd(g, single.map, cam, pose, t(c["depth"][5]), t(c["rgb"][5]), P().Weights.make(), 3e-6, 3e-3, 5, ws)
    torch.cuda.synchronize()
    _check(g, single.map, "descent")
