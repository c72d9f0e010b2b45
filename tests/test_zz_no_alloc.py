"""The allocation-free render Jacobian (prism_render_jacobian_noalloc) against
the workspace entry point (prism_render_jacobian), through the C ABI.

Both run the same kernels in the same order, so every output must agree bit
for bit.  Two calls in a row share the library's scratch array: the second,
smaller one must not see anything of the first.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, banner, cam_of, gpu_map, grid_of, t, P

pytestmark = pytest.mark.gpu

KEYS = ("neq", "depth", "rgb", "mask", "J", "resid", "rowmask")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P().lib()
    yield


def _outputs(n, H, W):
    return dict(neq=torch.full((n, P().NEQ), float("nan"), dtype=torch.float64, device=DEV),
                depth=torch.full((n, H, W), -1.0, dtype=torch.float32, device=DEV),
                rgb=torch.full((n, H, W, 3), -1.0, dtype=torch.float32, device=DEV),
                mask=torch.full((n, H, W), 7, dtype=torch.uint8, device=DEV),
                J=torch.full((n, H, W, 4, 6), -1.0, dtype=torch.float32, device=DEV),
                resid=torch.full((n, H, W, 4), -1.0, dtype=torch.float32, device=DEV),
                rowmask=torch.full((n, H, W), 7, dtype=torch.uint8, device=DEV))


def _both(grid, vm, cam, poses, od, oc):
    n = poses.shape[0]
    w = P().Weights.make()
    ref = P().render_jacobian(grid, vm, cam, poses, od, oc, w, want_render=True, want_J=True, want_resid=True)
    out = P().render_jacobian_noalloc(grid, vm, cam, poses, od, oc, w, _outputs(n, cam.height, cam.width))
    torch.cuda.synchronize()
    return ref, out


def _assert_same(ref, out, label):
    for k in KEYS:
        a, b = out[k].cpu().numpy(), ref[k].cpu().numpy()
        assert a.tobytes() == b.tobytes(), f"{label}: {k} differs from the workspace entry point"


def test_noalloc_matches_workspace_entry_point_twice():
    # call 1: 8 frames, 128^3 FP32 map, 320x240, K = 64 (1200 workgroups per frame)
    banner("render_jacobian_noalloc: 8 frames 128^3 FP32 320x240, then 1 frame 64^3 BF16 80x60")
    c = synth.trajectory_case(seed=1, n=128, width=320, height=240, n_samples=64, n_frames=8, frames=False)
    sc, cm, tr = c["scene"], c["cam"], c["traj"]
    mean, var = synth.gt_map(sc, dtype=np.float32)
    g = grid_of(sc, 0)
    cam = cam_of(cm)
    vm = gpu_map(g, mean, var)
    D, C = synth.raycast_torch(sc, cm, tr.t, tr.q, 11, 0.01, 0.02)
    poses = P().poses_tensor(np.stack([synth.pose7(tr.t[i] + 0.01, tr.q[i]) for i in range(8)]))
    ref, out = _both(g, vm, cam, poses, D, C)
    assert int(ref["neq"][:, 28].min().item()) > 1000, "first call: too few contributing pixels"
    _assert_same(ref, out, "call 1")
    del vm
    # call 2: smaller input (1 frame, 64^3 BF16 map, 80x60, K = 32)
    c1 = synth.single_frame_case(0)
    mean1, var1 = synth.gt_map(c1["scene"])
    g1 = grid_of(c1["scene"], 1)
    cam1 = cam_of(c1["cam"])
    vm1 = gpu_map(g1, mean1, var1)
    od, oc = synth.raycast(c1["scene"], c1["cam"], c1["t_gt"], c1["q_gt"], np.random.default_rng(3), 0.01, 0.02)
    pose1 = P().poses_tensor(synth.pose7(c1["t_init"], c1["q_init"]))
    ref1, out1 = _both(g1, vm1, cam1, pose1, t(od.astype(np.float32))[None], t(oc.astype(np.float32))[None])
    assert int(ref1["neq"][0, 28].item()) > 100, "second call: too few contributing pixels"
    _assert_same(ref1, out1, "call 2")


def test_noalloc_rejects_oversize_calls():
    banner("render_jacobian_noalloc: a call beyond the scratch array is refused")
    cap = P().render_jacobian_noalloc_max_bytes()
    assert cap == 8 << 20
    W, H, n = 640, 480, 8        # 8 x 4800 workgroups x 232 bytes > 8 MiB
    assert n * (W // 8) * (H // 8) * 232 > cap
    g = P().Grid.make(64, 0.1)
    vm = P().VoxelMap(g).init()
    cam = P().Camera.make(W, H, 480.0, 480.0, 320.0, 240.0, 0.1, 7.5, 64)
    poses = P().poses_tensor(np.tile(synth.pose7(np.full(3, 3.2), np.array([1.0, 0, 0, 0])), (n, 1)))
    od = torch.zeros((n, H, W), dtype=torch.float32, device=DEV)
    oc = torch.zeros((n, H, W, 3), dtype=torch.float32, device=DEV)
    out = _outputs(n, H, W)
    with pytest.raises(P().PrismError, match="scratch"):
        P().render_jacobian_noalloc(g, vm, cam, poses, od, oc, P().Weights.make(), out)
    torch.cuda.synchronize()
    assert torch.isnan(out["neq"]).all(), "a refused call must queue nothing"
    # the largest call that fits still runs
    n_ok = cap // ((W // 8) * (H // 8) * 232)
    assert n_ok == 7
    out = _outputs(n_ok, H, W)
    P().render_jacobian_noalloc(g, vm, cam, poses[:n_ok].contiguous(), od[:n_ok].contiguous(),
                                oc[:n_ok].contiguous(), P().Weights.make(), out)
    torch.cuda.synchronize()
    assert torch.isfinite(out["neq"]).all()
    assert int(out["neq"][:, 28].max().item()) == 0       # no observed depth: no contributing pixel
