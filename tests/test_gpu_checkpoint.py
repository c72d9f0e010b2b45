"""Filter checkpoints (prism_filter_save / prism_filter_load), the capture
status, and the low-inlier flag, through the C ABI.

A checkpoint carries the belief (q_t(M), q_t(x)) of Sec. 4.2-4.3: a filter
restored from one continues bit for bit as the saved filter does.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, banner, cam_of, t, P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P().lib()
    yield


@pytest.fixture(scope="module")
def traj():
    c = synth.trajectory_case(seed=2, n=128, width=160, height=120, n_samples=64, n_frames=8)
    return c


def _filter(c, dtype=0, capacity=0, **kw):
    sc = c["scene"]
    g = P().Grid.make(sc.n, sc.voxel, tuple(float(v) for v in sc.origin), dtype, capacity=capacity)
    f = P().Filter(g, cam_of(c["cam"]), P().FilterParams(**kw))
    f.map.init()
    tr = c["traj"]
    if kw.get("modes", 0) & P().MODE_ACCEL_BIAS:
        f.reset(np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0], np.zeros(3)]),
                np.diag([1e-6] * 6 + [1e-4] * 6 + [1e-4] * 3))
    else:
        f.reset(np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]]), np.diag([1e-6] * 6 + [1e-4] * 6))
    return f


def _frames(c, body=False):
    return t(c["depth"]), t(c["rgb"]), t(c["traj"].u_body if body else c["traj"].u, torch.float64)


def _snapshot(f):
    m, v = f.map.to_dense()
    a = f.anchor()
    torch.cuda.synchronize()
    bias = bytes(f.bias_state()) if f.params.modes & P().MODE_ACCEL_BIAS else b""
    return (bytes(f.state()), bias, m.cpu().numpy().tobytes(), v.cpu().numpy().tobytes(),
            a["depth"].cpu().numpy().tobytes(), a["normals"].cpu().numpy().tobytes())


@pytest.mark.parametrize("kind", ["fp32", "bf16_pool", "fp32_15d"])
def test_checkpoint_continues_bit_for_bit(traj, kind):
    banner(f"checkpoint round trip, {kind}")
    c = traj
    kw = {"fp32": dict(dtype=0), "bf16_pool": dict(dtype=1, capacity=(c["scene"].n // 8) ** 3 // 2),
          "fp32_15d": dict(dtype=0, modes=P().MODE_ACCEL_BIAS)}[kind]
    D, C, U = _frames(c, body=kind == "fp32_15d")
    a = _filter(c, **kw)
    for i in range(4):
        a.step(D[i], C[i], U[i - 1] if i else None)
    dev_ck = a.save()
    host_ck = torch.empty(a.save_bytes(), dtype=torch.uint8).pin_memory()
    a.save(host_ck)
    torch.cuda.synchronize()
    for i in range(4, 7):
        a.step(D[i], C[i], U[i - 1])
    want = _snapshot(a)
    # a fresh handle on other buffers, from the device and from the host checkpoint
    for src in (dev_ck, host_ck):
        b = _filter(c, **kw)
        b.step(D[7], C[7], None)                # some other history, overwritten by the load
        b.load(src)
        for i in range(4, 7):
            b.step(D[i], C[i], U[i - 1])
        got = _snapshot(b)
        for k, (x, y) in enumerate(zip(got, want)):
            assert x == y, f"part {k} of the belief differs after restoring ({'device' if src.is_cuda else 'host'})"
        del b
    # the saved handle itself, rewound
    a.load(dev_ck)
    for i in range(4, 7):
        a.step(D[i], C[i], U[i - 1])
    assert _snapshot(a) == want


def test_checkpoint_rejects_other_filters(traj):
    banner("checkpoint validation")
    c = traj
    a = _filter(c)
    ck = a.save()
    torch.cuda.synchronize()
    # another grid
    c2 = synth.trajectory_case(seed=2, n=64, width=160, height=120, n_samples=64, n_frames=1)
    b = _filter(c2)
    big = torch.zeros(max(ck.numel(), b.save_bytes()), dtype=torch.uint8, device=DEV)
    big[:ck.numel()] = ck
    with pytest.raises(P().PrismError, match="grid differs|sizes"):
        b.load(big)
    # not a checkpoint
    with pytest.raises(P().PrismError, match="magic"):
        a.load(torch.zeros_like(ck))
    # too small
    with pytest.raises(P().PrismError, match="hold"):
        a.load(ck[:1024].contiguous())
    with pytest.raises(P().PrismError, match="save_bytes"):
        a.save(torch.empty(1024, dtype=torch.uint8, device=DEV))


def test_capture_error_status(traj):
    """Calls that cannot run inside a stream capture say so with
    PRISM_CAPTURE_ERROR and queue nothing."""
    banner("capture error status")
    c = traj
    D, C, U = _frames(c)
    f = _filter(c)
    f.step(D[0], C[0], None)
    torch.cuda.synchronize()
    ck = f.save()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    x = torch.zeros(1, device=DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        x += 1
        with torch.cuda.graph(g, stream=s):
            x += 1                                    # recorded, runs at replay
            with pytest.raises(P().PrismError, match="status 5"):
                f.step_graph(D[1], C[1], U[0], s)
            with pytest.raises(P().PrismError, match="status 5"):
                f.load(ck, stream=s)
    g.replay()
    torch.cuda.synchronize()
    assert int(f.state().step) == 1
    assert x.item() == 2.0


def test_low_inliers_flag(traj):
    """PRISM_FLAG_LOW_INLIERS is raised exactly when the final objective has
    fewer contributing pixels than min_inlier_frac of the image."""
    banner("low-inlier flag")
    c = traj
    D, C, U = _frames(c)
    H, W = c["cam"].height, c["cam"].width
    f = _filter(c, min_inlier_frac=0.1)
    f.step(D[0], C[0], None)
    f.step(D[1], C[1], U[0])
    s = f.state()
    assert s.neq[28] >= 0.1 * W * H and not (s.flags & P().FLAG_LOW_INLIERS), (s.neq[28], s.flags)
    # a frame with valid depth on a small patch only
    d2 = torch.zeros_like(D[2])
    d2[:20, :30] = D[2][:20, :30]
    f.step(d2, C[2], U[1])
    s = f.state()
    limit = int(np.ceil(0.1 * W * H))
    assert 0 < s.neq[28] < limit, s.neq[28]
    assert s.flags & P().FLAG_LOW_INLIERS, s.flags
    # the flag is cleared by the next step with enough pixels
    f.step(D[3], C[3], U[2])
    s = f.state()
    assert s.neq[28] >= limit and not (s.flags & P().FLAG_LOW_INLIERS)
