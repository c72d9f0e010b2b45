"""Serving loop: admission by memory, continuous launching, per-slot graph
replay, and results that do not depend on the mix."""
import numpy as np
import pytest

import synth


def _specs(n_streams=4, n_frames=8, dtype=None):
    from gpu_util import P
    from paper_2212_02988_amd.serving import StreamSpec
    Pm = P()
    dtype = Pm.PRISM_BF16 if dtype is None else dtype
    streams = synth.serving_streams(n_streams, n_frames, sizes=((80, 60), (160, 120)), grids=(64, 128))
    specs, frames = [], {}
    import torch
    for i, s in enumerate(streams):
        sc, cm, tr = s["scene"], s["cam"], s["traj"]
        grid = Pm.Grid.make(sc.n, sc.voxel, tuple(float(v) for v in sc.origin), dtype=dtype)
        cam = Pm.Camera.make(cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy, cm.d_near, cm.d_far, cm.n_samples)
        x0 = np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]])
        P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
        specs.append(StreamSpec(i, grid, cam, Pm.FilterParams(), x0, P0, n_frames))
        D, C = synth.raycast_torch(sc, cm, tr.t, tr.q, s["seed"], 0.01, 0.02)
        U = torch.tensor(tr.u, dtype=torch.float64, device="cuda")
        frames[i] = (D, C, U, s["arrivals"])
    torch.cuda.synchronize()
    return specs, frames


def _source(frames, host=False):
    def get(sid, k):
        D, C, U, _ = frames[sid]
        u = None if k == 0 else U[k - 1]
        if host:
            return D[k].cpu().numpy(), C[k].cpu().numpy(), None if u is None else u.cpu().numpy()
        return D[k], C[k], u
    return get


def _schedule(specs, frames, ids=None):
    ids = [s.stream_id for s in specs] if ids is None else ids
    sched = [(float(frames[i][3][k]), i, k) for i in ids for k in range(specs[i].n_frames)]
    return sorted(sched)


def _run(specs, frames, ids, realtime=False, **kw):
    from paper_2212_02988_amd.serving import ServingLoop, run_schedule
    host = kw.pop("host", False)
    loop = ServingLoop(keep_final=True, staged=host, **kw)
    wall = run_schedule(loop, [specs[i] for i in ids], _schedule(specs, frames, ids), _source(frames, host),
                        realtime=realtime, timeout=120)
    return loop, wall


def _same(a, b):
    sa, sb = a["state"], b["state"]
    assert bytes(sa) == bytes(sb), "filter state differs"
    assert np.array_equal(a["mean"].numpy(), b["mean"].numpy())
    assert np.array_equal(a["var"].numpy(), b["var"].numpy())


@pytest.mark.gpu
def test_serving_alone_equals_mix_and_admission():
    from gpu_util import banner
    from paper_2212_02988_amd.serving import footprint_bytes
    banner("serving 4 streams: alone vs mix, admission by memory")
    specs, frames = _specs()
    ids = [s.stream_id for s in specs]
    alone = {}
    for i in ids:
        loop, _ = _run(specs, frames, [i])
        assert loop.completed == specs[i].n_frames
        alone[i] = loop.final[i]
        st = alone[i]["state"]
        assert st.step == specs[i].n_frames and st.flags == 0
    mix, _ = _run(specs, frames, ids, n_hip_streams=2)
    assert mix.completed == sum(s.n_frames for s in specs) and mix.max_concurrent == len(ids)
    for i in ids:
        _same(alone[i], mix.final[i])
    # a budget below the sum of all footprints: some streams wait for memory
    fp = sorted(footprint_bytes(s) for s in specs)
    tight, _ = _run(specs, frames, ids, hbm_budget=fp[-1] + fp[-2])
    assert tight.max_concurrent < len(ids) and tight.max_held_bytes <= tight.budget
    assert tight.completed == mix.completed
    for i in ids:
        _same(alone[i], tight.final[i])


@pytest.mark.gpu
def test_serving_graph_eager_and_staged_agree():
    from gpu_util import banner
    banner("serving: batched vs per-stream graph replay vs eager, host-staged vs resident frames")
    specs, frames = _specs(n_streams=3, n_frames=6)
    ids = [s.stream_id for s in specs]
    ref, _ = _run(specs, frames, ids, batched=False, use_graphs=False, depth=1)
    for kw in (dict(batched=False, use_graphs=True, depth=2), dict(batched=True, depth=2),
               dict(batched=True, depth=3, host=True, n_hip_streams=1)):
        got, _ = _run(specs, frames, ids, **kw)
        for i in ids:
            _same(ref.final[i], got.final[i])


@pytest.mark.gpu
def test_serving_waits_for_frames_from_another_stream():
    """Device frames written on a producer stream (behind a spin) and pushed
    with the producer's event: the agents' streams wait for them, so the
    results equal a run on frames that were complete when pushed."""
    import torch
    from gpu_util import banner
    banner("serving: frames produced on another HIP stream, pushed with an event")
    specs, frames = _specs(n_streams=2, n_frames=5)
    ids = [s.stream_id for s in specs]
    ref, _ = _run(specs, frames, ids)
    prod = torch.cuda.Stream()
    keep = []

    def produced(sid, k):
        D, C, U, _ = frames[sid]
        with torch.cuda.stream(prod):
            torch.cuda._sleep(2_000_000)                 # the producer is still busy when the step is launched
            d, c = D[k].clone(), C[k].clone()
            u = None if k == 0 else U[k - 1].clone()
            ev = torch.cuda.Event()
            ev.record(prod)
        keep.append((d, c, u))
        return d, c, u, ev

    from paper_2212_02988_amd.serving import ServingLoop, run_schedule
    loop = ServingLoop(keep_final=True)
    run_schedule(loop, [specs[i] for i in ids], _schedule(specs, frames, ids), produced, realtime=False, timeout=120)
    for i in ids:
        _same(ref.final[i], loop.final[i])


@pytest.mark.gpu
def test_serving_realtime_latency_and_budget_errors():
    from gpu_util import banner, P
    from paper_2212_02988_amd.serving import ServingLoop
    banner("serving: real-time arrivals, latency accounting, oversize stream")
    specs, frames = _specs(n_streams=3, n_frames=10)
    ids = [s.stream_id for s in specs]
    loop, wall = _run(specs, frames, ids, realtime=True)
    st = loop.stats()
    assert st["completed"] == 30 and len(loop.latencies) == 30
    last_arrival = max(frames[i][3][-1] for i in ids)
    assert wall >= last_arrival
    assert 0 < st["p50_ms"] <= st["p99_ms"] < 1000
    small = ServingLoop(hbm_budget=1 << 20)
    with pytest.raises(P().PrismError):
        small.open_stream(specs[0])


@pytest.mark.gpu
def test_step_graph_matches_step_via_c_abi():
    """prism_filter_step_graph (recorded per input slot) against
    prism_filter_step, bit for bit, over 6 frames alternating two slots."""
    import torch
    from gpu_util import banner, P
    banner("prism_filter_step_graph vs prism_filter_step")
    Pm = P()
    specs, frames = _specs(n_streams=1, n_frames=6, dtype=Pm.PRISM_F32)
    sp = specs[0]
    D, C, U, _ = frames[0]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fa = Pm.Filter(sp.grid, sp.cam, sp.params)
        fb = Pm.Filter(sp.grid, sp.cam, sp.params)
        slots = [(torch.empty_like(D[0]), torch.empty_like(C[0]), torch.empty_like(U[0])) for _ in range(2)]
        for f in (fa, fb):
            f.map.init(stream=s)
            f.reset(sp.x0, sp.P0, stream=s)
        for k in range(sp.n_frames):
            u = None if k == 0 else U[k - 1]
            fa.step(D[k], C[k], u, stream=s)
            d, c, uu = slots[k % 2]
            d.copy_(D[k]); c.copy_(C[k])
            if u is not None:
                uu.copy_(u)
            fb.step_graph(d, c, None if u is None else uu, stream=s)
    torch.cuda.synchronize()
    assert bytes(fa.state()) == bytes(fb.state())
    ma, va = fa.map.to_dense()
    mb, vb = fb.map.to_dense()
    assert torch.equal(ma, mb) and torch.equal(va, vb)


@pytest.mark.gpu
def test_submit_poll_via_c_abi():
    """prism_filter_submit / prism_filter_poll: two slots, steps replayed from
    per-slot graphs, bit for bit equal to prism_filter_step; a third
    submission while both slots are in flight is refused (PRISM_BUSY) and
    queues nothing; completions arrive in order."""
    import torch
    from gpu_util import banner, P
    banner("prism_filter_submit / prism_filter_poll")
    Pm = P()
    specs, frames = _specs(n_streams=1, n_frames=6)
    sp = specs[0]
    D, C, U, _ = frames[0]
    H, W = sp.cam.height, sp.cam.width
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fa = Pm.Filter(sp.grid, sp.cam, sp.params)
        fb = Pm.Filter(sp.grid, sp.cam, sp.params)
        for f in (fa, fb):
            f.map.init(stream=s)
            f.reset(sp.x0, sp.P0, stream=s)
        fb.set_slots([(torch.empty((H, W), device="cuda"), torch.empty((H, W, 3), device="cuda"),
                       torch.zeros(6, dtype=torch.float64, device="cuda")) for _ in range(2)])
        for k in range(sp.n_frames):
            fa.step(D[k], C[k], None if k == 0 else U[k - 1], stream=s)
    torch.cuda.synchronize()
    assert fb.poll() == 0
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)            # keep the stream busy so both slots stay in flight
    seqs = [fb.submit(D[0], C[0], None, stream=s), fb.submit(D[1], C[1], U[0], stream=s)]
    assert seqs == [0, 1]
    assert fb.submit(D[2], C[2], U[1], stream=s) is None
    torch.cuda.synchronize()
    assert fb.poll() == 2
    for k in range(2, sp.n_frames):
        while fb.submit(D[k], C[k], U[k - 1], stream=s) is None:
            pass
    torch.cuda.synchronize()
    assert fb.poll() == sp.n_frames
    assert bytes(fa.state()) == bytes(fb.state())
    ma, va = fa.map.to_dense()
    mb, vb = fb.map.to_dense()
    assert torch.equal(ma, mb) and torch.equal(va, vb)


@pytest.mark.gpu
@pytest.mark.parametrize("graphs", [False, True])
def test_step_batch_matches_single_steps(graphs):
    """prism_filter_step_batch over filters of different image sizes, grid
    sizes, storage types, objectives (P2 and the render-through P1),
    Gauss-Newton counts and paper modes (IRLS rows beside plain ones in one
    launch), one of them joining (first frame) while the others
    are mid-trajectory: every filter's state and map equal its own sequence
    of prism_filter_step calls, bit for bit -- with every batch launched
    stage by stage, and replayed from the graphs recorded per member set,
    slots and first-frame states (graphs=True)."""
    import dataclasses
    import torch
    from gpu_util import banner, P
    banner(f"prism_filter_step_batch vs single steps (mixed batch, graphs={graphs})")
    Pm = P()
    specs, frames = _specs(n_streams=4, n_frames=6)
    all_modes = Pm.MODE_TRANSITION_DT2 | Pm.MODE_LAPLACE_FACTOR1 | Pm.MODE_IRLS_L1 | Pm.MODE_ACCEL_BIAS
    kinds = [(Pm.PRISM_F32, 3, Pm.OBJ_P2, 0), (Pm.PRISM_BF16, 2, Pm.OBJ_P1, Pm.MODE_IRLS_L1),
             (Pm.PRISM_BF16, 3, Pm.OBJ_P2, all_modes), (Pm.PRISM_F32, 1, Pm.OBJ_P1, Pm.MODE_ACCEL_BIAS)]
    for sp, (dt, ngn, obj, modes) in zip(specs, kinds):
        sp.grid = Pm.Grid.make(sp.grid.n, sp.grid.voxel, tuple(sp.grid.origin), dtype=dt)
        sp.params = dataclasses.replace(sp.params, n_gn=ngn, objective=obj, modes=modes)
    # the 15-D members take the accelerometer's body-frame force and a 15-D belief
    streams = synth.serving_streams(4, 6, sizes=((80, 60), (160, 120)), grids=(64, 128))
    for i in (2, 3):
        D_, C_, _, arr = frames[i]
        frames[i] = (D_, C_, torch.tensor(streams[i]["traj"].u_body, dtype=torch.float64, device="cuda"), arr)
        specs[i].x0 = np.concatenate([specs[i].x0, np.zeros(3)])
        specs[i].P0 = np.diag([1e-6] * 6 + [1e-4] * 6 + [1e-4] * 3)
    join = {0: 0, 1: 0, 2: 0, 3: 2}        # frame index at which each filter starts
    s = torch.cuda.Stream()
    ref, bat = [], []
    with torch.cuda.stream(s):
        for sp in specs:
            H, W = sp.cam.height, sp.cam.width
            fa = Pm.Filter(sp.grid, sp.cam, sp.params)
            fb = Pm.Filter(sp.grid, sp.cam, sp.params)
            for f in (fa, fb):
                f.map.init(stream=s)
                f.reset(sp.x0, sp.P0, stream=s)
            fb.set_slots([(torch.empty((H, W), device="cuda"), torch.empty((H, W, 3), device="cuda"),
                           torch.zeros(6, dtype=torch.float64, device="cuda")) for _ in range(2)])
            ref.append(fa)
            bat.append(fb)
        for t in range(6):
            members, srcs = [], []
            for i, sp in enumerate(specs):
                k = t - join[i]
                if k < 0:
                    continue
                D, C, U, _ = frames[i]
                u = None if k == 0 else U[k - 1]
                ref[i].step(D[k], C[k], u, stream=s)
                members.append(bat[i])
                srcs.append((D[k], C[k], u))
            assert Pm.filter_step_batch(members, srcs, stream=s, flags=Pm.SUBMIT_GRAPH if graphs else 0)
            torch.cuda.synchronize()          # both slots are reused across iterations
    torch.cuda.synchronize()
    assert Pm.filters_poll(bat) == [6, 6, 6, 4]
    for i, (fa, fb) in enumerate(zip(ref, bat)):
        assert bytes(fa.state()) == bytes(fb.state())
        if i in (2, 3):
            assert bytes(fa.bias_state()) == bytes(fb.bias_state())
        ma, va = fa.map.to_dense()
        mb, vb = fb.map.to_dense()
        assert torch.equal(ma, mb) and torch.equal(va, vb)
        aa, ab = fa.anchor(), fb.anchor()
        for key in aa:
            assert torch.equal(aa[key], ab[key]), key
