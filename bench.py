#!/usr/bin/env python
"""Benchmark of the PRISM filter hot path on one MI355X.

Workload: single-stream trajectory, 256^3 grid (2.5 cm voxels, 6.4 m room),
320x240 RGB-D frames, 128 samples per ray, FP32 map, prediction-to-
observation objective with 3 Gauss-Newton iterations.  One step = one full
filter step (predict/split, 3 x (track + GN solve), final track + Laplace +
combine, map update, anchor render + normals), replayed from a HIP graph with
the frame's observation already resident in HBM.

Prints one JSON line (rank 0).  Besides steps/s it reports p50/p99 step
latency, render+Jacobian Mrays/s, the roofline of the dominant kernel and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--eager", action="store_true", help="launch each step eagerly instead of a graph")
    ap.add_argument("--calib", action="store_true", help="also run a 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported (each agent stream is "
              "independent; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2212_02988_amd import prism as P

    dev = "cuda"
    torch.cuda.set_device(0)
    n_frames = 2 + args.warmup + args.steps
    N, Wd, Ht, K = 256, 320, 240, 128
    t0 = time.time()
    case = synth.trajectory_case(seed=1, n=N, width=Wd, height=Ht, n_samples=K, n_frames=min(n_frames, 300))
    log(f"inputs generated in {time.time() - t0:.1f}s")
    tr = case["traj"]
    nf = len(tr.t)
    scene = case["scene"]
    cm = case["cam"]
    grid = P.Grid.make(N, scene.voxel, tuple(float(v) for v in scene.origin))
    cam = P.Camera.make(cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy, cm.d_near, cm.d_far, cm.n_samples)
    params = P.FilterParams(n_gn=3, objective=P.OBJ_P2)
    D = torch.from_numpy(case["depth"]).to(dev)
    C = torch.from_numpy(case["rgb"]).to(dev)
    U = torch.from_numpy(np.concatenate([tr.u, tr.u[-1:]], 0)).to(dev)       # [nf, 6]
    f = P.Filter(grid, cam, params)
    f.map.init()
    x0 = np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    f.reset(x0, P0)
    f.step(D[0], C[0], None)
    torch.cuda.synchronize()

    # Each filter step is one HIP graph (13 kernels) reading its frame
    # straight from the resident frame array; the timed region replays one
    # graph per step, with events on the stream between steps for the
    # per-step latencies (the launch of each graph is inside the timing).
    stream = torch.cuda.Stream()
    f.step(D[1], C[1], U[0], stream=stream)        # first step past the initial frame, eager
    torch.cuda.synchronize()
    t0 = time.time()
    graphs = []
    for i in range(2, 2 + args.warmup + args.steps):
        if args.eager:
            graphs.append(i)
            continue
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=stream):
            f.step(D[i], C[i], U[i - 1])
        graphs.append(gr)
    torch.cuda.synchronize()
    log(f"{len(graphs)} step graphs captured in {time.time() - t0:.2f}s")
    graph = None if args.eager else graphs[0]

    def run_step(j):
        if args.eager:
            i = graphs[j]
            f.step(D[i], C[i], U[i - 1], stream=stream)
        else:
            graphs[j].replay()

    with torch.cuda.stream(stream):
        for j in range(args.warmup):
            run_step(j)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    wall0 = time.perf_counter()
    with torch.cuda.stream(stream):
        evs[0].record()
        for j in range(args.steps):
            run_step(args.warmup + j)
            evs[j + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    st = f.state()
    last = int(st.step) - 1                      # frame index of the last step
    pos_err = float(np.linalg.norm(np.array(st.pose.t) - tr.t[min(last, nf - 1)]))
    log(f"{args.steps} steps: {ms_per_step:.3f} ms/step (events), wall {wall * 1e3 / args.steps:.3f} ms/step, "
        f"pos err {pos_err:.4f} m (frame {last}), flags {st.flags}")
    if args.calib:
        # plain copy of known size for scaling the FETCH_SIZE / WRITE_SIZE counters
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # ---- render + Jacobian throughput (render-through P1 objective) ------------------
    poses = P.poses_tensor(np.stack([np.concatenate([tr.t[i], tr.q[i]]) for i in range(8)]))
    ws = torch.empty(P.workspace_bytes(cam, 8), dtype=torch.uint8, device=dev)
    rj = dict(neq=torch.empty((8, 29), dtype=torch.float64, device=dev))
    obs_d, obs_c = D[:8].contiguous(), C[:8].contiguous()
    w = P.Weights.make()

    def timed(fn, reps):
        with torch.cuda.stream(stream):
            fn()
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_rj1 = timed(lambda: P.render_jacobian(grid, f.map, cam, poses[:1], obs_d[:1], obs_c[:1], w, want_render=False,
                                             ws=ws, out=dict(neq=rj["neq"][:1])), 50)
    ms_rj8 = timed(lambda: P.render_jacobian(grid, f.map, cam, poses, obs_d, obs_c, w, want_render=False, ws=ws,
                                             out=rj), 20)
    rays = Wd * Ht
    mrays_1 = rays / (ms_rj1 * 1e-3) / 1e6
    mrays_8 = 8 * rays / (ms_rj8 * 1e-3) / 1e6

    # ---- map update: the HBM-streaming kernel -----------------------------------------
    nup = torch.empty(1, dtype=torch.int64, device=dev)
    pose_last = P.poses_tensor(np.concatenate([np.array(st.pose.t), np.array(st.pose.q)]))
    fi = max(1, min(last, nf - 1))
    ms_mu = timed(lambda: P.map_update(grid, f.map, cam, pose_last, D[fi], C[fi], 4 * grid.voxel, 1.0,
                                       n_updated=nup), 50)
    n_upd = int(nup.item())
    mu_bytes = n_upd * 64 + Wd * Ht * 16
    mu_gbs = mu_bytes / (ms_mu * 1e-3) / 1e9

    # anchor render alone (per step)
    rout = P.render(grid, f.map, cam, pose_last)
    ms_r = timed(lambda: P.render(grid, f.map, cam, pose_last, out=rout), 50)
    log(f"render_jacobian: 1 frame {ms_rj1 * 1e3:.1f} us ({mrays_1:.0f} Mrays/s), 8 frames {ms_rj8 * 1e3:.1f} us "
        f"({mrays_8:.0f} Mrays/s); render {ms_r * 1e3:.1f} us; map_update {ms_mu * 1e3:.1f} us, "
        f"{n_upd} voxels, {mu_gbs:.0f} GB/s")

    # ---- CPU oracle baseline ------------------------------------------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(case, args.cpu_seconds)

    out = {
        "metric": "filter steps/s & p99 step latency (16 streams); Mrays/s render+Jacobian",
        "value": round(1000.0 / ms_per_step, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "p50_ms": round(float(np.percentile(per, 50)), 4),
        "p99_ms": round(float(np.percentile(per, 99)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single-stream trajectory: 256^3 grid (2.5 cm), 320x240 RGB-D, 128 samples/ray, "
                               "P2 objective, 3 Gauss-Newton iterations, FP32 map",
                   "grid": N, "width": Wd, "height": Ht, "samples": K, "n_gn": 3,
                   "launch": "eager" if graph is None else "hip-graph"},
        "render_jacobian_mrays_per_s": {"1_frame": round(mrays_1, 1), "8_frames": round(mrays_8, 1)},
        "kernels_us": {"render_jacobian_1f": round(ms_rj1 * 1e3, 2), "render": round(ms_r * 1e3, 2),
                       "map_update": round(ms_mu * 1e3, 2)},
        "roofline": {"kernel": "map_update", "bound": "hbm", "achieved": round(mu_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(mu_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes": mu_bytes, "updated_voxels": n_upd},
        "cpu_baseline": cpu,
        "pos_err_m": round(pos_err, 4),
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(case, budget_s):
    """FP64 oracle filter steps on the same frames, until ~budget_s of CPU work."""
    import oracle as orc
    tr = case["traj"]
    scene = case["scene"]
    g = orc.grid_from_scene(scene)
    cam = orc.cam_from(case["cam"])
    n = scene.n
    mean = np.zeros((4, n, n, n)); mean[0] = -0.001
    var = np.full((4, n, n, n), 1e4)
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    f = orc.Filter(g, cam, orc.Params(n_gn=3, objective="p2"),
                   dict(t=tr.t[0], q=tr.q[0], v=tr.v[0], w=tr.w[0]), P0, mean, var)
    f.step(case["depth"][0].astype(np.float64), case["rgb"][0].astype(np.float64), None)
    t0 = time.perf_counter()
    k = 0
    while k + 1 < len(tr.t):
        k += 1
        f.step(case["depth"][k].astype(np.float64), case["rgb"][k].astype(np.float64), tr.u[k - 1])
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    return {"value": round(k / dt, 4), "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} filter steps (frames 1..{k}) of the same workload after the first frame, "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
