"""Timing of the FP64 oracle on the benchmark workloads (test
infrastructure: run by bench.py's CPU-baseline leg, never by the library).

    python -m oracle.timing --config N [--frames F]

prints one JSON line with the wall time of the workload of config N on the
threads OpenMP was started with (set OMP_NUM_THREADS before launching: the
thread count is fixed when the oracle's library loads):

1. single frame, 64^3 (4 cm), 80x60, K = 32, FP64: render-through Jacobian
   at the perturbed pose against the oracle's render at the true pose, one
   Gauss-Newton step, Laplace covariance, map update onto the prior map;
2. single-stream trajectory, 256^3 (2.5 cm), 320x240, K = 128: the first F
   frames of the filter (P2, 3 Gauss-Newton iterations) from the prior map,
   plus one render and one map update on their own;
3. adjoint, 256^3 ground-truth map, 320x240, K = 128: one frame of the
   renderer's adjoint with random upstream gradients;
4. mixed-precision workload, 384^3 (1.67 cm), 640x480, K = 192: the first F
   frames of the filter with the 15-D state (accelerometer bias, 15x15
   covariance; the accelerometer's body-frame force as the linear control)
   on BF16-rounded inputs (the oracle computes in FP64 either way).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
import synth  # noqa: E402


def _prior(n):
    mean = np.zeros((4, n, n, n))
    mean[0] = -0.001
    return mean, np.full((4, n, n, n), 1e4)


def config1(reps=50):
    c = synth.single_frame_case(0)
    g, cam, p = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"]), orc.Params(n_gn=1, objective="p1")
    mean, _ = synth.gt_map(c["scene"])
    obs = orc.render(g, mean, cam, synth.pose7(c["t_gt"], c["q_gt"]))
    pose = synth.pose7(c["t_init"], c["q_init"])
    Lp = np.diag(1.0 / np.array([0.05, 0.05, 0.05, 0.02, 0.02, 0.02]) ** 2)
    wall, n_upd = 0.0, 0
    for _ in range(reps):
        pm, pv = _prior(g.n)
        t0 = time.perf_counter()
        jr = orc.render_jacobian(g, mean, cam, pose, obs["depth"], obs["rgb"], p)
        delta = orc.gn_solve(jr["neq"], Lp, np.zeros(6))
        post = orc.retract(pose, delta)
        jr2 = orc.render_jacobian(g, mean, cam, post, obs["depth"], obs["rgb"], p)
        orc.laplace(jr2["neq"], Lp)
        n_upd = orc.map_update(g, pm, pv, cam, post, obs["depth"], obs["rgb"], p)
        wall += time.perf_counter() - t0
    return {"seconds": wall / reps, "sequences_per_s": reps / wall,
            "unit_note": f"one single-frame sequence (render+Jacobian, GN step, render+Jacobian at the step, "
                         f"Laplace, map update), mean of {reps}", "voxels_updated": n_upd}


def _filter_frames(n, width, height, K, frames, bf16=False, seed=1, bias=False):
    c = synth.trajectory_case(seed=seed, n=n, width=width, height=height, n_samples=K, n_frames=frames)
    tr = c["traj"]
    g, cam = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
    mean, var = _prior(n)
    if bf16:
        mean = synth.bf16_round(mean).astype(np.float64)
        var = synth.bf16_round(var).astype(np.float64)
    x0 = dict(t=tr.t[0], q=tr.q[0], v=tr.v[0], w=tr.w[0])
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6)
    if bias:
        x0["b"] = np.zeros(3)
        P0 = np.diag([1e-6] * 6 + [1e-4] * 6 + [1e-4] * 3)
    f = orc.Filter(g, cam, orc.Params(accel_bias=bias), x0, P0, mean, var)
    u = tr.u_body if bias else tr.u
    del mean, var
    times = []
    for i in range(frames):
        d = c["depth"][i].astype(np.float64)
        rgb = c["rgb"][i].astype(np.float64)
        t0 = time.perf_counter()
        f.step(d, rgb, u[i - 1] if i else None)
        times.append(time.perf_counter() - t0)
    # one render and one map update on their own, at the last pose
    pose = f.s.pose
    t0 = time.perf_counter()
    orc.render(g, f.mean, cam, pose)
    t_render = time.perf_counter() - t0
    t0 = time.perf_counter()
    nu = orc.map_update(g, f.mean, f.var, cam, pose, c["depth"][-1].astype(np.float64),
                        c["rgb"][-1].astype(np.float64), orc.Params())
    t_upd = time.perf_counter() - t0
    steady = times[1:] if len(times) > 1 else times
    return {"seconds": float(sum(times)), "frames": frames, "filter_steps_per_s": len(steady) / sum(steady),
            "render_rays_per_s": width * height / t_render, "map_voxel_updates_per_s": nu / t_upd,
            "unit_note": f"{frames} filter frames (first frame: map update and anchor only)"}


def config3():
    c = synth.trajectory_case(seed=1, n=256, width=320, height=240, n_samples=128, n_frames=1, frames=False)
    g, cam = orc.grid_from_scene(c["scene"]), orc.cam_from(c["cam"])
    mean, _ = synth.gt_map(c["scene"])
    rng = np.random.default_rng(3)
    gd = rng.normal(size=(240, 320))
    gc = rng.normal(size=(240, 320, 3))
    pose = synth.pose7(c["traj"].t[0], c["traj"].q[0])
    t0 = time.perf_counter()
    orc.render_vjp(g, mean, cam, pose, gd, gc)
    wall = time.perf_counter() - t0
    return {"seconds": wall, "adjoint_rays_per_s": 320 * 240 / wall, "unit_note": "one frame of the adjoint"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, required=True, choices=(1, 2, 3, 4))
    ap.add_argument("--frames", type=int, default=20)
    a = ap.parse_args()
    orc.build(force=False)
    if a.config == 1:
        out = config1()
    elif a.config == 2:
        out = _filter_frames(256, 320, 240, 128, a.frames)
    elif a.config == 3:
        out = config3()
    else:
        out = _filter_frames(384, 640, 480, 192, a.frames, bf16=True, seed=4, bias=True)
    out.update(config=a.config, threads=int(os.environ.get("OMP_NUM_THREADS", "0")) or None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
