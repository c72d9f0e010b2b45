"""Helpers shared by the GPU parity tests: build the same seeded inputs for
the HIP library and for the FP64 oracle, and compare with stated tolerances."""
from __future__ import annotations

import numpy as np
import torch

import synth

DEV = "cuda"

# Tolerances (GPU single precision against the FP64 oracle)
DEPTH_RTOL = 1e-4      # |a-b| <= 1e-4 max(|b|, 1e-3 m)
RGB_RTOL = 1e-4        # |a-b| <= 1e-4 max(|b|, 1e-2)
POSE_T_TOL = 1e-5      # m
POSE_R_TOL = 1e-5      # rad


def banner(msg: str):
    print(f"[gpu-test] {msg}", flush=True)


def P():
    import paper_2212_02988_amd as pkg
    return pkg.prism


def grid_of(scene, dtype=0):
    return P().Grid.make(scene.n, scene.voxel, tuple(float(v) for v in scene.origin), dtype)


def cam_of(c):
    return P().Camera.make(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.d_near, c.d_far, c.n_samples, c.tau)


def gpu_map(grid, mean, var):
    """Upload dense float32 mean/var into a device map of `grid`'s dtype."""
    vm = P().VoxelMap(grid)
    vm.from_dense(torch.from_numpy(np.ascontiguousarray(mean, np.float32)).to(DEV),
                  torch.from_numpy(np.ascontiguousarray(var, np.float32)).to(DEV))
    return vm


def oracle_map_values(mean, dtype):
    """The exact values the GPU map holds, as float64 for the oracle."""
    m32 = np.asarray(mean, np.float32)
    if dtype == 1:
        m32 = synth.bf16_round(m32)
    return m32.astype(np.float64)


def depth_close(a, b, rtol=DEPTH_RTOL):
    return np.abs(a - b) <= rtol * np.maximum(np.abs(b), 1e-3)


def rgb_close(a, b, rtol=RGB_RTOL):
    return np.abs(a - b) <= rtol * np.maximum(np.abs(b), 1e-2)


def rot_angle(qa, qb):
    from oracle import quat_to_rot, so3_log
    return float(np.linalg.norm(so3_log(quat_to_rot(qa) @ quat_to_rot(qb).T)))


def t(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)
