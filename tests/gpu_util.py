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


def neq_check(a, b, label="", rtol=1e-4, floor=1e-2):
    """The 29 normal-equation entries of a frame compared one by one.

    Each entry is held to rtol times max(|entry|, its scale).  A pixel's rows
    are single precision, each entry off by ~1e-7 of the row's norm, so the
    error of H_ab is bounded by ~1e-7 sum_rows w |row|^2 = 1e-7 trace(H) and
    that of g_a by ~1e-7 sqrt(trace(H) cost); sums over pixels can cancel
    down to that level.  Scales: for H_ab, floor x the Cauchy-Schwarz bound
    sqrt(H_aa H_bb) or 1e-4 x trace(H), whichever is larger; for g_a, floor x
    sqrt(H_aa cost) or 1e-4 x sqrt(trace(H) cost).  The cost (a sum of non-
    negative terms) is compared relatively and the count of contributing
    pixels exactly.  Returns the largest scaled errors."""
    import oracle as orc
    Ha, ga, ca, na = orc.neq_unpack(np.asarray(a, np.float64))
    Hb, gb, cb, nb = orc.neq_unpack(np.asarray(b, np.float64))
    assert na == nb, f"{label}: contributing pixels {na} vs {nb}"
    tr = float(np.trace(Hb))
    dg = np.sqrt(np.maximum(np.diag(Hb), 0.0))
    cb_ = max(cb, 0.0)
    sH = np.maximum(np.abs(Hb), np.maximum(floor * np.outer(dg, dg), 1e-4 * tr))
    sg = np.maximum(np.abs(gb), np.maximum(floor * dg * np.sqrt(cb_), 1e-4 * np.sqrt(tr * cb_)))
    eH = np.abs(Ha - Hb) / np.where(sH > 0, sH, 1.0)
    eg = np.abs(ga - gb) / np.where(sg > 0, sg, 1.0)
    ec = abs(ca - cb) / max(cb, 1e-300)
    stats = dict(H=float(eH.max()), g=float(eg.max()), cost=float(ec), count=int(nb))
    print(f"[neq {label}] max scaled error H {stats['H']:.2e} g {stats['g']:.2e} cost {stats['cost']:.2e} "
          f"(count {int(nb)})", flush=True)
    assert stats["H"] <= rtol and stats["g"] <= rtol and stats["cost"] <= rtol, (label, stats)
    return stats


def rows_check(J, R, label="", rtol=1e-4, floor=1e-3):
    """Jacobian rows [pixels, 4, 6] compared element by element, each entry
    held to rtol x max(|entry|, norm of its row, floor x the largest row norm
    of its pixel).  A row's entries are single-precision sums whose rounding
    scales with the row, so an entry that cancels to ~0 is judged against its
    row; a colour row that is zero up to rounding (a flat colour patch, where
    the two samples' colours differ by an ulp of double precision times
    d(alpha)) is judged against the pixel's depth row."""
    J = np.asarray(J, np.float64)
    R = np.asarray(R, np.float64)
    norms = np.linalg.norm(R, axis=-1, keepdims=True)
    pix = norms.max(axis=-2, keepdims=True)
    scale = np.maximum(np.maximum(np.abs(R), norms), floor * pix)
    err = np.abs(J - R) / np.where(scale > 0, scale, 1.0)
    e = float(err.max()) if err.size else 0.0
    print(f"[rows {label}] {J.shape[0]} pixels, max scaled error {e:.2e}, 99.9% "
          f"{float(np.quantile(err.max(-1), 0.999)) if err.size else 0.0:.2e}", flush=True)
    assert e <= rtol, (label, e)
    return e
