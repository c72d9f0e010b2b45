"""Thin Python binding of libprism.so (the C ABI in include/prism.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory and the stream; tensors passed
in must already live on the GPU with the dtype and shape each call states.
There is no CPU fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprism.so")

PRISM_F32, PRISM_BF16 = 0, 1
OBJ_P2, OBJ_P1 = 0, 1
FLAG_NO_VALID_PIXELS, FLAG_CHOL_FALLBACK, FLAG_PRIOR_NOT_PD, FLAG_LOW_INLIERS = 1, 2, 4, 8
# the paper's literal forms (prism_filter_cfg.modes)
MODE_TRANSITION_DT2, MODE_LAPLACE_FACTOR1, MODE_IRLS_L1, MODE_ACCEL_BIAS = 1, 2, 4, 8
NEQ = 29


PRISM_BUSY = 4
PRISM_CAPTURE_ERROR = 5
SUBMIT_FROM_HOST = 1
SUBMIT_EAGER = 2
SUBMIT_GRAPH = 4


class PrismError(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# C structs
# ---------------------------------------------------------------------------
class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("voxel", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("occ_out", ctypes.c_double), ("rgb_out", ctypes.c_double),
                ("capacity", ctypes.c_int64)]

    @staticmethod
    def make(n: int, voxel: float, origin=(0.0, 0.0, 0.0), dtype: int = PRISM_F32,
             occ_out: float = -0.001, rgb_out: float = 0.0, capacity: int = 0) -> "Grid":
        """capacity 0: dense map; > 0: brick-pool map with that many brick slots."""
        return Grid(n, dtype, voxel, (ctypes.c_double * 3)(*origin), occ_out, rgb_out, capacity)


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("d_near", ctypes.c_double), ("d_far", ctypes.c_double), ("n_samples", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("tau", ctypes.c_double)]

    @staticmethod
    def make(width, height, fx, fy, cx, cy, d_near, d_far, n_samples, tau=0.0) -> "Camera":
        return Camera(width, height, fx, fy, cx, cy, d_near, d_far, n_samples, 0, tau)

    @staticmethod
    def paper_sampling(width, height, fx, fy, cx, cy, voxel: float, max_depth: float, tau=0.0) -> "Camera":
        """A camera whose samples lie at depths eps, 2 eps, ... up to max_depth,
        eps = 0.4 voxel (the library's prism_camera_paper_sampling)."""
        c = Camera(width, height, fx, fy, cx, cy, 0.0, 1.0, 2, 0, tau)
        _check(lib().prism_camera_paper_sampling(ctypes.byref(c), voxel, max_depth))
        return c


class Weights(ctypes.Structure):
    _fields_ = [("w_depth", ctypes.c_double), ("w_rgb", ctypes.c_double),
                ("gate_depth", ctypes.c_double), ("gate_rgb", ctypes.c_double)]

    @staticmethod
    def make(b_geo=0.02, b_rgb=0.1, gate_geo=0.45, gate_rgb=0.15) -> "Weights":
        return Weights(1.0 / b_geo ** 2, 1.0 / b_rgb ** 2, gate_geo, gate_rgb)


class MapParams(ctypes.Structure):
    _fields_ = [("trunc", ctypes.c_double), ("lam_update", ctypes.c_double)]


class Pose(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double * 3), ("q", ctypes.c_double * 4)]


class FilterCfg(ctypes.Structure):
    _fields_ = [("grid", Grid), ("cam", Camera), ("dt", ctypes.c_double),
                ("sigma_vel_t", ctypes.c_double), ("sigma_vel_r", ctypes.c_double),
                ("sigma_pose_t", ctypes.c_double), ("sigma_pose_r", ctypes.c_double),
                ("w", Weights), ("ema", ctypes.c_double), ("n_gn", ctypes.c_int32),
                ("objective", ctypes.c_int32), ("map", MapParams), ("normal_disc", ctypes.c_double),
                ("min_inlier_frac", ctypes.c_double), ("modes", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("irls_floor", ctypes.c_double), ("sigma_bias", ctypes.c_double), ("gravity", ctypes.c_double * 3)]


class FilterState(ctypes.Structure):
    _fields_ = [("pose", Pose), ("v", ctypes.c_double * 3), ("w", ctypes.c_double * 3),
                ("P", ctypes.c_double * 144), ("Sbar", ctypes.c_double * 36), ("anchor", Pose),
                ("prior", Pose), ("iter", Pose), ("vel_prior", ctypes.c_double * 6),
                ("Lp", ctypes.c_double * 36), ("D", ctypes.c_double * 36), ("Sv", ctypes.c_double * 36),
                ("S_lap", ctypes.c_double * 36), ("neq", ctypes.c_double * 29), ("u", ctypes.c_double * 6),
                ("step", ctypes.c_int64), ("n_updated", ctypes.c_int64), ("flags", ctypes.c_int32),
                ("has_sbar", ctypes.c_int32), ("n_updated_total", ctypes.c_int64)]


class BiasState(ctypes.Structure):
    _fields_ = [("b", ctypes.c_double * 3), ("P", ctypes.c_double * 225), ("D", ctypes.c_double * 54),
                ("Sv", ctypes.c_double * 81), ("rest_prior", ctypes.c_double * 9)]


class Frame(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("rgb", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class AdamParams(ctypes.Structure):
    """The paper's pose optimiser (App. G): Adam without momentum."""
    _fields_ = [("n_steps", ctypes.c_int32), ("n_pixels", ctypes.c_int32), ("lr_t", ctypes.c_double),
                ("lr_r", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]

    @staticmethod
    def make(n_steps=1000, n_pixels=200, lr_t=0.001, lr_r=0.00036, beta2=0.999, eps=1e-8) -> "AdamParams":
        return AdamParams(n_steps, n_pixels, lr_t, lr_r, beta2, eps)


# ---------------------------------------------------------------------------
# loading
# ---------------------------------------------------------------------------
_lib = None

_SIGS = {
    "prism_last_error": ([], ctypes.c_char_p),
    "prism_version": ([], ctypes.c_char_p),
    "prism_sizeof": ([ctypes.c_char_p], ctypes.c_size_t),
    "prism_map_bytes": (["p", "p"], None),
    "prism_map_init": (["p", "p", ctypes.c_float, ctypes.c_float, ctypes.c_float, "p"], None),
    "prism_map_pool_usage": (["p", "p", "p", "p"], None),
    "prism_map_from_dense": (["p", "p", "p", "p", "p"], None),
    "prism_map_to_dense": (["p", "p", "p", "p", "p"], None),
    "prism_map_refresh": (["p", "p", "p"], None),
    "prism_bricks_to_dense": ([ctypes.c_int32, ctypes.c_int32, "p", "p", "p"], None),
    "prism_dense_to_bricks": ([ctypes.c_int32, ctypes.c_int32, "p", "p", "p"], None),
    "prism_render": (["p", "p", "p", "p", ctypes.c_int32, "p", "p", "p", "p", "p", "p", ctypes.c_double, "p"], None),
    "prism_reduce_workspace_bytes": (["p", ctypes.c_int32, "p"], None),
    "prism_camera_paper_sampling": (["p", ctypes.c_double, ctypes.c_double], None),
    "prism_render_jacobian": (["p", "p", "p", "p", ctypes.c_int32, "p", "p", "p", "p", "p", "p", "p", "p", "p",
                               "p", "p", ctypes.c_size_t, "p"], None),
    "prism_render_jacobian_noalloc_max_bytes": ([], ctypes.c_size_t),
    "prism_render_jacobian_noalloc": (["p", "p", "p", "p", ctypes.c_int32, "p", "p", "p", "p", "p", "p", "p", "p",
                                       "p", "p", "p"], None),
    "prism_track_p2": (["p", "p", "p", "p", "p", "p", "p", "p", "p", "p", "p", "p", "p", "p", "p", "p",
                        ctypes.c_size_t, "p"], None),
    "prism_render_vjp": (["p", "p", "p", "p", ctypes.c_int32, "p", "p", "p", "p", "p", "p", ctypes.c_size_t,
                          "p"], None),
    "prism_map_update": (["p", "p", "p", "p", "p", "p", "p", "p", "p"], None),
    "prism_map_gd_workspace_bytes": (["p", "p", "p"], None),
    "prism_map_gd": (["p", "p", "p", "p", "p", "p", "p", ctypes.c_double, ctypes.c_double, ctypes.c_int32, "p",
                      "p", ctypes.c_size_t, "p"], None),
    "prism_filter_bytes": (["p", "p"], None),
    "prism_filter_create": (["p", "p", "p", "p"], None),
    "prism_filter_destroy": (["p"], None),
    "prism_filter_reset": (["p", "p", "p", "p"], None),
    "prism_filter_reset_bias": (["p", "p", "p", "p"], None),
    "prism_filter_bias_state_ptr": (["p", "p"], None),
    "prism_pose_update": (["p", "p", "p"], None),
    "prism_pose_update_adam": (["p", "p", "p", "p", "p"], None),
    "prism_filter_step_adam": (["p", "p", "p", "p", "p"], None),
    "prism_rollout": (["p", "p", ctypes.c_int32, ctypes.c_int32, "p", "p", "p", "p", "p", "p", "p", "p", "p"], None),
    "prism_filter_step": (["p", ctypes.c_int32, "p", "p"], None),
    "prism_filter_step_graph": (["p", ctypes.c_int32, "p", "p"], None),
    "prism_filter_set_slots": (["p", ctypes.c_int32, "p"], None),
    "prism_filter_submit": (["p", "p", ctypes.c_int32, "p", "p"], None),
    "prism_filter_poll": (["p", "p"], None),
    "prism_filter_step_batch": (["p", ctypes.c_int32, "p", ctypes.c_int32, "p"], None),
    "prism_filter_poll_batch": (["p", ctypes.c_int32, "p"], None),
    "prism_stage_timer_arm": ([ctypes.c_int32], None),
    "prism_stage_timer_read": (["p", "p"], None),
    "prism_filter_state_ptr": (["p", "p"], None),
    "prism_filter_save_bytes": (["p", "p"], None),
    "prism_filter_save": (["p", "p", ctypes.c_size_t, "p"], None),
    "prism_filter_load": (["p", "p", ctypes.c_size_t, "p"], None),
    "prism_pose_retract": (["p", "p", ctypes.c_int32, "p", "p"], None),
    "prism_filter_anchor": (["p", "p", "p", "p", "p", "p"], None),
}


def lib() -> ctypes.CDLL:
    """Load libprism.so (built in-tree by the package's build step)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2212_02988_amd.build` "
                          "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = [ctypes.c_void_p if a == "p" else a for a in args]
        fn.restype = res if res is not None else ctypes.c_int32
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        msg = lib().prism_last_error().decode(errors="replace")
        raise PrismError(f"prism status {status}: {msg}")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str, shape: Optional[Sequence[int]] = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PrismError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise PrismError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise PrismError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise PrismError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _by(s):
    return ctypes.byref(s)


# ---------------------------------------------------------------------------
# map
# ---------------------------------------------------------------------------
def map_bytes(grid: Grid) -> int:
    b = ctypes.c_size_t()
    _check(lib().prism_map_bytes(_by(grid), _by(b)))
    return b.value


class VoxelMap:
    """Device voxel map (opaque brick layout) owned by a torch buffer."""

    def __init__(self, grid: Grid, device="cuda", buffer: Optional[torch.Tensor] = None):
        self.grid = grid
        nbytes = map_bytes(grid)
        if buffer is None:
            # 256-byte alignment: torch's caching allocator returns >= 512-byte aligned blocks
            buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        if buffer.numel() < nbytes or buffer.data_ptr() % 256:
            raise PrismError("map buffer too small or misaligned")
        self.buf = buffer

    @property
    def n(self) -> int:
        return self.grid.n

    def init(self, occ0=-0.001, rgb0=0.0, var0=1e4, stream=None):
        _check(lib().prism_map_init(_by(self.grid), _ptr(self.buf), occ0, rgb0, var0, _stream(stream)))
        return self

    def from_dense(self, mean4: Optional[torch.Tensor], var4: Optional[torch.Tensor], stream=None):
        n = self.n
        if mean4 is not None:
            _dev(mean4, torch.float32, "mean4", (4, n, n, n))
        if var4 is not None:
            _dev(var4, torch.float32, "var4", (4, n, n, n))
        _check(lib().prism_map_from_dense(_by(self.grid), _ptr(self.buf), _ptr(mean4), _ptr(var4), _stream(stream)))
        return self

    def pool_usage(self, stream=None) -> torch.Tensor:
        """Brick-pool maps: int32 [bricks with a slot, dropped brick updates]."""
        out = torch.zeros(2, dtype=torch.int32, device=self.buf.device)
        _check(lib().prism_map_pool_usage(_by(self.grid), _ptr(self.buf), _ptr(out), _stream(stream)))
        return out

    def refresh(self, stream=None):
        """Recompute the brick summary after writing the mean planes directly."""
        _check(lib().prism_map_refresh(_by(self.grid), _ptr(self.buf), _stream(stream)))
        return self

    def to_dense(self, stream=None):
        n = self.n
        mean4 = torch.empty((4, n, n, n), dtype=torch.float32, device=self.buf.device)
        var4 = torch.empty_like(mean4)
        _check(lib().prism_map_to_dense(_by(self.grid), _ptr(self.buf), _ptr(mean4), _ptr(var4), _stream(stream)))
        return mean4, var4

    def mean_planes(self) -> torch.Tensor:
        """FP32 maps only: the four mean planes as a [4, n^3] float view (brick order)."""
        if self.grid.dtype != PRISM_F32:
            raise PrismError("mean_planes needs an FP32 map")
        nv = self.n ** 3
        return self.buf[: 16 * nv].view(torch.float32).view(4, nv)


def bricks_to_dense(n: int, planes: torch.Tensor, stream=None) -> torch.Tensor:
    c = planes.shape[0]
    _dev(planes, torch.float32, "planes", (c, n ** 3))
    out = torch.empty((c, n, n, n), dtype=torch.float32, device=planes.device)
    _check(lib().prism_bricks_to_dense(n, c, _ptr(planes), _ptr(out), _stream(stream)))
    return out


def dense_to_bricks(n: int, dense: torch.Tensor, stream=None) -> torch.Tensor:
    c = dense.shape[0]
    _dev(dense, torch.float32, "dense", (c, n, n, n))
    out = torch.empty((c, n ** 3), dtype=torch.float32, device=dense.device)
    _check(lib().prism_dense_to_bricks(n, c, _ptr(dense), _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# emission, Jacobians, tracking, map update
# ---------------------------------------------------------------------------
def poses_tensor(poses, device="cuda") -> torch.Tensor:
    """[n, 7] float64 (t, q) on the device."""
    p = torch.as_tensor(poses, dtype=torch.float64)
    if p.dim() == 1:
        p = p[None]
    return p.to(device).contiguous()


def workspace_bytes(cam: Camera, n_frames: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().prism_reduce_workspace_bytes(_by(cam), n_frames, _by(b)))
    return b.value


def _workspace(cam, n_frames, device, ws=None):
    nb = workspace_bytes(cam, n_frames)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=device)
    return ws


def render(grid: Grid, vmap: VoxelMap, cam: Camera, poses: torch.Tensor, normals: bool = False,
           hit_k: bool = False, normal_disc: float = 0.1, out: Optional[Dict] = None, stream=None) -> Dict:
    n = poses.shape[0]
    _dev(poses, torch.float64, "poses", (n, 7))
    H, W, dev = cam.height, cam.width, poses.device
    if out is None:
        out = dict(depth=torch.empty((n, H, W), dtype=torch.float32, device=dev),
                   rgb=torch.empty((n, H, W, 3), dtype=torch.float32, device=dev),
                   mask=torch.empty((n, H, W), dtype=torch.uint8, device=dev))
        if hit_k:
            out["hit_k"] = torch.empty((n, H, W), dtype=torch.int32, device=dev)
        if normals:
            out["normals"] = torch.empty((n, H, W, 3), dtype=torch.float32, device=dev)
            out["nmask"] = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    _check(lib().prism_render(_by(grid), _ptr(vmap.buf), _by(cam), _ptr(poses), n, _ptr(out["depth"]),
                              _ptr(out["rgb"]), _ptr(out["mask"]), _ptr(out.get("hit_k")),
                              _ptr(out.get("normals")), _ptr(out.get("nmask")), normal_disc, _stream(stream)))
    return out


def render_jacobian(grid: Grid, vmap: VoxelMap, cam: Camera, poses: torch.Tensor, obs_depth: torch.Tensor,
                    obs_rgb: torch.Tensor, w: Weights, want_render: bool = True, want_J: bool = False,
                    want_resid: bool = False, ws: Optional[torch.Tensor] = None, out: Optional[Dict] = None,
                    stream=None) -> Dict:
    n = poses.shape[0]
    H, W, dev = cam.height, cam.width, poses.device
    _dev(poses, torch.float64, "poses", (n, 7))
    _dev(obs_depth, torch.float32, "obs_depth", (n, H, W))
    _dev(obs_rgb, torch.float32, "obs_rgb", (n, H, W, 3))
    if out is None:
        out = dict(neq=torch.empty((n, NEQ), dtype=torch.float64, device=dev))
        if want_render:
            out.update(depth=torch.empty((n, H, W), dtype=torch.float32, device=dev),
                       rgb=torch.empty((n, H, W, 3), dtype=torch.float32, device=dev),
                       mask=torch.empty((n, H, W), dtype=torch.uint8, device=dev))
        if want_J:
            out["J"] = torch.empty((n, H, W, 4, 6), dtype=torch.float32, device=dev)
        if want_resid:
            out["resid"] = torch.empty((n, H, W, 4), dtype=torch.float32, device=dev)
            out["rowmask"] = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    ws = _workspace(cam, n, dev, ws)
    _check(lib().prism_render_jacobian(_by(grid), _ptr(vmap.buf), _by(cam), _ptr(poses), n, _ptr(obs_depth),
                                       _ptr(obs_rgb), _by(w), _ptr(out.get("depth")), _ptr(out.get("rgb")),
                                       _ptr(out.get("mask")), _ptr(out.get("J")), _ptr(out.get("resid")),
                                       _ptr(out.get("rowmask")), _ptr(out["neq"]), _ptr(ws), ws.numel(),
                                       _stream(stream)))
    return out


def pose_retract(poses: torch.Tensor, delta: torch.Tensor, stream=None) -> torch.Tensor:
    """Poses [n,7] (t, q) perturbed by delta [n,6] = (dt, dtheta): t + dt,
    Exp(dtheta) R (the library's left, world-frame retraction), float64 on
    the device."""
    n = poses.shape[0]
    _dev(poses, torch.float64, "poses", (n, 7))
    _dev(delta, torch.float64, "delta", (n, 6))
    out = torch.empty_like(poses)
    _check(lib().prism_pose_retract(_ptr(poses), _ptr(delta), n, _ptr(out), _stream(stream)))
    return out


def render_jacobian_noalloc(grid: Grid, vmap: VoxelMap, cam: Camera, poses: torch.Tensor, obs_depth: torch.Tensor,
                            obs_rgb: torch.Tensor, w: Weights, out: Dict, stream=None) -> Dict:
    """render_jacobian through the allocation-free entry point: no workspace;
    every output buffer comes from the caller in `out` (neq required; depth,
    rgb, mask, J, resid, rowmask optional)."""
    n = poses.shape[0]
    H, W = cam.height, cam.width
    _dev(poses, torch.float64, "poses", (n, 7))
    _dev(obs_depth, torch.float32, "obs_depth", (n, H, W))
    _dev(obs_rgb, torch.float32, "obs_rgb", (n, H, W, 3))
    _dev(out["neq"], torch.float64, "neq", (n, NEQ))
    _check(lib().prism_render_jacobian_noalloc(_by(grid), _ptr(vmap.buf), _by(cam), _ptr(poses), n, _ptr(obs_depth),
                                               _ptr(obs_rgb), _by(w), _ptr(out.get("depth")), _ptr(out.get("rgb")),
                                               _ptr(out.get("mask")), _ptr(out.get("J")), _ptr(out.get("resid")),
                                               _ptr(out.get("rowmask")), _ptr(out["neq"]), _stream(stream)))
    return out


def render_jacobian_noalloc_max_bytes() -> int:
    return int(lib().prism_render_jacobian_noalloc_max_bytes())


def track_p2(cam: Camera, pose: torch.Tensor, pose_prev: torch.Tensor, obs_depth: torch.Tensor,
             obs_rgb: torch.Tensor, anchor: Dict[str, torch.Tensor], w: Weights, want_J: bool = False,
             want_resid: bool = False, ws: Optional[torch.Tensor] = None, stream=None) -> Dict:
    H, W, dev = cam.height, cam.width, pose.device
    _dev(pose, torch.float64, "pose", (1, 7))
    _dev(pose_prev, torch.float64, "pose_prev", (1, 7))
    _dev(obs_depth, torch.float32, "obs_depth", (H, W))
    _dev(obs_rgb, torch.float32, "obs_rgb", (H, W, 3))
    ad = _dev(anchor["depth"], torch.float32, "anchor depth", (H, W))
    ar = _dev(anchor["rgb"], torch.float32, "anchor rgb", (H, W, 3))
    am = _dev(anchor["mask"], torch.uint8, "anchor mask", (H, W))
    an = _dev(anchor["normals"], torch.float32, "anchor normals", (H, W, 3))
    anm = _dev(anchor["nmask"], torch.uint8, "anchor nmask", (H, W))
    out = dict(neq=torch.empty((1, NEQ), dtype=torch.float64, device=dev))
    if want_J:
        out["J"] = torch.empty((H, W, 4, 6), dtype=torch.float32, device=dev)
    if want_resid:
        out["resid"] = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
        out["rowmask"] = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ws = _workspace(cam, 1, dev, ws)
    _check(lib().prism_track_p2(_by(cam), _ptr(pose), _ptr(pose_prev), _ptr(obs_depth), _ptr(obs_rgb), _ptr(ad),
                                _ptr(ar), _ptr(am), _ptr(an), _ptr(anm), _by(w), _ptr(out.get("J")),
                                _ptr(out.get("resid")), _ptr(out.get("rowmask")), _ptr(out["neq"]), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return out


def render_vjp(grid: Grid, vmap: VoxelMap, cam: Camera, poses: torch.Tensor, hit_k: torch.Tensor,
               g_depth: torch.Tensor, g_rgb: torch.Tensor, grad_mean: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None, stream=None):
    """Adjoint of render: returns (grad_mean [4, n^3] brick order, accumulated; grad_pose [n, 6])."""
    n = poses.shape[0]
    H, W, dev = cam.height, cam.width, poses.device
    nv = grid.n ** 3
    _dev(poses, torch.float64, "poses", (n, 7))
    _dev(hit_k, torch.int32, "hit_k", (n, H, W))
    _dev(g_depth, torch.float32, "g_depth", (n, H, W))
    _dev(g_rgb, torch.float32, "g_rgb", (n, H, W, 3))
    if grad_mean is None:
        grad_mean = torch.zeros((4, nv), dtype=torch.float32, device=dev)
    _dev(grad_mean, torch.float32, "grad_mean", (4, nv))
    grad_pose = torch.empty((n, 6), dtype=torch.float64, device=dev)
    ws = _workspace(cam, n, dev, ws)
    _check(lib().prism_render_vjp(_by(grid), _ptr(vmap.buf), _by(cam), _ptr(poses), n, _ptr(hit_k), _ptr(g_depth),
                                  _ptr(g_rgb), _ptr(grad_mean), _ptr(grad_pose), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return grad_mean, grad_pose


def map_gd_workspace(grid: Grid, cam: Camera, device="cuda") -> torch.Tensor:
    """A zero-filled workspace for map_gd (reusable across calls that do not
    overlap)."""
    b = ctypes.c_size_t()
    _check(lib().prism_map_gd_workspace_bytes(_by(grid), _by(cam), _by(b)))
    return torch.zeros(b.value, dtype=torch.uint8, device=device)


def map_gd(grid: Grid, vmap: VoxelMap, cam: Camera, pose: torch.Tensor, obs_depth: torch.Tensor,
           obs_rgb: torch.Tensor, weights: Weights, lr_occ: float, lr_rgb: float, n_iters: int,
           ws: torch.Tensor, cost: Optional[torch.Tensor] = None, stream=None) -> Optional[torch.Tensor]:
    """Map inference by gradient descent through the renderer, in place on
    vmap (FP32): n_iters steps on the map-filter objective of one frame.
    Returns the objective before each step when `cost` (float64 [n_iters])
    is given."""
    H, W = cam.height, cam.width
    _dev(pose, torch.float64, "pose", (1, 7))
    _dev(obs_depth, torch.float32, "obs_depth", (H, W))
    _dev(obs_rgb, torch.float32, "obs_rgb", (H, W, 3))
    _dev(ws, torch.uint8, "ws")
    if cost is not None:
        _dev(cost, torch.float64, "cost", (n_iters,))
    _check(lib().prism_map_gd(_by(grid), _ptr(vmap.buf), _by(cam), _ptr(pose), _ptr(obs_depth), _ptr(obs_rgb),
                              _by(weights), float(lr_occ), float(lr_rgb), int(n_iters), _ptr(cost), _ptr(ws),
                              ws.numel(), _stream(stream)))
    return cost


def map_update(grid: Grid, vmap: VoxelMap, cam: Camera, pose: torch.Tensor, obs_depth: torch.Tensor,
               obs_rgb: torch.Tensor, trunc: float, lam_update: float = 1.0,
               n_updated: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    H, W, dev = cam.height, cam.width, pose.device
    _dev(pose, torch.float64, "pose", (1, 7))
    _dev(obs_depth, torch.float32, "obs_depth", (H, W))
    _dev(obs_rgb, torch.float32, "obs_rgb", (H, W, 3))
    if n_updated is None:
        n_updated = torch.empty(1, dtype=torch.int64, device=dev)
    p = MapParams(trunc, lam_update)
    _check(lib().prism_map_update(_by(grid), _ptr(vmap.buf), _by(cam), _ptr(pose), _ptr(obs_depth),
                                  _ptr(obs_rgb), _by(p), _ptr(n_updated), _stream(stream)))
    return n_updated


# ---------------------------------------------------------------------------
# filter
# ---------------------------------------------------------------------------
@dataclass
class FilterParams:
    dt: float = 0.1
    sigma_vel_t: float = 0.03
    sigma_vel_r: float = 0.03
    sigma_pose_t: float = 0.05
    sigma_pose_r: float = 0.02
    b_geo: float = 0.02
    b_rgb: float = 0.1
    gate_geo: float = 0.45
    gate_rgb: float = 0.15
    ema: float = 0.8
    n_gn: int = 3
    objective: int = OBJ_P2
    trunc_voxels: float = 4.0
    sigma_update: float = 1.0
    normal_disc: float = 0.1
    min_inlier_frac: float = 0.1
    modes: int = 0             # MODE_* bits: the paper's literal forms, the 15-D state
    irls_floor: float = 0.01   # MODE_IRLS_L1: residual floor as a fraction of each row's scale b
    sigma_bias: float = 0.001  # MODE_ACCEL_BIAS: bias random walk per step (m/s^2)
    gravity: tuple = (0.0, 0.0, -9.81)   # MODE_ACCEL_BIAS: world-frame gravity


def filter_cfg(grid: Grid, cam: Camera, p: FilterParams) -> FilterCfg:
    return FilterCfg(grid, cam, p.dt, p.sigma_vel_t, p.sigma_vel_r, p.sigma_pose_t, p.sigma_pose_r,
                     Weights.make(p.b_geo, p.b_rgb, p.gate_geo, p.gate_rgb), p.ema, p.n_gn, p.objective,
                     MapParams(p.trunc_voxels * grid.voxel, 1.0 / p.sigma_update ** 2), p.normal_disc,
                     p.min_inlier_frac, p.modes, 0, p.irls_floor, p.sigma_bias,
                     (ctypes.c_double * 3)(*[float(v) for v in p.gravity]))


def filter_bytes(cfg: FilterCfg) -> int:
    b = ctypes.c_size_t()
    _check(lib().prism_filter_bytes(_by(cfg), _by(b)))
    return b.value


class Filter:
    """One agent's filter: device state buffer + voxel map, borrowed by a
    library handle."""

    def __init__(self, grid: Grid, cam: Camera, params: FilterParams = FilterParams(), device="cuda",
                 state_buf: Optional[torch.Tensor] = None, vmap: Optional[VoxelMap] = None):
        self.grid, self.cam, self.params = grid, cam, params
        self.cfg = filter_cfg(grid, cam, params)
        nb = filter_bytes(self.cfg)
        self.state_buf = state_buf if state_buf is not None else torch.zeros(nb, dtype=torch.uint8, device=device)
        self.map = vmap if vmap is not None else VoxelMap(grid, device)
        h = ctypes.c_void_p()
        _check(lib().prism_filter_create(_by(self.cfg), _ptr(self.state_buf), _ptr(self.map.buf), _by(h)))
        self.h = h
        sp = ctypes.c_void_p()
        _check(lib().prism_filter_state_ptr(self.h, _by(sp)))
        self._state_ptr = sp.value
        self._state_off = self._state_ptr - self.state_buf.data_ptr()

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.prism_filter_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def reset(self, x0, P0, stream=None):
        """x0 = (t, q, v, w) and P0 12x12; with MODE_ACCEL_BIAS x0 = (t, q, v,
        w, b) and P0 15x15."""
        n = 15 if self.params.modes & MODE_ACCEL_BIAS else 12
        x = (ctypes.c_double * (n + 1))(*[float(v) for v in x0])
        P = (ctypes.c_double * (n * n))(*[float(v) for v in torch.as_tensor(P0, dtype=torch.float64).flatten()])
        fn = lib().prism_filter_reset_bias if n == 15 else lib().prism_filter_reset
        _check(fn(self.h, x, P, _stream(stream)))
        # the source buffer of the upload lives in the handle; no sync needed

    @staticmethod
    def frame(depth: torch.Tensor, rgb: torch.Tensor, u: Optional[torch.Tensor]) -> Frame:
        return Frame(depth.data_ptr(), rgb.data_ptr(), u.data_ptr() if u is not None else None)

    def step(self, depth: torch.Tensor, rgb: torch.Tensor, u: Optional[torch.Tensor], stream=None):
        fr = self.frame(depth, rgb, u)
        arr = (ctypes.c_void_p * 1)(self.h)
        _check(lib().prism_filter_step(arr, 1, _by(fr), _stream(stream)))

    def step_graph(self, depth: torch.Tensor, rgb: torch.Tensor, u: Optional[torch.Tensor], stream):
        """Same as step, replayed from a graph the handle records per input
        buffer set (stream: a non-default torch stream)."""
        fr = self.frame(depth, rgb, u)
        arr = (ctypes.c_void_p * 1)(self.h)
        _check(lib().prism_filter_step_graph(arr, 1, _by(fr), _stream(stream)))

    def set_slots(self, slots):
        """Register serving input slots: a list of (depth [H,W] f32, rgb
        [H,W,3] f32, u [6] f64) device tensors, 16-byte aligned."""
        H, W = self.cam.height, self.cam.width
        for d, c, u in slots:
            _dev(d, torch.float32, "slot depth", (H, W))
            _dev(c, torch.float32, "slot rgb", (H, W, 3))
            _dev(u, torch.float64, "slot u", (6,))
        arr = (Frame * len(slots))(*[Filter.frame(d, c, u) for d, c, u in slots])
        _check(lib().prism_filter_set_slots(self.h, len(slots), arr))
        self._slots = list(slots)          # keep the buffers alive

    def submit(self, depth, rgb, u, stream, flags: int = 0) -> Optional[int]:
        """Queue one step (see prism_filter_submit); returns its submission
        number, or None when every slot is in flight.  depth/rgb/u are device
        tensors, or pinned host tensors with flags |= SUBMIT_FROM_HOST."""
        fr = self.frame(depth, rgb, u)
        seq = ctypes.c_int64()
        st = lib().prism_filter_submit(self.h, _by(fr), flags, _stream(stream), _by(seq))
        if st == PRISM_BUSY:
            return None
        _check(st)
        return seq.value

    def poll(self) -> int:
        """Number of submitted steps that have completed."""
        c = ctypes.c_int64()
        _check(lib().prism_filter_poll(self.h, _by(c)))
        return c.value

    def pose_update(self, depth, rgb, u, stream=None):
        fr = self.frame(depth, rgb, u)
        _check(lib().prism_pose_update(self.h, _by(fr), _stream(stream)))

    def _adam_args(self, params: AdamParams, pixels: torch.Tensor):
        _dev(pixels, torch.int32, "pixels", (params.n_steps, params.n_pixels))
        return _by(params), _ptr(pixels)

    def pose_update_adam(self, depth, rgb, u, params: AdamParams, pixels: torch.Tensor, stream=None):
        """State filter with the paper's optimiser; pixels: int32 [n_steps, n_pixels]."""
        fr = self.frame(depth, rgb, u)
        _check(lib().prism_pose_update_adam(self.h, _by(fr), *self._adam_args(params, pixels), _stream(stream)))

    def step_adam(self, depth, rgb, u, params: AdamParams, pixels: torch.Tensor, stream=None):
        fr = self.frame(depth, rgb, u)
        _check(lib().prism_filter_step_adam(self.h, _by(fr), *self._adam_args(params, pixels), _stream(stream)))

    def rollout(self, u: torch.Tensor, noise: Optional[torch.Tensor] = None, moments: bool = True,
                frames: bool = False, stream=None) -> Dict[str, torch.Tensor]:
        """Predictive rollout from the current belief: u float64 [k, 6]
        controls; noise float64 [n_samples, k+1, n] standard normals (n = 12,
        15 with MODE_ACCEL_BIAS).  Returns poses [n_samples, k, 7], mean
        [k, n+1] / cov [k, n, n] (if moments), depth/rgb/mask [n_samples*k,
        ...] (if frames), flags [1]."""
        k = u.shape[0]
        n = 15 if self.params.modes & MODE_ACCEL_BIAS else 12
        _dev(u, torch.float64, "u", (k, 6))
        dev = u.device
        ns = 0 if noise is None else noise.shape[0]
        if noise is not None:
            _dev(noise, torch.float64, "noise", (ns, k + 1, n))
        out = dict(flags=torch.zeros(1, dtype=torch.int32, device=dev))
        out["poses"] = torch.empty((max(ns, 1), k, 7), dtype=torch.float64, device=dev)
        if moments:
            out["mean"] = torch.empty((k, n + 1), dtype=torch.float64, device=dev)
            out["cov"] = torch.empty((k, n, n), dtype=torch.float64, device=dev)
        if frames:
            H, W = self.cam.height, self.cam.width
            out["depth"] = torch.empty((ns * k, H, W), dtype=torch.float32, device=dev)
            out["rgb"] = torch.empty((ns * k, H, W, 3), dtype=torch.float32, device=dev)
            out["mask"] = torch.empty((ns * k, H, W), dtype=torch.uint8, device=dev)
        _check(lib().prism_rollout(self.h, _ptr(u), k, ns, _ptr(noise), _ptr(out["poses"]), _ptr(out.get("mean")),
                                   _ptr(out.get("cov")), _ptr(out.get("depth")), _ptr(out.get("rgb")),
                                   _ptr(out.get("mask")), _ptr(out["flags"]), _stream(stream)))
        if ns == 0:
            out["poses"] = out["poses"][:0]
        return out

    def save_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().prism_filter_save_bytes(_by(self.cfg), _by(b)))
        return b.value

    def save(self, dst: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Checkpoint of the belief (map and state) into dst, a uint8 tensor
        (device, or pinned host) of save_bytes(); allocated on the device if
        None.  Asynchronous on the stream."""
        nb = self.save_bytes()
        if dst is None:
            dst = torch.empty(nb, dtype=torch.uint8, device=self.state_buf.device)
        if dst.dtype != torch.uint8 or dst.numel() < nb or not dst.is_contiguous():
            raise PrismError("checkpoint buffer must be a contiguous uint8 tensor of save_bytes()")
        _check(lib().prism_filter_save(self.h, _ptr(dst), dst.numel(), _stream(stream)))
        return dst

    def load(self, src: torch.Tensor, stream=None):
        """Restore a checkpoint made by save() of a filter with the same grid
        and camera (waits for the stream to read its header)."""
        if src.dtype != torch.uint8 or not src.is_contiguous():
            raise PrismError("checkpoint must be a contiguous uint8 tensor")
        _check(lib().prism_filter_load(self.h, _ptr(src), src.numel(), _stream(stream)))

    def state(self) -> FilterState:
        """Synchronous read-back of the device state."""
        nb = ctypes.sizeof(FilterState)
        raw = self.state_buf[self._state_off:self._state_off + nb].cpu().numpy().tobytes()
        return FilterState.from_buffer_copy(raw)

    def bias_state(self) -> BiasState:
        """Synchronous read-back of the 15-D state's bias part (MODE_ACCEL_BIAS)."""
        p = ctypes.c_void_p()
        _check(lib().prism_filter_bias_state_ptr(self.h, _by(p)))
        off = p.value - self.state_buf.data_ptr()
        nb = ctypes.sizeof(BiasState)
        raw = self.state_buf[off:off + nb].cpu().numpy().tobytes()
        return BiasState.from_buffer_copy(raw)

    def anchor(self) -> Dict[str, torch.Tensor]:
        ptrs = [ctypes.c_void_p() for _ in range(5)]
        _check(lib().prism_filter_anchor(self.h, *[_by(p) for p in ptrs]))
        H, W = self.cam.height, self.cam.width
        base = self.state_buf.data_ptr()

        def view(p, nbytes, dtype, shape):
            off = p.value - base
            return self.state_buf[off:off + nbytes].view(dtype).view(*shape)
        return dict(depth=view(ptrs[0], 4 * H * W, torch.float32, (H, W)),
                    rgb=view(ptrs[1], 12 * H * W, torch.float32, (H, W, 3)),
                    mask=view(ptrs[2], H * W, torch.uint8, (H, W)),
                    normals=view(ptrs[3], 12 * H * W, torch.float32, (H, W, 3)),
                    nmask=view(ptrs[4], H * W, torch.uint8, (H, W)))


def filter_step_graph(filters: Sequence[Filter], depths, rgbs, us, stream):
    """filter_step with each steady-state step replayed from a per-handle graph."""
    n = len(filters)
    frames = (Frame * n)(*[Filter.frame(d, r, u) for d, r, u in zip(depths, rgbs, us)])
    hs = (ctypes.c_void_p * n)(*[f.h for f in filters])
    _check(lib().prism_filter_step_graph(hs, n, frames, _stream(stream)))


def filter_step_batch(filters: Sequence[Filter], frames, stream, flags: int = 0) -> bool:
    """Continuous batching: one step for each filter (frames[i] = (depth, rgb,
    u) for filters[i]) with one launch per stage for the whole batch (see
    prism_filter_step_batch).  False, with nothing queued, when some filter
    has every input slot in flight."""
    n = len(filters)
    fr = (Frame * n)(*[Filter.frame(d, c, u) for d, c, u in frames])
    hs = (ctypes.c_void_p * n)(*[f.h for f in filters])
    st = lib().prism_filter_step_batch(hs, n, fr, flags, _stream(stream))
    if st == PRISM_BUSY:
        return False
    _check(st)
    return True


def filters_poll(filters: Sequence[Filter]) -> list:
    """Completed-step counts of several filters with one call."""
    n = len(filters)
    hs = (ctypes.c_void_p * n)(*[f.h for f in filters])
    out = (ctypes.c_int64 * n)()
    _check(lib().prism_filter_poll_batch(hs, n, out))
    return list(out)


STAGES = ("staging", "predict", "track", "gn", "laplace", "cull", "map_update", "render", "normals", "first_frame")


def stage_timer_arm(cap: int):
    """Time every batched stage launch (up to cap per stage) from now on."""
    _check(lib().prism_stage_timer_arm(cap))


def stage_timer_read() -> Dict[str, tuple]:
    """{stage: (summed launch ms, launches)}; disarms the timer."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int64 * len(STAGES))()
    _check(lib().prism_stage_timer_read(ms, n))
    return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}


def filter_step(filters: Sequence[Filter], depths, rgbs, us, stream=None):
    """One batched step over several filters (one frame each)."""
    n = len(filters)
    frames = (Frame * n)(*[Filter.frame(d, r, u) for d, r, u in zip(depths, rgbs, us)])
    hs = (ctypes.c_void_p * n)(*[f.h for f in filters])
    _check(lib().prism_filter_step(hs, n, frames, _stream(stream)))
