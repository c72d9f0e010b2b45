"""FP64 CPU oracle of the PRISM filter hot path -- test infrastructure only.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It shares no code with the GPU library: the per-ray and
per-voxel loops live in ``prism_oracle.c`` (plain C, double precision, built
with gcc), the small linear-Gaussian algebra lives here in NumPy float64.

Paper: Mirchev et al., PRISM (CoRL 2022, arXiv 2212.02988).

=====================  ===================================================
function               passage it follows
=====================  ===================================================
render                 App. B, ray-marching emission, first crossing of
                       tau and the depth-interpolation equation; colour
                       "analogously to depth"
normals                App. E.3 (normal of the rendered depth image),
                       App. G (discontinuous depth ignored)
render_jacobian        Sec. 4.3.2 MAP objective with the render-through
                       likelihood; App. G weights and gating
track_p2               App. E.3 prediction-to-observation objective
                       (point-to-plane and photometric terms)
map_update             App. D Gaussian product in precision form, App. G
                       update region, truncation and update scale
render_vjp             adjoint of App. B's emission (App. B notes the
                       emission is differentiable)
map_gd                 Sec. 4.3.1 alternative: the map-filter objective
                       (emission likelihood times previous map belief)
                       minimised by gradient descent through the renderer,
                       as compared against the closed form in Sec. 5.3
predict / split        App. E.1 linearised transition, E.2 closed-form
                       propagation and split into pose prior + velocity
                       conditional
adam_pose              Sec. 4.3.2 MAP pose by the paper's optimiser (App. G:
                       Adam without momentum, per-component step sizes,
                       sampled pixels)
gn_solve / laplace     Sec. 4.3.2 MAP pose + Laplace approximation;
                       Sec. 5.1 / App. G.2 Hessian as squared Jacobian, EMA 0.8
combine                Sec. 4.3.2 product of pose posterior and velocity
                       conditional
rollout                App. J predictive rollout: generative transition
                       (App. B) sampled from the belief, closed-form
                       predicted moments (App. E.2), renders (App. B)
filter_step            Sec. 4.3 map filter then state filter ordering
=====================  ===================================================

Readings where the paper is silent or ambiguous are stated next to the code
they affect.

Parity status: every function above is pinned by a CPU test against a
closed form, a brute force or finite differences, except ``filter_step`` as a
whole, whose parity beyond its components is unpinned.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prism_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (double precision, no FMA
    contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pad_", ctypes.c_int32), ("voxel", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("occ_out", ctypes.c_double),
                ("rgb_out", ctypes.c_double)]


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("d_near", ctypes.c_double), ("d_far", ctypes.c_double),
                ("n_samples", ctypes.c_int32), ("pad_", ctypes.c_int32), ("tau", ctypes.c_double)]


class _Weights(ctypes.Structure):
    _fields_ = [("w_depth", ctypes.c_double), ("w_rgb", ctypes.c_double),
                ("gate_depth", ctypes.c_double), ("gate_rgb", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_render.argtypes = [P, P, P, P, ctypes.c_int, P, P, P, P]
        lib.orc_normals.argtypes = [P, P, P, ctypes.c_double, P, P]
        lib.orc_render_jacobian.argtypes = [P, P, P, P, ctypes.c_int, P, P, P, P, P, P, P, P, P, P]
        lib.orc_track_p2.argtypes = [P, P, P, ctypes.c_int, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_map_update.argtypes = [P, P, P, P, P, ctypes.c_int, P, P, ctypes.c_double,
                                       ctypes.c_double, P]
        lib.orc_map_update.restype = ctypes.c_int64
        lib.orc_render_vjp.argtypes = [P, P, P, P, ctypes.c_int, P, P, P, P]
        lib.orc_pose_to_rot.argtypes = [P, P]
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    n: int
    voxel: float
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    occ_out: float = -0.001      # App. G: first map belief has occupancy -0.001
    rgb_out: float = 0.0         # ... and colour 0

    def c(self) -> _Grid:
        return _Grid(self.n, 0, self.voxel, (ctypes.c_double * 3)(*self.origin), self.occ_out,
                     self.rgb_out)


@dataclass
class Cam:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    d_near: float
    d_far: float
    n_samples: int
    tau: float = 0.0             # App. G: hit threshold 0

    def c(self) -> _Cam:
        return _Cam(self.width, self.height, self.fx, self.fy, self.cx, self.cy, self.d_near,
                    self.d_far, self.n_samples, 0, self.tau)


@dataclass
class Params:
    """Filter hyper-parameters (App. G defaults where the paper gives them)."""
    dt: float = 0.1
    sigma_vel_t: float = 0.03    # App. G transition scales, per step
    sigma_vel_r: float = 0.03
    sigma_pose_t: float = 0.05
    sigma_pose_r: float = 0.02
    b_geo: float = 0.02          # App. G Laplace scales (EuRoC / TUM values)
    b_rgb: float = 0.1
    gate_geo: float = 0.45       # App. G gating
    gate_rgb: float = 0.15
    ema: float = 0.8             # App. G Laplace EMA coefficient
    n_gn: int = 3
    trunc_voxels: float = 4.0    # App. G truncation (Blackbird value)
    sigma_update: float = 1.0    # App. G update scale
    normal_disc: float = 0.1     # depth discontinuity for anchor normals (m)
    objective: str = "p2"        # "p2" surrogate (paper) or "p1" render-through
    # the paper's literal forms, off by default (each default is a reading)
    transition_dt2: bool = False  # App. E.1 as printed: v' = v + u dt^2 (default v + u dt)
    laplace_factor: float = 2.0   # Laplace covariance (factor H_o + Lp)^-1; Sec. 5.1 prints 2, 1 is the
                                  # covariance of a Gaussian likelihood with precision w
    irls: bool = False            # Gauss-Newton iterations minimise the L1 data terms of App. E.3 by
                                  # iteratively reweighted least squares
    irls_floor: float = 0.01      # IRLS residual floor, as a fraction of each row's Laplace scale b
    # 15-D state: pose, velocities and an accelerometer bias (a reading added for
    # trajectories simulated with a biased IMU; the paper's state is 12-D)
    accel_bias: bool = False      # the linear control is the body-frame specific force f, the
                                  # acceleration R (f - b) + g
    sigma_bias: float = 0.001     # per-step bias random walk (m/s^2)
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)

    def weights(self) -> _Weights:
        return _Weights(1.0 / self.b_geo ** 2, 1.0 / self.b_rgb ** 2, self.gate_geo, self.gate_rgb)


def grid_from_scene(scene) -> Grid:
    return Grid(scene.n, scene.voxel, tuple(float(v) for v in scene.origin))


def paper_sample_camera(width: int, height: int, fx: float, fy: float, cx: float, cy: float, voxel: float,
                        max_depth: float, tau: float = 0.0) -> Cam:
    """Camera whose ray samples are the paper's: depth offsets eps, 2 eps,
    3 eps, ... (App. B) with eps = 0.4 voxel (App. G rendering), up to the
    maximum camera depth (App. G: 7, 8 or 20 m): K = floor(max_depth / eps)
    samples from eps to K eps."""
    eps = 0.4 * voxel
    K = int(math.floor(max_depth / eps))
    return Cam(width, height, fx, fy, cx, cy, eps, K * eps, K, tau)


def cam_from(c) -> Cam:
    return Cam(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.d_near, c.d_far, c.n_samples, c.tau)


# ---------------------------------------------------------------------------
# per-ray / per-voxel loops (C)
# ---------------------------------------------------------------------------
def render(grid: Grid, mean: np.ndarray, cam: Cam, pose: np.ndarray, decide32: bool = True,
           normals: bool = False, normal_disc: float = 0.1) -> Dict[str, np.ndarray]:
    """App. B emission for one frame: depth, rgb, mask, hit sample index;
    optionally the anchor normals."""
    lib = _load()
    H, W = cam.height, cam.width
    mean = _f64(mean)
    pose = _f64(pose)
    out = dict(depth=np.zeros((H, W)), rgb=np.zeros((H, W, 3)), mask=np.zeros((H, W), np.uint8),
               hit_k=np.zeros((H, W), np.int32))
    g, c = grid.c(), cam.c()
    lib.orc_render(ctypes.byref(g), _p(mean), ctypes.byref(c), _p(pose), int(decide32),
                   _p(out["depth"]), _p(out["rgb"]), _p(out["mask"]), _p(out["hit_k"]))
    if normals:
        nrm, nmask = normals_of(cam, out["depth"], out["mask"], normal_disc)
        out["normals"], out["nmask"] = nrm, nmask
    return out


def normals_of(cam: Cam, depth: np.ndarray, mask: np.ndarray, disc: float = 0.1):
    lib = _load()
    H, W = cam.height, cam.width
    nrm = np.zeros((H, W, 3))
    nmask = np.zeros((H, W), np.uint8)
    c = cam.c()
    lib.orc_normals(ctypes.byref(c), _p(_f64(depth)), _p(np.ascontiguousarray(mask, np.uint8)),
                    disc, _p(nrm), _p(nmask))
    return nrm, nmask


def _neq_out():
    return np.zeros(29)


def render_jacobian(grid: Grid, mean, cam: Cam, pose, obs_depth, obs_rgb, params: Params,
                    decide32: bool = True, want_J: bool = False) -> Dict[str, np.ndarray]:
    """P1: render, per-ray 4x6 pose Jacobian, gated weighted normal equations."""
    lib = _load()
    H, W = cam.height, cam.width
    out = dict(depth=np.zeros((H, W)), rgb=np.zeros((H, W, 3)), mask=np.zeros((H, W), np.uint8),
               neq=_neq_out(), resid=np.zeros((H, W, 4)), rowmask=np.zeros((H, W), np.uint8))
    if want_J:
        out["J"] = np.zeros((H, W, 4, 6))
    g, c, w = grid.c(), cam.c(), params.weights()
    lib.orc_render_jacobian(ctypes.byref(g), _p(_f64(mean)), ctypes.byref(c), _p(_f64(pose)),
                            int(decide32), _p(_f64(obs_depth)), _p(_f64(obs_rgb)), ctypes.byref(w),
                            _p(out["depth"]), _p(out["rgb"]), _p(out["mask"]), _p(out.get("J")),
                            _p(out["resid"]), _p(out["rowmask"]), _p(out["neq"]))
    return out


def track_p2(cam: Cam, pose, pose_prev, obs_depth, obs_rgb, anchor: Dict[str, np.ndarray],
             params: Params, decide32: bool = True, want_J: bool = False) -> Dict[str, np.ndarray]:
    """P2: prediction-to-observation residuals against the previous render."""
    lib = _load()
    H, W = cam.height, cam.width
    out = dict(neq=_neq_out(), resid=np.zeros((H, W, 4)), rowmask=np.zeros((H, W), np.uint8))
    if want_J:
        out["J"] = np.zeros((H, W, 4, 6))
    c, w = cam.c(), params.weights()
    lib.orc_track_p2(ctypes.byref(c), _p(_f64(pose)), _p(_f64(pose_prev)), int(decide32),
                     _p(_f64(obs_depth)), _p(_f64(obs_rgb)), _p(_f64(anchor["depth"])),
                     _p(_f64(anchor["rgb"])), _p(np.ascontiguousarray(anchor["mask"], np.uint8)),
                     _p(_f64(anchor["normals"])), _p(np.ascontiguousarray(anchor["nmask"], np.uint8)),
                     ctypes.byref(w), _p(out.get("J")), _p(out["resid"]), _p(out["rowmask"]),
                     _p(out["neq"]))
    return out


def map_update(grid: Grid, mean: np.ndarray, var: np.ndarray, cam: Cam, pose, obs_depth, obs_rgb,
               params: Params, decide32: bool = True, want_mask: bool = False):
    """App. D closed-form update, in place on (mean, var).  Returns the count
    of updated voxels (and the per-voxel flag if asked)."""
    lib = _load()
    assert mean.dtype == np.float64 and mean.flags.c_contiguous
    assert var.dtype == np.float64 and var.flags.c_contiguous
    upd = np.zeros(mean.shape[1:], np.uint8) if want_mask else None
    g, c = grid.c(), cam.c()
    trunc = params.trunc_voxels * grid.voxel
    n = lib.orc_map_update(ctypes.byref(g), _p(mean), _p(var), ctypes.byref(c), _p(_f64(pose)),
                           int(decide32), _p(_f64(obs_depth)), _p(_f64(obs_rgb)), trunc,
                           1.0 / params.sigma_update ** 2, _p(upd))
    return (int(n), upd) if want_mask else int(n)


def render_vjp(grid: Grid, mean, cam: Cam, pose, g_depth, g_rgb, decide32: bool = True):
    """Adjoint of render: (dL/dmean [4][N][N][N], dL/ddelta [6])."""
    lib = _load()
    mean = _f64(mean)
    gm = np.zeros_like(mean)
    gp = np.zeros(6)
    g, c = grid.c(), cam.c()
    lib.orc_render_vjp(ctypes.byref(g), _p(mean), ctypes.byref(c), _p(_f64(pose)), int(decide32),
                       _p(_f64(g_depth)), _p(_f64(g_rgb)), _p(gm), _p(gp))
    return gm, gp


def map_gd_objective(grid: Grid, mean, mean0, var0, cam: Cam, pose, obs_depth, obs_rgb,
                     params: Params, decide32: bool = True):
    """Negative log of the map-filter target at the nominal pose (Sec. 4.3.1:
    emission likelihood of the frame times the previous map belief), up to
    constants:

        E(mu) = sum over kept rows  w r(mu)^2  +  1/2 sum (mu - mu0)^2 / var0

    The rows, weights and gates are those of the render-through objective
    (Sec. 4.3.2, App. G): r = rendered - observed per valid ray with valid
    observed depth.  Returns (E, dE/dmu) with the gradient through the
    renderer's adjoint (first crossing held fixed)."""
    rj = render_jacobian(grid, mean, cam, pose, obs_depth, obs_rgb, params, decide32)
    r, rm = rj["resid"], rj["rowmask"]
    g_depth = np.where(rm & 1, 2.0 / params.b_geo ** 2 * r[..., 0], 0.0)
    g_rgb = np.where((rm & 2)[..., None] != 0, 2.0 / params.b_rgb ** 2 * r[..., 1:], 0.0)
    g_data, _ = render_vjp(grid, mean, cam, pose, g_depth, g_rgb, decide32)
    lam0 = 1.0 / var0
    diff = mean - mean0
    E = rj["neq"][27] + 0.5 * float(np.sum(lam0 * diff * diff))
    return E, g_data + lam0 * diff


def map_gd(grid: Grid, mean0: np.ndarray, var0: np.ndarray, cam: Cam, pose, obs_depth, obs_rgb,
           params: Params, lr_occ: float, lr_rgb: float, n_iters: int, decide32: bool = True,
           store32: bool = True):
    """Map inference by plain gradient descent on map_gd_objective, starting
    from the previous belief's means: mu <- mu - lr * dE/dmu, one step size
    for occupancy and one for colour.  MAP descent estimates no variance: the
    variances stay those of the previous belief.  With store32 the means are
    rounded to single precision after every step, the storage precision of
    an FP32 map.  Returns (means, [E before each step])."""
    mean = _f64(mean0).copy()
    mean0 = _f64(mean0)
    var0 = _f64(var0)
    lr = np.array([lr_occ, lr_rgb, lr_rgb, lr_rgb]).reshape(4, 1, 1, 1)
    costs = []
    for _ in range(n_iters):
        E, g = map_gd_objective(grid, mean, mean0, var0, cam, pose, obs_depth, obs_rgb, params, decide32)
        costs.append(E)
        mean = mean - lr * g
        if store32:
            mean = mean.astype(np.float32).astype(np.float64)
    return mean, costs


# ---------------------------------------------------------------------------
# rotations (NumPy float64)
# ---------------------------------------------------------------------------
def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def so3_exp(phi) -> np.ndarray:
    """Rodrigues' formula."""
    phi = np.asarray(phi, float)
    th = np.linalg.norm(phi)
    K = skew(phi)
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def so3_log(R) -> np.ndarray:
    c = (np.trace(R) - 1.0) / 2.0
    c = min(1.0, max(-1.0, c))
    th = math.acos(c)
    w = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-8:
        return 0.5 * w
    if math.pi - th < 1e-6:
        # near pi: axis from the symmetric part
        A = (R + np.eye(3)) / 2.0
        ax = A[:, int(np.argmax(np.diag(A)))]
        ax = ax / np.linalg.norm(ax)
        return th * ax
    return th / (2.0 * math.sin(th)) * w


def so3_left_jacobian(phi) -> np.ndarray:
    """J_l(phi) with Exp(phi + d) ~= Exp(J_l(phi) d) Exp(phi)."""
    phi = np.asarray(phi, float)
    th = np.linalg.norm(phi)
    K = skew(phi)
    if th < 1e-6:
        return np.eye(3) + 0.5 * K + K @ K / 6.0
    return (np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K)


def quat_to_rot(q) -> np.ndarray:
    w, x, y, z = np.asarray(q, float) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rot_to_quat(R) -> np.ndarray:
    """Rotation matrix to a unit quaternion with w >= 0 (branch on the largest
    diagonal term for stability)."""
    t = np.trace(R)
    if t > 0:
        s = 2.0 * math.sqrt(t + 1.0)
        q = np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s])
    else:
        i = int(np.argmax(np.diag(R)))
        j, k = (i + 1) % 3, (i + 2) % 3
        s = 2.0 * math.sqrt(1.0 + R[i, i] - R[j, j] - R[k, k])
        q = np.zeros(4)
        q[0] = (R[k, j] - R[j, k]) / s
        q[1 + i] = 0.25 * s
        q[1 + j] = (R[j, i] + R[i, j]) / s
        q[1 + k] = (R[k, i] + R[i, k]) / s
    if q[0] < 0:
        q = -q
    return q / np.linalg.norm(q)


def retract(pose: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """Pose perturbation: t <- t + dt (world), R <- Exp(dtheta) R (left, world)."""
    t = pose[:3] + delta[:3]
    R = so3_exp(delta[3:]) @ quat_to_rot(pose[3:])
    return np.concatenate([t, rot_to_quat(R)])


def pose_error(pose: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Tangent of `pose` relative to `ref`: (t - t_ref, Log(R R_ref^T))."""
    return np.concatenate([pose[:3] - ref[:3],
                           so3_log(quat_to_rot(pose[3:]) @ quat_to_rot(ref[3:]).T)])


# ---------------------------------------------------------------------------
# linear-Gaussian state filter (App. E)
# ---------------------------------------------------------------------------
def neq_unpack(neq: np.ndarray) -> Tuple[np.ndarray, np.ndarray, float, float]:
    """29-vector -> (H 6x6 symmetric, g 6, cost, count)."""
    H = np.zeros((6, 6))
    q = 0
    for a in range(6):
        for b in range(a, 6):
            H[a, b] = H[b, a] = neq[q]
            q += 1
    return H, np.array(neq[21:27]), float(neq[27]), float(neq[28])


def transition_mean(x: Dict[str, np.ndarray], u: np.ndarray, dt: float, dt2: bool = False) -> Dict[str, np.ndarray]:
    """Euler integration (App. B / E.1): velocity first, then the pose with the
    *new* velocity.  Reading: v' = v + u dt (the printed (dt)^2 is read as a
    typo for an acceleration control); dt2 selects the printed form
    v' = v + u dt^2."""
    du = dt * dt if dt2 else dt
    v = x["v"] + u[:3] * du
    w = x["w"] + u[3:] * du
    t = x["t"] + v * dt
    R = so3_exp(w * dt) @ quat_to_rot(x["q"])
    return dict(t=t, q=rot_to_quat(R), v=v, w=w)


def transition_mean_bias(x: Dict[str, np.ndarray], u: np.ndarray, dt: float, g, dt2: bool = False):
    """The transition with an accelerometer bias b in the state: the linear
    control is the body-frame specific force f (the accelerometer's mean over
    the interval), the acceleration a = R (f - b) + g with the state's own
    rotation R; then as transition_mean (velocities first, the pose with the
    new velocities); b is carried over (a random walk)."""
    R = quat_to_rot(x["q"])
    a = R @ (u[:3] - x["b"]) + np.asarray(g, float)
    xn = transition_mean(x, np.concatenate([a, u[3:]]), dt, dt2)
    xn["b"] = np.array(x["b"], float)
    return xn


def transition_jacobians_bias(x: Dict[str, np.ndarray], x_new: Dict[str, np.ndarray], u: np.ndarray, dt: float,
                              dt2: bool = False):
    """First-order error-state transition of the 15-D state (tangent order
    dt, dtheta, dv, dw, db): the 12-D blocks of transition_jacobians plus the
    acceleration's dependence on the rotation and the bias at the start of the
    step, da = -[R (f - b)]x dtheta - R db (left perturbation R <- Exp(dtheta) R),
    entering v' with the control factor du and t' through v' dt; the bias
    noise n_b enters b' directly."""
    du = dt * dt if dt2 else dt
    M12, G12 = transition_jacobians(x_new, dt)
    R = quat_to_rot(x["q"])
    Ra = R @ (u[:3] - x["b"])
    M = np.zeros((15, 15))
    M[:12, :12] = M12
    dv_dth = -du * skew(Ra)
    dv_db = -du * R
    M[6:9, 3:6] += dv_dth
    M[6:9, 12:15] += dv_db
    M[0:3, 3:6] += dt * dv_dth
    M[0:3, 12:15] += dt * dv_db
    M[12:15, 12:15] = np.eye(3)
    G = np.zeros((15, 15))
    G[:12, :12] = G12
    G[12:15, 12:15] = np.eye(3)
    return M, G


def transition_jacobians(x_new: Dict[str, np.ndarray], dt: float):
    """First-order error-state transition (App. E.1 linearisation) for the
    tangent (dt, dtheta, dv, dw): returns M (12x12, old error -> new error)
    and G (12x12, noise (n_t, n_theta, n_v, n_w) -> new error)."""
    I = np.eye(3)
    phi = x_new["w"] * dt
    E = so3_exp(phi)
    Jl = so3_left_jacobian(phi)
    M = np.zeros((12, 12))
    M[0:3, 0:3] = I
    M[0:3, 6:9] = dt * I
    M[3:6, 3:6] = E
    M[3:6, 9:12] = dt * Jl
    M[6:9, 6:9] = I
    M[9:12, 9:12] = I
    G = np.zeros((12, 12))
    G[0:3, 0:3] = I
    G[0:3, 6:9] = dt * I
    G[3:6, 3:6] = I
    G[3:6, 9:12] = dt * Jl
    G[6:9, 6:9] = I
    G[9:12, 9:12] = I
    return M, G


def predict(x: Dict[str, np.ndarray], P: np.ndarray, u: np.ndarray, p: Params):
    """Closed-form propagation of the Gaussian state belief through the
    linearised transition (App. E.2): returns the prior mean and covariance
    (12-D, or 15-D with the accelerometer bias)."""
    q = [p.sigma_pose_t ** 2] * 3 + [p.sigma_pose_r ** 2] * 3 + [p.sigma_vel_t ** 2] * 3 + [p.sigma_vel_r ** 2] * 3
    if p.accel_bias:
        xn = transition_mean_bias(x, u, p.dt, p.gravity, p.transition_dt2)
        M, G = transition_jacobians_bias(x, xn, u, p.dt, p.transition_dt2)
        q = q + [p.sigma_bias ** 2] * 3
    else:
        xn = transition_mean(x, u, p.dt, p.transition_dt2)
        M, G = transition_jacobians(xn, p.dt)
    Qd = np.diag(q)
    Pn = M @ P @ M.T + G @ Qd @ G.T
    return xn, 0.5 * (Pn + Pn.T)


def split(P: np.ndarray):
    """Split a joint Gaussian over (pose, velocity) into the pose marginal and
    the linear-Gaussian velocity conditional N(v; mu_v + D (pose - mu_p), S)."""
    Spp = P[:6, :6]
    Svp = P[6:, :6]
    Svv = P[6:, 6:]
    D = np.linalg.solve(Spp, Svp.T).T          # Svp Spp^-1 (Spp symmetric)
    S = Svv - D @ Svp.T
    return Spp, D, 0.5 * (S + S.T)


def gn_solve(neq: np.ndarray, Lp: np.ndarray, e_p: np.ndarray) -> np.ndarray:
    """One Gauss-Newton step on  sum w r^2 + 1/2 e^T Lp e :
    (2 H + Lp) delta = -(2 g + Lp e)."""
    H, g, _, _ = neq_unpack(neq)
    A = 2.0 * H + Lp
    b = -(2.0 * g + Lp @ e_p)
    L = np.linalg.cholesky(A)
    return np.linalg.solve(L.T, np.linalg.solve(L, b))


def irls_weight(r, b: float, floor: float):
    """IRLS weight of an L1 row |r|/b (App. E.3 objective) at the current
    residual r0: |r| <= r^2 / (2|r0|) + |r0|/2 with equality at r = r0, so
    the row enters the squared objective sum w r^2 with w = 1 / (2 b |r0|);
    |r0| is held at least floor * b."""
    return 1.0 / (2.0 * b * np.maximum(np.abs(r), floor * b))


def neq_from_rows(J: np.ndarray, r: np.ndarray, rowmask: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Normal equations (the 29-vector: upper triangle of H = sum w J^T J,
    g = sum w J^T r, cost sum w r^2, contributing pixels) of per-pixel rows
    J [P][4][6], r [P][4] with row weights w [P][4]; rowmask bit 1 keeps a
    pixel's depth row, bit 2 its three colour rows."""
    J = J.reshape(-1, 4, 6)
    r = r.reshape(-1, 4)
    rm = rowmask.reshape(-1)
    keep = np.zeros(r.shape, bool)
    keep[:, 0] = (rm & 1) != 0
    keep[:, 1:] = ((rm & 2) != 0)[:, None]
    Jk, rk, wk = J[keep], r[keep], w.reshape(-1, 4)[keep]
    H = Jk.T @ (wk[:, None] * Jk)
    g = Jk.T @ (wk * rk)
    out = np.zeros(29)
    q = 0
    for a in range(6):
        for b2 in range(a, 6):
            out[q] = H[a, b2]
            q += 1
    out[21:27] = g
    out[27] = float(np.sum(wk * rk * rk))
    out[28] = float(np.count_nonzero(rm))
    return out


def irls_neq(rows: Dict[str, np.ndarray], params: Params) -> np.ndarray:
    """Normal equations of one IRLS iteration: the rows of the objective
    with weights irls_weight at their current residuals (depth rows scale
    b_geo, colour rows b_rgb; the gates are those of the squared form)."""
    r = rows["resid"].reshape(-1, 4)
    w = np.empty_like(r)
    w[:, 0] = irls_weight(r[:, 0], params.b_geo, params.irls_floor)
    w[:, 1:] = irls_weight(r[:, 1:], params.b_rgb, params.irls_floor)
    return neq_from_rows(rows["J"], r, rows["rowmask"], w)


def adam_gradient(cam: Cam, pose, prior, Lp, pose_prev, obs_depth, obs_rgb, anchor, params: Params,
                  pixels: np.ndarray, decide32: bool = True) -> np.ndarray:
    """Gradient w.r.t. the pose perturbation of the MAP objective whose data
    term is the P2 rows of the sampled pixels (row-major indices; outside the
    image: no rows; repeats count repeatedly), scaled by (image pixels /
    sampled pixels) to estimate the full-frame sum:
        scale * sum 2 w r dr/ddelta  +  Lp e(pose, prior)."""
    H, W = cam.height, cam.width
    out = track_p2(cam, pose, pose_prev, obs_depth, obs_rgb, anchor, params, decide32, want_J=True)
    J = out["J"].reshape(H * W, 4, 6)
    r = out["resid"].reshape(H * W, 4)
    rm = out["rowmask"].reshape(H * W)
    idx = np.asarray(pixels)
    idx = idx[(idx >= 0) & (idx < H * W)]
    g = np.zeros(6)
    geo = idx[(rm[idx] & 1) != 0]
    g += (1.0 / params.b_geo ** 2) * (r[geo, 0, None] * J[geo, 0]).sum(0)
    pho = idx[(rm[idx] & 2) != 0]
    g += (1.0 / params.b_rgb ** 2) * (r[pho, 1:, None] * J[pho, 1:]).sum((0, 1))
    scale = H * W / len(pixels)
    return 2.0 * scale * g + Lp @ pose_error(pose, prior)


def adam_pose(cam: Cam, prior, Lp, pose_prev, obs_depth, obs_rgb, anchor, params: Params,
              pixels: np.ndarray, lr_t: float, lr_r: float, beta2: float = 0.999, eps: float = 1e-8,
              decide32: bool = True) -> np.ndarray:
    """The paper's pose optimiser (App. G) on the MAP objective of Sec. 4.3.2
    with the P2 data term: Adam with the first moment switched off (each
    step follows the current gradient), per-component step sizes (lr_t for
    translation, lr_r for rotation), one row of `pixels` per step, starting
    from the prior mean.  Steps are left retractions, as in Gauss-Newton."""
    lr = np.array([lr_t] * 3 + [lr_r] * 3)
    it = _f64(prior).copy()
    v = np.zeros(6)
    for k in range(len(pixels)):
        g = adam_gradient(cam, it, prior, Lp, pose_prev, obs_depth, obs_rgb, anchor, params, pixels[k], decide32)
        v = beta2 * v + (1.0 - beta2) * g * g
        vhat = v / (1.0 - beta2 ** (k + 1))
        it = retract(it, -lr * g / (np.sqrt(vhat) + eps))
    return it


def laplace(neq: np.ndarray, Lp: np.ndarray, factor: float = 2.0) -> np.ndarray:
    """Laplace covariance at the MAP pose, Hessian from the squared Jacobian of
    the full objective including the dynamics prior: (2 H + Lp)^-1 as Sec. 5.1
    prints it, or (H + Lp)^-1 with factor 1."""
    H, _, _, _ = neq_unpack(neq)
    A = factor * H + Lp
    Ai = np.linalg.inv(A)
    return 0.5 * (Ai + Ai.T)


def combine(pose_post: np.ndarray, S_pose: np.ndarray, prior_pose: np.ndarray, mu_v: np.ndarray,
            D: np.ndarray, S_v: np.ndarray):
    """Product of the pose posterior N(m, S_pose) with the velocity
    conditional: velocity mean mu_v + D e (e = posterior offset from the prior
    pose) and the joint covariance [[S, S D^T], [D S, S_v + D S D^T]]."""
    e = pose_error(pose_post, prior_pose)
    v_mean = mu_v + D @ e
    n = 6 + len(mu_v)
    P = np.zeros((n, n))
    P[:6, :6] = S_pose
    P[:6, 6:] = S_pose @ D.T
    P[6:, :6] = D @ S_pose
    P[6:, 6:] = S_v + D @ S_pose @ D.T
    return v_mean, 0.5 * (P + P.T)


def transition_sample(x: Dict[str, np.ndarray], u: np.ndarray, n: np.ndarray, dt: float,
                      dt2: bool = False) -> Dict[str, np.ndarray]:
    """One draw of the generative transition (App. B): Euler integration with
    additive noise n = (n_t, n_theta, n_v, n_w): velocities first, then the
    position with the new velocity, the rotation by Exp(w' dt) and the
    rotation noise on the left.  dt2: the control enters as u dt^2 (App. E.1
    as printed)."""
    du = dt * dt if dt2 else dt
    v = x["v"] + u[:3] * du + n[6:9]
    w = x["w"] + u[3:] * du + n[9:12]
    t = x["t"] + v * dt + n[0:3]
    R = so3_exp(n[3:6]) @ so3_exp(w * dt) @ quat_to_rot(x["q"])
    return dict(t=t, q=rot_to_quat(R), v=v, w=w)


def transition_sample_bias(x: Dict[str, np.ndarray], u: np.ndarray, n: np.ndarray, dt: float, g,
                           dt2: bool = False) -> Dict[str, np.ndarray]:
    """One draw of the 15-D transition: the acceleration R (f - b) + g from the
    draw's own rotation and bias, then transition_sample with the first 12
    noise components; the bias walks by n_b = n[12:15]."""
    R = quat_to_rot(x["q"])
    a = R @ (u[:3] - x["b"]) + np.asarray(g, float)
    xn = transition_sample(x, np.concatenate([a, u[3:]]), n[:12], dt, dt2)
    xn["b"] = x["b"] + n[12:15]
    return xn


def rollout(grid: Grid, mean: np.ndarray, cam: Cam, x: Dict[str, np.ndarray], P: np.ndarray, u: np.ndarray,
            noise: np.ndarray, params: Params, decide32: bool = True, frames: bool = True):
    """Predictive rollout (App. J): from the belief N(x, P) and the map means,
    under controls u [k][6]: for each sample s the start state x (+) L z[s,0]
    (P = L L^T; tangent order t, theta, v, w, and b for the 15-D state) and k
    draws of the transition with noise sqrt(diag Q) z[s,j+1]; the closed-form
    predicted moments after each control (means t, q, v, w and b); the frames
    rendered at every sampled pose."""
    k = len(u)
    nd = 15 if params.accel_bias else 12
    sig = np.sqrt([params.sigma_pose_t ** 2] * 3 + [params.sigma_pose_r ** 2] * 3 +
                  [params.sigma_vel_t ** 2] * 3 + [params.sigma_vel_r ** 2] * 3 +
                  ([params.sigma_bias ** 2] * 3 if params.accel_bias else []))
    try:
        L = np.linalg.cholesky(P)
        ok = True
    except np.linalg.LinAlgError:
        L, ok = np.zeros((nd, nd)), False
    poses = np.zeros((len(noise), k, 7))
    for s in range(len(noise)):
        e = L @ noise[s, 0]
        p0 = retract(np.concatenate([x["t"], x["q"]]), e[:6])
        xs = dict(t=p0[:3], q=p0[3:], v=x["v"] + e[6:9], w=x["w"] + e[9:12])
        if params.accel_bias:
            xs["b"] = x["b"] + e[12:15]
        for j in range(k):
            if params.accel_bias:
                xs = transition_sample_bias(xs, u[j], sig * noise[s, j + 1], params.dt, params.gravity,
                                            params.transition_dt2)
            else:
                xs = transition_sample(xs, u[j], sig * noise[s, j + 1], params.dt, params.transition_dt2)
            poses[s, j] = np.concatenate([xs["t"], xs["q"]])
    means, covs = np.zeros((k, nd + 1)), np.zeros((k, nd, nd))
    xm, Pm = dict(x), P
    for j in range(k):
        xm, Pm = predict(xm, Pm, u[j], params)
        means[j] = np.concatenate([xm["t"], xm["q"], xm["v"], xm["w"]] + ([xm["b"]] if params.accel_bias else []))
        covs[j] = Pm
    out = dict(poses=poses, mean=means, cov=covs, ok=ok)
    if frames:
        out["frames"] = [render(grid, mean, cam, poses[s, j], decide32) for s in range(len(noise)) for j in range(k)]
    return out


# ---------------------------------------------------------------------------
# the filter (Sec. 4.3)
# ---------------------------------------------------------------------------
def _is_pd(A: np.ndarray) -> bool:
    try:
        np.linalg.cholesky(A)
        return True
    except np.linalg.LinAlgError:
        return False


@dataclass
class FilterState:
    t: np.ndarray
    q: np.ndarray
    v: np.ndarray
    w: np.ndarray
    P: np.ndarray                      # 12x12 covariance, tangent (dt, dth, dv, dw); 15x15 with db
    Sbar: Optional[np.ndarray] = None  # EMA of Laplace pose covariances
    b: Optional[np.ndarray] = None     # accelerometer bias (15-D state only)
    step: int = 0
    anchor: Optional[Dict[str, np.ndarray]] = None
    anchor_pose: Optional[np.ndarray] = None
    last: Dict = field(default_factory=dict)

    @property
    def pose(self) -> np.ndarray:
        return np.concatenate([self.t, self.q])


class Filter:
    """FP64 reference of one agent's PRISM filter: map belief (dense mean and
    variance) plus the Gaussian state belief."""

    def __init__(self, grid: Grid, cam: Cam, params: Params, x0: Dict[str, np.ndarray],
                 P0: np.ndarray, mean: np.ndarray, var: np.ndarray, decide32: bool = True):
        self.grid, self.cam, self.p = grid, cam, params
        self.mean = _f64(mean).copy()
        self.var = _f64(var).copy()
        self.decide32 = decide32
        self.s = FilterState(b=_f64(x0.get("b", np.zeros(3))).copy() if params.accel_bias else None,
                             t=_f64(x0["t"]).copy(), q=_f64(x0["q"]).copy(),
                             v=_f64(x0["v"]).copy(), w=_f64(x0["w"]).copy(), P=_f64(P0).copy())

    def _observe_and_anchor(self, pose, depth, rgb):
        """Map update at the current mean (App. C nominal state), then render
        the next anchor from the updated map at that mean."""
        n = map_update(self.grid, self.mean, self.var, self.cam, pose, depth, rgb, self.p,
                       self.decide32)
        a = render(self.grid, self.mean[0:4], self.cam, pose, self.decide32, normals=True,
                   normal_disc=self.p.normal_disc)
        self.s.anchor = a
        self.s.anchor_pose = pose.copy()
        self.s.last["n_updated"] = n

    def step(self, depth: np.ndarray, rgb: np.ndarray, u: Optional[np.ndarray],
             adam: Optional[Dict] = None) -> FilterState:
        """One filter step; `adam` (keys pixels, lr_t, lr_r, beta2, eps)
        replaces the Gauss-Newton iterations by the paper's optimiser."""
        s, p = self.s, self.p
        if s.step == 0:
            self._observe_and_anchor(s.pose, depth, rgb)
            s.step += 1
            return s
        # predict and split (App. E.1-E.2)
        xn, Pm = predict(dict(t=s.t, q=s.q, v=s.v, w=s.w, b=s.b), s.P, u, p)
        prior = np.concatenate([xn["t"], xn["q"]])
        if not _is_pd(Pm[:6, :6]):
            # the paper assumes a proper Gaussian belief; a predicted pose
            # covariance that is not positive definite has no MAP problem,
            # so the step keeps the prediction and still updates the map
            s.t, s.q, s.v, s.w, s.P = xn["t"], xn["q"], xn["v"], xn["w"], Pm
            if p.accel_bias:
                s.b = xn["b"]
            s.last.update(neq=None, S_lap=None, prior=prior, prior_not_pd=True)
            self._observe_and_anchor(prior, depth, rgb)
            s.step += 1
            return s
        s.last["prior_not_pd"] = False
        Spp, D, Sv = split(Pm)
        Lp = np.linalg.inv(Spp)
        Lp = 0.5 * (Lp + Lp.T)
        # MAP pose from the prior mean (Sec. 4.3.2): Gauss-Newton, or the
        # paper's optimiser on sampled pixels (App. G)
        it = prior.copy()
        if adam is not None:
            assert p.objective == "p2"
            it = adam_pose(self.cam, prior, Lp, self.s.anchor_pose, depth, rgb, self.s.anchor, p, adam["pixels"],
                           adam["lr_t"], adam["lr_r"], adam.get("beta2", 0.999), adam.get("eps", 1e-8),
                           self.decide32)
        else:
            for _ in range(p.n_gn):
                neq = self._objective(it, depth, rgb, irls=p.irls)
                delta = gn_solve(neq, Lp, pose_error(it, prior))
                it = retract(it, delta)
        # the Laplace Hessian is the squared Jacobian of the objective's rows
        # (App. E.3), also when the iterations minimised the L1 form
        neq = self._objective(it, depth, rgb)
        S_lap = laplace(neq, Lp, p.laplace_factor)
        s.Sbar = S_lap if s.Sbar is None else p.ema * s.Sbar + (1.0 - p.ema) * S_lap
        vel_prior = np.concatenate([xn["v"], xn["w"]] + ([xn["b"]] if p.accel_bias else []))
        v_mean, P = combine(it, s.Sbar, prior, vel_prior, D, Sv)
        s.t, s.q = it[:3].copy(), it[3:].copy()
        s.v, s.w = v_mean[:3].copy(), v_mean[3:6].copy()
        if p.accel_bias:
            s.b = v_mean[6:9].copy()
        s.P = P
        s.last.update(neq=neq, S_lap=S_lap, prior=prior)
        # map filter with the current state mean, then the next anchor
        self._observe_and_anchor(it, depth, rgb)
        s.step += 1
        return s

    def _objective(self, pose, depth, rgb, irls: bool = False):
        if self.p.objective == "p1":
            out = render_jacobian(self.grid, self.mean, self.cam, pose, depth, rgb, self.p,
                                  self.decide32, want_J=irls)
        else:
            out = track_p2(self.cam, pose, self.s.anchor_pose, depth, rgb, self.s.anchor, self.p,
                           self.decide32, want_J=irls)
        return irls_neq(out, self.p) if irls else out["neq"]
