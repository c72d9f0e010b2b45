"""Seeded synthetic inputs: rooms, boxes, cameras, trajectories, RGB-D frames.

This module produces the *inputs* of the filter and nothing else.  It holds
none of the method's arithmetic (no rendering through the voxel field, no map
or pose updates); it uses analytic geometry only:

* a room is the complement of an axis-aligned "inner box" (walls are solid out
  to infinity), plus a few solid axis-aligned boxes inside it;
* the ground-truth voxel map is the clamped negative signed distance of that
  union, sampled at voxel centres, with the colour of the nearest solid;
* observed depth and colour come from exact ray/box intersections, plus
  Gaussian noise.

Conventions (shared by every consumer of these inputs, not by their code):
world is right-handed with z up; a camera pose (t, q) maps camera coordinates
to world coordinates, X_w = R(q) X_c + t, q = (w, x, y, z); the camera frame is
the usual pinhole one (x right, y down, z forward); a pixel (u, v) looks along
((u + 1/2 - cx)/fx, (v + 1/2 - cy)/fy, 1), so depth is z-depth.

Dense map arrays are float64 [4][N][N][N] (channel, k, j, i), x fastest;
channel 0 is occupancy (= -SDF, positive inside solids), 1..3 are RGB.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

G_WORLD = np.array([0.0, 0.0, -9.81])


# --------------------------------------------------------------------------
# small rotation helpers (generator-side only)
# --------------------------------------------------------------------------
def _quat_to_mat(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _mat_to_quat(R: np.ndarray) -> np.ndarray:
    # Shepperd's method
    tr = np.trace(R)
    if tr > 0:
        S = math.sqrt(tr + 1.0) * 2
        q = [0.25 * S, (R[2, 1] - R[1, 2]) / S, (R[0, 2] - R[2, 0]) / S, (R[1, 0] - R[0, 1]) / S]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        S = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / S, 0.25 * S, (R[0, 1] + R[1, 0]) / S, (R[0, 2] + R[2, 0]) / S]
    elif R[1, 1] > R[2, 2]:
        S = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / S, (R[0, 1] + R[1, 0]) / S, 0.25 * S, (R[1, 2] + R[2, 1]) / S]
    else:
        S = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / S, (R[0, 2] + R[2, 0]) / S, (R[1, 2] + R[2, 1]) / S, 0.25 * S]
    q = np.array(q)
    if q[0] < 0:
        q = -q
    return q / np.linalg.norm(q)


def _axis_angle(v: np.ndarray) -> np.ndarray:
    th = float(np.linalg.norm(v))
    K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    K = K / th
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * (K @ K)


def camera_rotation(yaw: float, pitch: float = 0.0, roll: float = 0.0) -> np.ndarray:
    """Camera->world rotation for an optical axis at heading `yaw` (radians
    about world z), tilted by `pitch` (positive lowers the axis towards -z)
    and rolled by `roll` about the axis."""
    fwd = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.array([0.0, 0.0, -1.0])
    R0 = np.stack([right, down, fwd], axis=1)
    # pitch about camera x (negative: up), roll about camera z
    Rp = _axis_angle(np.array([-pitch, 0.0, 0.0]))
    Rr = _axis_angle(np.array([0.0, 0.0, roll]))
    return R0 @ Rp @ Rr


# --------------------------------------------------------------------------
# scene
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    n: int                    # voxels per axis
    voxel: float              # voxel edge (m)
    origin: np.ndarray        # grid min corner (m), shape [3]
    inner_lo: np.ndarray      # room interior (free) box
    inner_hi: np.ndarray
    boxes: np.ndarray         # [nb, 2, 3]: centre, half-size
    colours: np.ndarray       # [6 + nb, 3]: walls (-x,+x,-y,+y,-z,+z), then boxes
    clamp_voxels: float = 4.0
    texture: float = 0.0      # amplitude of a smooth solid colour texture (0: flat colours)
    tex_waves: np.ndarray | None = None   # [2, 3, 3] wave vectors (cycles/m) per channel
    tex_phase: np.ndarray | None = None   # [2, 3]

    def colour_at(self, sid: np.ndarray, p: np.ndarray) -> np.ndarray:
        """Colour of solid `sid` at points p: flat colour plus the texture."""
        c = self.colours[sid]
        if self.texture > 0:
            t = np.zeros(c.shape)
            for w in range(2):
                t += np.sin(2 * np.pi * (p @ self.tex_waves[w].T) + self.tex_phase[w])
            c = np.clip(c + 0.5 * self.texture * t, 0.0, 1.0)
        return c

    @property
    def extent(self) -> float:
        return self.n * self.voxel

    @property
    def centre(self) -> np.ndarray:
        return self.origin + 0.5 * self.extent


def _box_sdf(p: np.ndarray, c: np.ndarray, h: np.ndarray) -> np.ndarray:
    d = np.abs(p - c) - h
    out = np.linalg.norm(np.maximum(d, 0.0), axis=-1)
    ins = np.minimum(np.max(d, axis=-1), 0.0)
    return out + ins


def make_scene(n: int, voxel: float, seed: int, n_boxes: int = 3,
               keep_clear: np.ndarray | None = None, clear_radius: float = 0.5,
               texture: float = 0.0) -> Scene:
    """Room filling the grid (4-voxel wall shell) plus `n_boxes` random boxes.

    Boxes closer than `clear_radius` to any point of `keep_clear` (camera
    positions) are rejected and redrawn.  `texture` > 0 adds a smooth solid
    colour texture (wavelengths 0.4-1 m) so photometric alignment is
    well posed on flat walls."""
    rng = np.random.default_rng(seed)
    E = n * voxel
    origin = np.zeros(3)
    wall = 4 * voxel
    inner_lo = origin + wall
    inner_hi = origin + E - wall
    colours = rng.uniform(0.0, 1.0, size=(6 + n_boxes, 3))
    boxes = []
    tries = 0
    while len(boxes) < n_boxes:
        tries += 1
        if tries > 10000:
            raise RuntimeError("could not place boxes")
        h = rng.uniform(0.05, 0.15, size=3) * E
        c = rng.uniform(inner_lo + h, inner_hi - h)
        if keep_clear is not None and len(keep_clear):
            d = _box_sdf(np.asarray(keep_clear, float), c, h)
            if np.min(d) < clear_radius:
                continue
        boxes.append((c, h))
    trng = np.random.default_rng(seed + 104729)
    waves = trng.normal(size=(2, 3, 3))
    waves *= trng.uniform(1.0, 2.5, size=(2, 3, 1)) / np.linalg.norm(waves, axis=-1, keepdims=True)
    phase = trng.uniform(0, 2 * np.pi, size=(2, 3))
    return Scene(n=n, voxel=voxel, origin=origin, inner_lo=inner_lo, inner_hi=inner_hi,
                 boxes=np.array(boxes).reshape(n_boxes, 2, 3), colours=colours,
                 texture=texture, tex_waves=waves, tex_phase=phase)


def scene_sdf(scene: Scene, p: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Signed distance to the solid union (positive in free space) and the
    index of the nearest solid (0..5 walls, 6.. boxes) for points p[..., 3]."""
    p = np.asarray(p, float)
    lo, hi = scene.inner_lo, scene.inner_hi
    # walls: distance from p to each inner face (positive inside the room)
    faces = np.stack([p[..., 0] - lo[0], hi[0] - p[..., 0],
                      p[..., 1] - lo[1], hi[1] - p[..., 1],
                      p[..., 2] - lo[2], hi[2] - p[..., 2]], axis=-1)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo)
    room_sdf = -_box_sdf(p, c, h)          # positive inside the room
    wall_id = np.argmin(faces, axis=-1)
    sdf = room_sdf
    sid = wall_id
    for b in range(scene.boxes.shape[0]):
        db = _box_sdf(p, scene.boxes[b, 0], scene.boxes[b, 1])
        closer = db < sdf
        sdf = np.where(closer, db, sdf)
        sid = np.where(closer, 6 + b, sid)
    return sdf, sid


def voxel_centres(scene: Scene) -> np.ndarray:
    n, s = scene.n, scene.voxel
    ax = (np.arange(n) + 0.5) * s
    z, y, x = np.meshgrid(ax + scene.origin[2], ax + scene.origin[1], ax + scene.origin[0],
                          indexing="ij")
    return np.stack([x, y, z], axis=-1)   # [k][j][i][3]


def gt_map(scene: Scene, var: float = 1e-2, dtype=np.float64) -> Tuple[np.ndarray, np.ndarray]:
    """Ground-truth dense map (mean [4][N][N][N], var [4][N][N][N]): occupancy
    = -SDF clamped to +-clamp_voxels voxels, colour of the nearest solid at
    the voxel centre."""
    n = scene.n
    mean = np.empty((4, n, n, n), dtype)
    clamp = scene.clamp_voxels * scene.voxel
    ax = (np.arange(n) + 0.5) * scene.voxel
    y, x = np.meshgrid(ax + scene.origin[1], ax + scene.origin[0], indexing="ij")
    step = max(1, (1 << 21) // (n * n))
    for k0 in range(0, n, step):  # slabs, to bound memory
        ks = np.arange(k0, min(n, k0 + step))
        zc = scene.origin[2] + (ks + 0.5) * scene.voxel
        p = np.stack(np.broadcast_arrays(x[None], y[None], zc[:, None, None]), axis=-1)
        sdf, sid = scene_sdf(scene, p)
        mean[0, ks] = np.clip(-sdf, -clamp, clamp)
        mean[1:, ks] = np.moveaxis(scene.colour_at(sid, p), -1, 0)
    return mean, np.full_like(mean, var)


# --------------------------------------------------------------------------
# cameras and analytic ray casting
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    d_near: float
    d_far: float
    n_samples: int
    tau: float = 0.0

    @staticmethod
    def scaled(width: int, height: int, n_samples: int, d_near: float, d_far: float) -> "Camera":
        f = 0.75 * width
        return Camera(width, height, f, f, width / 2.0, height / 2.0, d_near, d_far, n_samples)


def pixel_dirs(cam: Camera) -> np.ndarray:
    """Camera-frame ray directions with unit z, [H, W, 3]."""
    u = np.arange(cam.width) + 0.5
    v = np.arange(cam.height) + 0.5
    uu, vv = np.meshgrid(u, v)
    return np.stack([(uu - cam.cx) / cam.fx, (vv - cam.cy) / cam.fy, np.ones_like(uu)], axis=-1)


def _ray_box_entry(o, d, c, h):
    """Entry parameter of rays o + t d into box (c, h); inf if missed or t <= 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t1 = (c - h - o) * inv
        t2 = (c + h - o) * inv
    tmin = np.max(np.minimum(t1, t2), axis=-1)
    tmax = np.min(np.maximum(t1, t2), axis=-1)
    hit = (tmax >= tmin) & (tmin > 0)
    return np.where(hit, tmin, np.inf)


def raycast(scene: Scene, cam: Camera, t: np.ndarray, q: np.ndarray,
            rng: np.random.Generator | None = None, depth_noise: float = 0.0,
            rgb_noise: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """Exact z-depth [H, W] and colour [H, W, 3] of the first solid along each
    pixel ray, with optional Gaussian noise.  Misses give depth 0 (invalid)."""
    R = _quat_to_mat(np.asarray(q, float))
    dc = pixel_dirs(cam)
    d = dc @ R.T
    o = np.broadcast_to(np.asarray(t, float), d.shape)
    lo, hi = scene.inner_lo, scene.inner_hi
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
    # exit of the room box = first wall hit (camera is inside the room)
    texit_axes = np.maximum(t1, t2)
    wall_axis = np.argmin(texit_axes, axis=-1)
    tw = np.min(texit_axes, axis=-1)
    wall_side = np.take_along_axis(d, wall_axis[..., None], -1)[..., 0] > 0
    sid = 2 * wall_axis + wall_side.astype(int)
    tbest = tw
    for b in range(scene.boxes.shape[0]):
        tb = _ray_box_entry(o, d, scene.boxes[b, 0], scene.boxes[b, 1])
        closer = tb < tbest
        tbest = np.where(closer, tb, tbest)
        sid = np.where(closer, 6 + b, sid)
    depth = tbest.copy()
    hitp = o + np.where(np.isfinite(tbest), tbest, 0.0)[..., None] * d
    rgb = scene.colour_at(sid, hitp)
    if rng is not None:
        if depth_noise > 0:
            depth = depth + rng.normal(0.0, depth_noise, size=depth.shape)
        if rgb_noise > 0:
            rgb = rgb + rng.normal(0.0, rgb_noise, size=rgb.shape)
    depth = np.where(np.isfinite(depth) & (depth > 0), depth, 0.0)
    return depth, rgb


# --------------------------------------------------------------------------
# trajectories and inertial controls
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Trajectory:
    dt: float
    t: np.ndarray      # [T, 3] camera position (world)
    q: np.ndarray      # [T, 4] camera->world quaternion (w, x, y, z)
    v: np.ndarray      # [T, 3] linear velocity (world)
    w: np.ndarray      # [T, 3] angular velocity (world)
    u: np.ndarray      # [T-1, 6] controls between frames: (lin. accel, ang. accel), world
    # [T-1, 6] the same with the accelerometer's body-frame specific force (its
    # mean over the interval, bias and noise included) as the linear part
    u_body: Optional[np.ndarray] = None
    acc_bias: Optional[np.ndarray] = None   # [T-1, 3] true accelerometer bias at each interval's start


def _skew_inv(S):
    return np.array([S[2, 1], S[0, 2], S[1, 0]])


def uav_trajectory(seed: int, n_frames: int, centre: np.ndarray, dt: float = 0.1,
                   max_acc: float = 4.0, max_rate: float = 2.0, amp_cap: float = 1.2,
                   tilt: float = 0.2, imu_hz: float = 200.0, acc_noise: float = 0.02,
                   gyro_noise: float = 0.002, acc_bias_walk: float = 0.001,
                   gyro_bias_walk: float = 0.0001) -> Trajectory:
    """Smooth 6-DoF trajectory: per-axis sinusoids with peak acceleration
    <= max_acc, yaw sinusoid with peak rate <= max_rate, small roll/pitch.

    Controls between frames come from a simulated IMU (accelerometer and gyro
    at `imu_hz` with white noise and a bias random walk): the linear control is
    the frame-interval mean of the rotated specific force plus gravity, the
    angular control is the change of the rotated gyro rate over the interval."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.2, 0.4, size=3)
    A = np.minimum(max_acc / (2 * np.pi * f) ** 2, amp_cap)
    A[2] *= 0.3
    ph = rng.uniform(0, 2 * np.pi, size=3)
    g = rng.uniform(0.1, 0.3)
    Y = min(max_rate / (2 * np.pi * g), np.pi)
    yaw0 = rng.uniform(0, 2 * np.pi)
    fr = rng.uniform(0.2, 0.5, size=2)
    phr = rng.uniform(0, 2 * np.pi, size=2)

    def pose_at(tt):
        p = centre + A * np.sin(2 * np.pi * f * tt + ph)
        yaw = yaw0 + Y * math.sin(2 * np.pi * g * tt)
        pitch = tilt * math.sin(2 * np.pi * fr[0] * tt + phr[0])
        roll = tilt * math.sin(2 * np.pi * fr[1] * tt + phr[1])
        return p, camera_rotation(yaw, pitch, roll)

    def vel_at(tt, h=1e-4):
        p1, R1 = pose_at(tt - h)
        p2, R2 = pose_at(tt + h)
        v = (p2 - p1) / (2 * h)
        Rd = (R2 - R1) / (2 * h)
        _, R = pose_at(tt)
        w = _skew_inv(Rd @ R.T)
        return v, w

    def acc_at(tt):
        return -A * (2 * np.pi * f) ** 2 * np.sin(2 * np.pi * f * tt + ph)

    T = n_frames
    ts = np.arange(T) * dt
    P = np.zeros((T, 3)); Q = np.zeros((T, 4)); V = np.zeros((T, 3)); W = np.zeros((T, 3))
    for i, tt in enumerate(ts):
        p, R = pose_at(tt)
        P[i] = p
        Q[i] = _mat_to_quat(R)
        V[i], W[i] = vel_at(tt)
    # simulated IMU
    n_sub = int(round(imu_hz * dt))
    hs = dt / n_sub
    ba = np.zeros(3); bg = np.zeros(3)
    U = np.zeros((T - 1, 6))
    UB = np.zeros((T - 1, 6))
    BA = np.zeros((T - 1, 3))
    for i in range(T - 1):
        accs, fbs = [], []
        BA[i] = ba
        for j in range(n_sub + 1):
            tt = ts[i] + j * hs
            _, R = pose_at(tt)
            f_b = R.T @ (acc_at(tt) - G_WORLD) + ba + rng.normal(0, acc_noise, 3)
            fbs.append(f_b)
            accs.append(R @ (f_b - 0.0) + G_WORLD)
            ba = ba + rng.normal(0, acc_bias_walk, 3)
        gy = []
        for tt in (ts[i], ts[i + 1]):
            _, R = pose_at(tt)
            _, w = vel_at(tt)
            w_b = R.T @ w + bg + rng.normal(0, gyro_noise, 3)
            gy.append(R @ w_b)
            bg = bg + rng.normal(0, gyro_bias_walk, 3)
        U[i, :3] = np.mean(accs[:-1], axis=0)
        U[i, 3:] = (gy[1] - gy[0]) / dt
        UB[i, :3] = np.mean(fbs[:-1], axis=0)
        UB[i, 3:] = U[i, 3:]
    return Trajectory(dt=dt, t=P, q=Q, v=V, w=W, u=U, u_body=UB, acc_bias=BA)


# --------------------------------------------------------------------------
# workload presets
# --------------------------------------------------------------------------
def perturb_pose(rng: np.random.Generator, t: np.ndarray, q: np.ndarray,
                 sigma_t: float, sigma_r: float) -> Tuple[np.ndarray, np.ndarray]:
    """t + N(0, sigma_t^2 I); rotation left-multiplied by Exp(N(0, sigma_r^2 I))."""
    dt = rng.normal(0.0, sigma_t, 3)
    dr = rng.normal(0.0, sigma_r, 3)
    R = _axis_angle(dr) @ _quat_to_mat(q)
    return t + dt, _mat_to_quat(R)


def single_frame_case(seed: int = 0, n: int = 64, voxel: float = 0.04,
                      width: int = 80, height: int = 60, n_samples: int = 32,
                      d_near: float = 0.1, d_far: float = 3.0) -> Dict:
    """Small single-frame case: 64^3 room of 4 cm voxels, 80x60 camera at the
    room centre with a random heading, 32 samples per ray in [0.1, 3.0] m,
    initial pose perturbed by 2 cm / 1 degree."""
    rng = np.random.default_rng(seed)
    E = n * voxel
    centre = np.full(3, E / 2)
    scene = make_scene(n, voxel, seed, keep_clear=centre[None], clear_radius=0.5)
    yaw = rng.uniform(0, 2 * np.pi)
    q_gt = _mat_to_quat(camera_rotation(yaw))
    t_gt = centre.copy()
    t0, q0 = perturb_pose(rng, t_gt, q_gt, 0.02, math.radians(1.0))
    cam = Camera(width, height, 0.75 * width, 0.75 * width, width / 2, height / 2,
                 d_near, d_far, n_samples)
    return dict(scene=scene, cam=cam, t_gt=t_gt, q_gt=q_gt, t_init=t0, q_init=q0)


def trajectory_case(seed: int = 1, n: int = 256, width: int = 320, height: int = 240,
                    n_samples: int = 128, n_frames: int = 300, room: float = 6.4,
                    d_near: float = 0.1, d_far: float = 7.5, depth_noise: float = 0.01,
                    rgb_noise: float = 0.02, frames: bool = True, texture: float = 0.25) -> Dict:
    """Single-stream trajectory: N^3 grid over a `room`-metre cube, W x H RGB-D
    frames at 10 Hz along a UAV-like trajectory, depth noise N(0, 1 cm),
    colour noise N(0, 0.02)."""
    voxel = room / n
    centre = np.full(3, room / 2)
    traj = uav_trajectory(seed, n_frames, centre)
    scene = make_scene(n, voxel, seed, keep_clear=traj.t, clear_radius=0.5, texture=texture)
    cam = Camera.scaled(width, height, n_samples, d_near, d_far)
    out = dict(scene=scene, cam=cam, traj=traj)
    if frames:
        rng = np.random.default_rng(seed + 7919)
        D = np.zeros((n_frames, height, width), np.float32)
        C = np.zeros((n_frames, height, width, 3), np.float32)
        for i in range(n_frames):
            d, c = raycast(scene, cam, traj.t[i], traj.q[i], rng, depth_noise, rgb_noise)
            D[i] = d
            C[i] = c
        out["depth"] = D
        out["rgb"] = C
    return out


def sample_pixels(seed: int, n_steps: int, n_pixels: int, height: int, width: int) -> np.ndarray:
    """Pixel indices v*W+u drawn uniformly with replacement, one row of
    n_pixels per optimisation step: int32 [n_steps][n_pixels]."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, height * width, size=(n_steps, n_pixels), dtype=np.int64).astype(np.int32)


def pose7(t: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Pose as the 7 doubles (tx, ty, tz, qw, qx, qy, qz)."""
    return np.concatenate([np.asarray(t, float), np.asarray(q, float)])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float32 (exactly representable)."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


# --------------------------------------------------------------------------
# device-side frame generation (large serving workloads)
# --------------------------------------------------------------------------
def raycast_torch(scene: Scene, cam: Camera, ts: np.ndarray, qs: np.ndarray, seed: int,
                  depth_noise: float = 0.0, rgb_noise: float = 0.0, device="cuda", chunk: int = 16):
    """Same analytic ray cast as `raycast`, for a batch of poses ts [F,3],
    qs [F,4], evaluated with torch on `device` in float64 and returned as
    float32 depth [F,H,W] and colour [F,H,W,3].  Noise comes from a torch
    generator seeded with `seed` (so values differ from `raycast`'s numpy
    noise; the noise-free part agrees to rounding)."""
    import torch
    F = len(ts)
    H, W = cam.height, cam.width
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dc = torch.as_tensor(pixel_dirs(cam), dtype=torch.float64, device=device)          # [H,W,3]
    Rs = torch.as_tensor(np.stack([_quat_to_mat(np.asarray(q, float)) for q in qs]), dtype=torch.float64,
                         device=device)
    T = torch.as_tensor(np.asarray(ts, float), dtype=torch.float64, device=device)
    lo = torch.as_tensor(scene.inner_lo, dtype=torch.float64, device=device)
    hi = torch.as_tensor(scene.inner_hi, dtype=torch.float64, device=device)
    cols = torch.as_tensor(scene.colours, dtype=torch.float64, device=device)
    boxes = torch.as_tensor(scene.boxes, dtype=torch.float64, device=device)
    depth_out = torch.empty((F, H, W), dtype=torch.float32, device=device)
    rgb_out = torch.empty((F, H, W, 3), dtype=torch.float32, device=device)
    for f0 in range(0, F, chunk):
        f1 = min(F, f0 + chunk)
        d = torch.einsum("hwj,fij->fhwi", dc, Rs[f0:f1])                             # world directions
        o = T[f0:f1, None, None, :].expand_as(d)
        inv = 1.0 / d
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
        texit = torch.maximum(t1, t2)
        tw, wall_axis = torch.min(texit, dim=-1)
        wall_side = torch.gather(d, -1, wall_axis[..., None])[..., 0] > 0
        sid = 2 * wall_axis + wall_side.long()
        tbest = tw
        for b in range(boxes.shape[0]):
            c, h = boxes[b, 0], boxes[b, 1]
            b1 = (c - h - o) * inv
            b2 = (c + h - o) * inv
            tmin = torch.minimum(b1, b2).amax(-1)
            tmax = torch.maximum(b1, b2).amin(-1)
            hit = (tmax >= tmin) & (tmin > 0)
            tb = torch.where(hit, tmin, torch.full_like(tmin, math.inf))
            closer = tb < tbest
            tbest = torch.where(closer, tb, tbest)
            sid = torch.where(closer, torch.full_like(sid, 6 + b), sid)
        fin = torch.isfinite(tbest)
        hitp = o + torch.where(fin, tbest, torch.zeros_like(tbest))[..., None] * d
        c = cols[sid]
        if scene.texture > 0:
            wv = torch.as_tensor(scene.tex_waves, dtype=torch.float64, device=device)
            ph = torch.as_tensor(scene.tex_phase, dtype=torch.float64, device=device)
            tex = torch.zeros_like(c)
            for w in range(2):
                tex = tex + torch.sin(2 * math.pi * (hitp @ wv[w].T) + ph[w])
            c = torch.clamp(c + 0.5 * scene.texture * tex, 0.0, 1.0)
        depth = tbest
        if depth_noise > 0:
            depth = depth + depth_noise * torch.randn(depth.shape, generator=gen, dtype=torch.float64, device=device)
        if rgb_noise > 0:
            c = c + rgb_noise * torch.randn(c.shape, generator=gen, dtype=torch.float64, device=device)
        depth = torch.where(torch.isfinite(depth) & (depth > 0), depth, torch.zeros_like(depth))
        depth_out[f0:f1] = depth.float()
        rgb_out[f0:f1] = c.float()
    return depth_out, rgb_out


def serving_streams(n_streams: int = 16, n_frames: int = 300, seed_base: int = 1000,
                    sizes=((160, 120), (320, 240), (640, 480)), grids=(128, 256, 384),
                    room: float = 6.4, d_near: float = 0.1, d_far: float = 7.5, period: float = 0.1,
                    jitter_mean: float = 0.01) -> List[Dict]:
    """Agent streams for the serving workload.  Stream i (seed seed_base + i)
    draws its image size from `sizes` and its grid from `grids` (K = N/2
    samples over [d_near, d_far] in a `room`-metre cube), has its own scene
    and UAV trajectory, and its frame k arrives at T_i + period*k + J_k with
    T_i ~ U[0, period) and J_k ~ Exp(mean jitter_mean) (kept in order)."""
    out = []
    for i in range(n_streams):
        seed = seed_base + i
        rng = np.random.default_rng(seed)
        w, h = sizes[int(rng.integers(len(sizes)))]
        n = int(grids[int(rng.integers(len(grids)))])
        T0 = rng.uniform(0.0, period)
        arr = T0 + period * np.arange(n_frames) + rng.exponential(jitter_mean, n_frames)
        arr = np.maximum.accumulate(arr)
        voxel = room / n
        traj = uav_trajectory(seed, n_frames, np.full(3, room / 2))
        scene = make_scene(n, voxel, seed, keep_clear=traj.t, clear_radius=0.5, texture=0.25)
        cam = Camera.scaled(w, h, n // 2, d_near, d_far)
        out.append(dict(seed=seed, width=w, height=h, n=n, scene=scene, cam=cam, traj=traj, arrivals=arr))
    return out
