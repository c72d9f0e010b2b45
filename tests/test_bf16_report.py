"""Mixed precision on the large workload: BF16 map storage, single-precision
ray accumulation, FP64 normal equations / Cholesky / covariance update,
against the FP64 oracle, output by output.

Workload: 384^3 grid over a 6.4 m room (1.67 cm voxels), 640x480 RGB-D, 192
samples per ray in [0.1, 7.5] m, 200 frames of a UAV-like trajectory, the
prediction-to-observation objective with 3 Gauss-Newton iterations.  The GPU
filter runs the whole trajectory with a BF16 map.  At checkpoint frames the
oracle is teacher-forced: it starts from exactly the GPU's state before the
step (pose, velocities, covariance, EMA'd Laplace covariance, anchor frame
and pose, and the map values the BF16 map holds, in float64) and takes the
same step with float64 map storage (the map update and the next anchor at
the GPU's posterior mean).  Per output the difference then measures
what BF16 storage and single-precision arithmetic cost in one step, with no
closed-loop drift mixed in:

* map mean and variance: the only rounding is the final store, so every
  voxel is within 2^-8 (+ the FP32 rounding before it) of the oracle's value,
  relative;
* pose and covariance: within the pose tolerance (1e-5 m / rad) and 1e-4
  relative (Frobenius);
* anchor depth and colour rendered from the updated map: reported as
  quantiles; bounded loosely (BF16 moves the occupancy zero crossing).

Run twice: with the paper's 12-D state, and with the 15-D state that adds an
accelerometer bias (fed the accelerometer's body-frame force; the 15x15
covariance and the bias are compared too, the bias within 1e-4).

The reports are written to $PRISM_REPORT_DIR (default: gpurun_out/ at the
repository root, the folder GPU runs bring back) as bf16_error_report.json
and bf16_error_report_15d.json."""
import json
import os

import numpy as np
import pytest

import oracle as orc
import synth

CHECK = (1, 2, 3, 25, 50, 100, 150, 199)


def _q(x, qs=(50, 99, 100)):
    x = np.asarray(x, float)
    return {f"p{q}": float(np.percentile(x, q)) if x.size else 0.0 for q in qs}


@pytest.mark.gpu
@pytest.mark.parametrize("state_dim", [12, 15])
def test_bf16_per_output_error_vs_fp64_oracle(state_dim):
    import torch
    from gpu_util import banner, P, rot_angle
    Pm = P()
    bias = state_dim == 15
    banner(f"BF16 384^3 640x480 K=192, 200 frames, {state_dim}-D state: per-output error vs FP64 oracle")
    n, W, H, K, nf = 384, 640, 480, 192, 200
    case = synth.trajectory_case(seed=4, n=n, width=W, height=H, n_samples=K, n_frames=nf, frames=False)
    sc, cm, tr = case["scene"], case["cam"], case["traj"]
    D, C = synth.raycast_torch(sc, cm, tr.t, tr.q, 4, 0.01, 0.02)
    U = torch.tensor(tr.u_body if bias else tr.u, dtype=torch.float64, device="cuda")
    grid = Pm.Grid.make(n, sc.voxel, tuple(float(v) for v in sc.origin), dtype=Pm.PRISM_BF16)
    cam = Pm.Camera.make(cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy, cm.d_near, cm.d_far, cm.n_samples)
    params = Pm.FilterParams(n_gn=3, objective=Pm.OBJ_P2, modes=Pm.MODE_ACCEL_BIAS if bias else 0)
    op = orc.Params(n_gn=3, objective="p2", accel_bias=bias, sigma_bias=params.sigma_bias,
                    gravity=tuple(params.gravity))
    og, oc = orc.grid_from_scene(sc), orc.cam_from(cm)
    torch.cuda.synchronize()
    f = Pm.Filter(grid, cam, params)
    f.map.init()
    P0 = np.diag([1e-6] * 6 + [1e-4] * 6 + ([1e-4] * 3 if bias else []))
    f.reset(np.concatenate([tr.t[0], tr.q[0], tr.v[0], tr.w[0]] + ([np.zeros(3)] if bias else [])), P0)
    report = {"workload": f"384^3 BF16 map, 640x480, K=192, P2 x 3 GN, 200 frames, {state_dim}-D state"
                          + (" (accelerometer bias; body-frame force as the linear control)" if bias else ""),
              "frames": []}
    rel_bound = 2.0 ** -8 + 2.0 ** -22      # round to 8 significant bits, after the FP32 rounding
    for k in range(nf):
        u = None if k == 0 else U[k - 1]
        if k not in CHECK:
            f.step(D[k], C[k], u)
            continue
        torch.cuda.synchronize()
        st = f.state()
        a = {key: v.cpu().numpy() for key, v in f.anchor().items()}
        mean, var = f.map.to_dense()
        mean64 = mean.cpu().numpy().astype(np.float64)      # exactly the BF16 values the map holds
        var64 = var.cpu().numpy().astype(np.float64)
        del mean, var
        # oracle state filter from the GPU's state (its map is not used by the P2 objective)
        x0 = dict(t=np.array(st.pose.t), q=np.array(st.pose.q), v=np.array(st.v), w=np.array(st.w))
        Pst = np.array(st.P).reshape(12, 12)
        if bias:
            xb = f.bias_state()
            x0["b"] = np.array(xb.b)
            Pst = np.array(xb.P).reshape(15, 15)
        dummy = np.zeros((4, 1, 1, 1))
        of = orc.Filter(og, oc, op, x0, Pst, dummy, dummy)
        of._observe_and_anchor = lambda pose, depth, rgb: None
        of.s.step = int(st.step)
        if st.has_sbar:
            of.s.Sbar = np.array(st.Sbar).reshape(6, 6)
        of.s.anchor = dict(depth=a["depth"].astype(np.float64), rgb=a["rgb"].astype(np.float64), mask=a["mask"],
                           normals=a["normals"].astype(np.float64), nmask=a["nmask"])
        of.s.anchor_pose = np.concatenate([np.array(st.anchor.t), np.array(st.anchor.q)])
        f.step(D[k], C[k], u)
        d64 = D[k].cpu().numpy().astype(np.float64)
        c64 = C[k].cpu().numpy().astype(np.float64)
        of.step(d64, c64, None if u is None else u.cpu().numpy())
        torch.cuda.synchronize()
        sg = f.state()
        assert sg.flags == 0
        e_t = float(np.linalg.norm(np.array(sg.pose.t) - of.s.t))
        e_r = rot_angle(np.array(sg.pose.q), of.s.q)
        Pg = np.array(f.bias_state().P).reshape(15, 15) if bias else np.array(sg.P).reshape(12, 12)
        e_P = float(np.linalg.norm(Pg - of.s.P) / np.linalg.norm(of.s.P))
        e_b = float(np.linalg.norm(np.array(f.bias_state().b) - of.s.b)) if bias else 0.0
        # oracle map filter and anchor with float64 storage, at the GPU's posterior mean
        pose_g = np.concatenate([np.array(sg.pose.t), np.array(sg.pose.q)])
        orc.map_update(og, mean64, var64, oc, pose_g, d64, c64, op)
        ao = orc.render(og, mean64, oc, pose_g, normals=True, normal_disc=op.normal_disc)
        mg, vg = f.map.to_dense()
        row = {"frame": k, "pose_t_m": e_t, "pose_r_rad": e_r, "cov_rel_fro": e_P}
        if bias:
            row["bias_m_s2"] = e_b
        for name, g, o in (("map_mean", mg, mean64), ("map_var", vg, var64)):
            g = g.cpu().numpy().astype(np.float64)
            diff = np.abs(g - o)
            rel = diff / np.maximum(np.abs(o), 1e-30)
            changed = diff > 0
            row[name] = {"max_rel": float(rel.max()), "n_differ": int(changed.sum()), "max_abs": float(diff.max())}
            assert rel.max() <= rel_bound, (k, name, float(rel.max()))
            del g, diff, rel, changed
        del mg, vg
        ag = {key: v.cpu().numpy() for key, v in f.anchor().items()}
        both = (ag["mask"] == 1) & (ao["mask"] == 1)
        either = (ag["mask"] == 1) | (ao["mask"] == 1)
        dd = np.abs(ag["depth"].astype(np.float64) - ao["depth"])[both]
        drel = dd / np.maximum(ao["depth"][both], 1e-3)
        dc = np.abs(ag["rgb"].astype(np.float64) - ao["rgb"])[both].max(-1)
        step_len = (cm.d_far - cm.d_near) / (cm.n_samples - 1)
        row["anchor_depth_rel"] = _q(drel)
        row["anchor_depth_m"] = _q(dd)
        row["anchor_rgb_abs"] = _q(dc)
        row["anchor_valid_mismatch_frac"] = float((either & ~both).sum() / max(either.sum(), 1))
        row["anchor_hit_moved_frac"] = float((dd > 0.5 * step_len).sum() / max(both.sum(), 1))
        report["frames"].append(row)
        print(json.dumps(row), flush=True)
        assert e_t <= 1e-5 and e_r <= 1e-5, row
        assert e_P <= 1e-4, row
        assert e_b <= 1e-4, row
        assert row["anchor_valid_mismatch_frac"] <= 0.01 and row["anchor_depth_rel"]["p50"] <= 1e-3, row
        del of, ao, ag, mean64, var64
    out_dir = os.environ.get("PRISM_REPORT_DIR") or os.path.join(
        os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "bf16_error_report_15d.json" if bias else "bf16_error_report.json"), "w") as fh:
        json.dump(report, fh, indent=1)
