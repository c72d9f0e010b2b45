"""Oracle defaults against the hyper-parameters printed in App. G."""
import json
import os

GOLD = os.path.join(os.path.dirname(__file__), "golden", "app_g_hyperparameters.json")


def test_oracle_defaults_match_app_g(orc):
    g = json.load(open(GOLD))
    p = orc.Params()
    ts = g["transition_scales"]
    assert (p.sigma_vel_t, p.sigma_pose_t) == (ts["translation_sigma_vel"], ts["translation_sigma_pose"])
    assert (p.sigma_vel_r, p.sigma_pose_r) == (ts["rotation_sigma_vel"], ts["rotation_sigma_pose"])
    mu = g["map_updates"]
    assert p.trunc_voxels == mu["truncation_voxels_blackbird"]
    assert p.sigma_update == mu["sigma_update"]
    grid = orc.Grid(8, 0.1)
    assert (grid.occ_out, grid.rgb_out) == (mu["initial_occupancy"], mu["initial_colour"])
    po = g["pose_optimisation"]
    assert (p.gate_geo, p.gate_rgb) == (po["geometric_gate"], po["photometric_gate"])
    assert (p.b_rgb, p.b_geo) == (po["laplace_scale_colour_euroc_tum"], po["laplace_scale_geometric_euroc_tum"])
    assert p.ema == g["laplace_approximation"]["ema_coefficient"]
    assert orc.Cam(1, 1, 1, 1, 0, 0, 0.1, 1, 2).tau == g["rendering"]["tau"]
