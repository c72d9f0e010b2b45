"""The C-ABI library loads on the CPU host, exports every entry point that
include/prism.h declares, its struct mirrors match, and host-side argument
validation rejects bad input (no GPU needed: validation runs before any HIP
call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "prism.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prism_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def P():
    from paper_2212_02988_amd import prism
    return prism


def test_every_declared_symbol_is_exported(P):
    L = P.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_struct_mirrors(P):
    L = P.lib()
    for name, cls in [("prism_grid", P.Grid), ("prism_camera", P.Camera), ("prism_pose", P.Pose),
                      ("prism_weights", P.Weights), ("prism_map_params", P.MapParams),
                      ("prism_filter_cfg", P.FilterCfg), ("prism_filter_state", P.FilterState),
                      ("prism_filter_bias_state", P.BiasState),
                      ("prism_frame", P.Frame), ("prism_adam_params", P.AdamParams)]:
        assert L.prism_sizeof(name.encode()) == ctypes.sizeof(cls), name
    assert L.prism_sizeof(b"nope") == 0


def test_map_bytes_and_validation(P):
    L = P.lib()
    b = ctypes.c_size_t()
    g = P.Grid.make(64, 0.04)
    assert L.prism_map_bytes(ctypes.byref(g), ctypes.byref(b)) == 0
    nb3 = (64 // 8) ** 3
    r256 = lambda x: (x + 255) // 256 * 256
    nseg = (nb3 + 255) // 256
    # summary, free-space bits (plain and dilated), counts, brick list, segment lengths, pose scratch
    aux = r256(4 * nb3) + r256(8 * ((nb3 + 31) // 32)) + r256(4 * 2048) + r256(4 * nseg * 256) + r256(4 * nseg) + 256
    assert b.value == 8 * 64 ** 3 * 4 + aux
    g = P.Grid.make(64, 0.04, dtype=P.PRISM_BF16)
    assert L.prism_map_bytes(ctypes.byref(g), ctypes.byref(b)) == 0
    assert b.value == 8 * 64 ** 3 * 2 + aux
    for bad in (P.Grid.make(60, 0.04), P.Grid.make(64, 0.04, dtype=7), P.Grid.make(2048, 0.01)):
        assert L.prism_map_bytes(ctypes.byref(bad), ctypes.byref(b)) == 2
        assert b"unsupported" in L.prism_last_error()
    assert L.prism_map_bytes(ctypes.byref(P.Grid.make(64, -1.0)), ctypes.byref(b)) == 1
    assert L.prism_map_bytes(None, ctypes.byref(b)) == 1


def test_render_rejects_bad_arguments(P):
    L = P.lib()
    g = P.Grid.make(64, 0.04)
    cam = P.Camera.make(80, 60, 60, 60, 40, 30, 0.1, 3.0, 32)
    # NULL map
    st = L.prism_render(ctypes.byref(g), None, ctypes.byref(cam), ctypes.c_void_p(256), 1, ctypes.c_void_p(256),
                        ctypes.c_void_p(256), ctypes.c_void_p(256), None, None, None, 0.1, None)
    assert st == 1 and b"map" in L.prism_last_error()
    bad = P.Camera.make(80, 60, 60, 60, 40, 30, 3.0, 0.1, 32)     # d_far < d_near
    st = L.prism_render(ctypes.byref(g), ctypes.c_void_p(256), ctypes.byref(bad), ctypes.c_void_p(256), 1,
                        ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256), None, None, None, 0.1,
                        None)
    assert st == 1
    one = P.Camera.make(80, 60, 60, 60, 40, 30, 0.1, 3.0, 1)       # K < 2
    st = L.prism_render(ctypes.byref(g), ctypes.c_void_p(256), ctypes.byref(one), ctypes.c_void_p(256), 1,
                        ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256), None, None, None, 0.1,
                        None)
    assert st == 2
    # misaligned map
    st = L.prism_render(ctypes.byref(g), ctypes.c_void_p(260), ctypes.byref(cam), ctypes.c_void_p(256), 1,
                        ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256), None, None, None, 0.1,
                        None)
    assert st == 1 and b"aligned" in L.prism_last_error()


def test_workspace_and_filter_sizes(P):
    L = P.lib()
    cam = P.Camera.make(320, 240, 240, 240, 160, 120, 0.1, 7.5, 128)
    b = ctypes.c_size_t()
    assert L.prism_reduce_workspace_bytes(ctypes.byref(cam), 2, ctypes.byref(b)) == 0
    assert b.value == 2 * (40 * 30) * 29 * 8      # 8x8-pixel workgroups of the render Jacobian
    cfg = P.filter_cfg(P.Grid.make(256, 0.025), cam, P.FilterParams())
    assert L.prism_filter_bytes(ctypes.byref(cfg), ctypes.byref(b)) == 0
    assert b.value >= 30 * 320 * 240
    bad = P.filter_cfg(P.Grid.make(256, 0.025), cam, P.FilterParams(n_gn=100))
    assert L.prism_filter_bytes(ctypes.byref(bad), ctypes.byref(b)) == 1


def test_paper_modes_are_validated(P):
    """cfg.modes takes the four documented bits in any combination; the L1
    mode needs a positive floor, the 15-D state a finite bias walk and
    gravity; unknown bits are refused."""
    L = P.lib()
    cam = P.Camera.make(64, 48, 50, 50, 32, 24, 0.1, 4.0, 64)
    g = P.Grid.make(64, 0.04)
    b = ctypes.c_size_t()
    for modes in range(16):
        cfg = P.filter_cfg(g, cam, P.FilterParams(modes=modes))
        assert L.prism_filter_bytes(ctypes.byref(cfg), ctypes.byref(b)) == 0, modes
    for bad in (P.FilterParams(modes=16), P.FilterParams(modes=P.MODE_IRLS_L1, irls_floor=0.0),
                P.FilterParams(modes=P.MODE_IRLS_L1, irls_floor=float("nan")),
                P.FilterParams(modes=P.MODE_ACCEL_BIAS, sigma_bias=-1.0),
                P.FilterParams(modes=P.MODE_ACCEL_BIAS, gravity=(0.0, 0.0, float("inf")))):
        cfg = P.filter_cfg(g, cam, bad)
        assert L.prism_filter_bytes(ctypes.byref(cfg), ctypes.byref(b)) == 1
        assert any(k in L.prism_last_error() for k in (b"modes", b"irls_floor", b"sigma_bias"))
    # the floor is not read without the L1 mode
    cfg = P.filter_cfg(g, cam, P.FilterParams(modes=P.MODE_LAPLACE_FACTOR1, irls_floor=0.0))
    assert L.prism_filter_bytes(ctypes.byref(cfg), ctypes.byref(b)) == 0


def test_paper_sampling_camera_matches_the_oracle(P):
    """prism_camera_paper_sampling gives the oracle's camera for the paper's
    sampling (offsets eps, 2 eps, ... up to the maximum depth, eps = 0.4
    voxel) bit for bit; counts outside 2..4096 and bad arguments are refused
    and leave the camera unchanged."""
    import oracle as orc
    L = P.lib()
    for voxel, dmax in ((0.025, 8.0), (0.05, 7.0), (0.1, 20.0), (0.0125, 8.0), (0.03, 0.025),
                        (0.001, 8.0), (0.1, 0.05)):
        ref = orc.paper_sample_camera(64, 48, 50.0, 50.0, 32.0, 24.0, voxel, dmax)
        cam = P.Camera.make(64, 48, 50, 50, 32, 24, 0.1, 4.0, 64)
        st = L.prism_camera_paper_sampling(ctypes.byref(cam), voxel, dmax)
        if not 2 <= ref.n_samples <= 4096:
            assert st == 2 and cam.n_samples == 64 and cam.d_near == 0.1 and cam.d_far == 4.0
            continue
        assert st == 0
        assert (cam.d_near, cam.d_far, cam.n_samples) == (ref.d_near, ref.d_far, ref.n_samples)
        assert (cam.width, cam.fx, cam.tau) == (64, 50.0, 0.0)
    cam = P.Camera.make(64, 48, 50, 50, 32, 24, 0.1, 4.0, 64)
    for voxel, dmax in ((0.0, 8.0), (-1.0, 8.0), (0.05, float("inf")), (0.05, 0.0)):
        assert L.prism_camera_paper_sampling(ctypes.byref(cam), voxel, dmax) == 1
    assert L.prism_camera_paper_sampling(None, 0.05, 8.0) == 1


def test_brick_pool_map_bytes_and_init_checks(P):
    """Brick-pool maps: size = pool planes + the dense summaries + the slot
    table and pool header; capacity bounded by the brick count; init must use
    the outside values (validation only, no device call)."""
    L = P.lib()
    b = ctypes.c_size_t()
    r256 = lambda x: (x + 255) // 256 * 256
    dense = P.Grid.make(64, 0.04)
    assert L.prism_map_bytes(ctypes.byref(dense), ctypes.byref(b)) == 0
    dense_bytes = b.value
    nb3 = 8 ** 3
    for cap in (1, 37, nb3):
        g = P.Grid.make(64, 0.04, capacity=cap)
        assert L.prism_map_bytes(ctypes.byref(g), ctypes.byref(b)) == 0
        assert b.value == dense_bytes - 8 * 64 ** 3 * 4 + r256(8 * cap * 512 * 4) + r256(4 * nb3) + 256
    for bad in (-1, nb3 + 1):
        g = P.Grid.make(64, 0.04, capacity=bad)
        assert L.prism_map_bytes(ctypes.byref(g), ctypes.byref(b)) == 1
        assert b"capacity" in L.prism_last_error()
    g = P.Grid.make(64, 0.04, capacity=10)
    st = L.prism_map_init(ctypes.byref(g), ctypes.c_void_p(256), 0.5, 0.0, 1e4, None)
    assert st == 1 and b"occ_out" in L.prism_last_error()
    st = L.prism_map_from_dense(ctypes.byref(g), ctypes.c_void_p(256), None, None, None)
    assert st == 2
    st = L.prism_map_pool_usage(ctypes.byref(dense), ctypes.c_void_p(256), ctypes.c_void_p(256), None)
    assert st == 2
