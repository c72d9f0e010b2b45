"""MI355X-native PRISM filter hot path (Mirchev et al., CoRL 2022).

The compute lives in ``libprism.so`` (hand-written HIP for gfx950, C ABI in
``include/prism.h``); ``prism`` is its ctypes binding, ``autograd`` wraps the
renderer's adjoint for PyTorch and ``serving`` runs many agent streams.
"""
from . import prism  # noqa: F401
from .prism import (  # noqa: F401
    Camera, Filter, FilterParams, Grid, VoxelMap, Weights, filter_step, filter_step_graph, map_update, render,
    render_jacobian,
    render_vjp, track_p2, PRISM_BF16, PRISM_F32, OBJ_P1, OBJ_P2,
)
