"""MI355X (gfx950) differentiable Monte Carlo polarization ray trace through a
geometric waveguide, with per-hit transfer-matrix thin-film solves
(arXiv 2601.04370, Methods).

The compute path is the HIP library ``libgwg.so`` (C ABI in include/gwg.h);
this package only marshals arguments to it.
"""
from .gwg import (  # noqa: F401
    FP64, FP32_MIXED, FP32, PRECISIONS, Context, GwgError, SceneSpec, load_library,
    make_trace_function, records_view, EXPORTS, LIB_PATH, KERNEL_FORWARD, KERNEL_ADJOINT,
    TIMING_RING, GWG_FWD_GRAD, GWG_FWD_MEMO, GWG_FWD_TABLE, source_hash,
)
