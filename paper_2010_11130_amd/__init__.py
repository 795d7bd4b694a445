"""airhdg: space-time HDG + lAIR-preconditioned FGMRES on one MI355X.

The compute path is the HIP library ``libairhdg.so`` (C-ABI in
``include/airhdg.h``); this package only marshals arguments.
"""
from .api import (Mesh, System, Hierarchy, AIRSolve, HDGSolve, GaussSource, sizes, quad_rule,
                  source_gauss, source_gauss_T, air_params, solve_params, use_torch_allocator,
                  pool_trim)
from ._lib import lib, AirHdgError, LIB_PATH
from .march import SlabMarch

__all__ = ["Mesh", "System", "Hierarchy", "AIRSolve", "HDGSolve", "GaussSource", "sizes", "quad_rule",
           "source_gauss", "source_gauss_T", "air_params", "solve_params", "use_torch_allocator", "pool_trim", "lib",
           "AirHdgError", "LIB_PATH", "SlabMarch"]
