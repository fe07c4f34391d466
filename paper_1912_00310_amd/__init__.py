"""MI355X-native stochastic-LLG dynamic-hysteresis engine.

The hot path (Heun integration of the stochastic Landau-Lifshitz-Gilbert
equation on macrospin grids, with the loop reduced every step) runs in the
gfx950 kernels of ``libsllg.so`` behind the C ABI of ``include/sllg.h``;
``sllg`` is its Python binding.
"""
from .sllg import (PLAN_AUTO, PLAN_DEMAG, PLAN_LANES, PLAN_RESIDENT, PLAN_SLAB, PLAN_STREAM, Sim,  # noqa: F401
                   SllgError, lib, loop_area_hc, philox_probe)

__all__ = ["Sim", "SllgError", "lib", "loop_area_hc", "philox_probe", "PLAN_AUTO", "PLAN_RESIDENT", "PLAN_DEMAG",
           "PLAN_STREAM", "PLAN_SLAB", "PLAN_LANES"]
