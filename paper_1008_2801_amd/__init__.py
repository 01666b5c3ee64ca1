"""MI355X (gfx950) unsplit PPM hydro step behind the C ABI of include/ppm.h.

Modules:
  ppm     ctypes binding of libppm.so (Level, Graph, hydro_step, params, ...)
  inputs  seeded synthetic layouts and initial states
  build   hipcc build of libppm.so
"""
from . import inputs  # noqa: F401
from .ppm import (BATCHED, PER_BOX, BC_OUTFLOW, BC_PERIODIC, BC_REFLECT, FLAG_FLOOR, FLAG_NONPHYS,  # noqa: F401
                  Graph, Level, PPMError, fill_boundary_host, hydro_step, lib, params, plan_build,
                  plan_cache_stats)
