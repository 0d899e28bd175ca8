"""MI355X-native KBC entropic lattice Boltzmann hot path (HIP library + binding).

The compute lives in ``libkbc_lbm.so`` (hand-written HIP for gfx950 behind the
C ABI of ``include/lbm.h``); ``lbm`` is its ctypes binding.
"""
from . import lbm  # noqa: F401
from .lbm import (LBMError, Solver, TorchAllocator, lbm_autotune, lbm_create,  # noqa: F401
                  lbm_destroy, lbm_get_populations, lbm_info, lbm_init_fields, lbm_moments,
                  lbm_set_geometry, lbm_set_launch_mode, lbm_set_populations, lbm_set_stats,
                  lbm_set_variant, lbm_step, lbm_synchronize, lbm_wall_force, make_desc)
