"""Messenger-field CMB mapmaking on MI355X (Huffenberger & Naess).

The compute path is libmm.so (hand-written HIP kernels for gfx950 behind the C
ABI of include/mm.h); ``paper_1705_01893_amd.mm`` is its ctypes binding.
"""

from . import mm  # noqa: F401
from . import autograd  # noqa: F401
from .mm import (MM_FP64, MM_MIXED, MMError, Plan, mm_apply, mm_cg_solve, mm_chi2, mm_cooling_levels,  # noqa: F401
                 mm_lift_rhs, mm_messenger_iter, mm_plan, mm_plan_hits, mm_plan_nsolvable, mm_plan_solvable,
                 mm_plan_workspace_bytes, mm_plan_binning_stats, mm_solve, mm_status_str, mm_set_timing, mm_get_timing,
                 mm_plan_set_noise, mm_tod_apply, mm_noise_grad)
