"""MI355X machine fast Gauss transform (continuous sources on adaptive trees).

The transform runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/fgt.h (libfgt.so); this package is its thin Python binding plus the
seeded synthetic input generator (``synth``).
"""

from .api import (FGT_FP32, FGT_FP64, FGT_FREE, FGT_PERIODIC, FgtError, Plan,  # noqa: F401
                  fgt_destroy, fgt_execute, fgt_periodic_terms, fgt_plan, fgt_plan_array,
                  fgt_plan_info, fgt_pw_terms, fgt_stage_times, fgt_strerror, fgt_sync)
