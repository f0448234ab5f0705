"""MI355X machine fast Gauss transform (continuous sources on adaptive trees).

The transform runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/fgt.h, include/fgt_serve.h, include/fgt_batch.h, include/fgt_output.h and
include/fgt_density.h (libfgt.so); this package is its thin Python binding plus the
seeded synthetic input generator (``synth``).
"""

from .api import (FGT_FP32, FGT_FP64, FGT_FREE, FGT_PERIODIC, Batch, FgtError, OutputTree, Plan,  # noqa: F401
                  Server, fgt_batch_bind, fgt_batch_create, fgt_batch_destroy, fgt_batch_execute,
                  fgt_batch_info, fgt_batch_tune, fgt_destroy, fgt_execute, fgt_periodic_terms, fgt_plan,
                  fgt_plan_array, fgt_plan_info, fgt_pw_terms, fgt_server_create,
                  fgt_server_destroy, fgt_server_drain, fgt_server_poll, fgt_server_stats,
                  fgt_server_submit, fgt_server_wait, fgt_stage_times, fgt_strerror, fgt_sync,
                  fgt_interp, fgt_output_destroy, fgt_output_info, fgt_output_resolve, fgt_output_tree,
                  fgt_output_values, fgt_tree_balance, interp, resolve_gaussians, sample_gaussians)
