"""SubApSnap online solve on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libsubap.so`` (include/subap.h),
built from ``csrc/*.hip``; ``binding`` is its ctypes wrapper.  Importing
this package does not load the library; ``binding.load()`` does, and fails
loudly when the library is missing.
"""
from . import binding  # noqa: F401
from .binding import (BF16X3, FP16X3, FP32, FP64, Model, SubapError, subap_lift,  # noqa: F401
                      subap_model_basis, subap_model_dims, subap_model_free, subap_model_rows,
                      subap_offline, subap_profile_enable, subap_profile_read, subap_profile_reset,
                      subap_sketched_residual, subap_solve_batch, subap_plan_create, subap_plan_execute,
                      subap_plan_shape, subap_plan_free, subap_solve_multi)
