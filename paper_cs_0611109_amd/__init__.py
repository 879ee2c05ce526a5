"""Cyclic-group RAID-6 (Z_p-RAID) on AMD Instinct MI355X.

The computation lives in the HIP kernels of ``libraid6c.so`` (C ABI in
``include/raid6c.h``); this package is its thin Python binding, with the
same names, plus a helper that lays stripes out in one device tensor.
"""

from ._lib import (  # noqa: F401
    LIB_PATH,
    RAID6C_JOB_ENCODE,
    RAID6C_JOB_RECOVER,
    RAID6C_ORDER_BY_PRIME,
    RAID6C_ORDER_LARGEST_FIRST,
    RAID6C_ORDER_SUBMITTED,
    raid6c_job,
    raid6c_plan_autotune,
    raid6c_plan_create,
    raid6c_plan_destroy,
    raid6c_plan_get_schedule,
    raid6c_plan_info,
    raid6c_plan_run,
    raid6c_plan_set_schedule,
    raid6c_plan_stats,
    raid6c_run_jobs,
    raid6c_schedule,
    RAID6C_E_ARG,
    RAID6C_E_HIP,
    RAID6C_E_NOMEM,
    RAID6C_E_STATE,
    RAID6C_E_UNSUPPORTED,
    RAID6C_OK,
    Raid6cError,
    load,
    raid6c_autotune_n,
    raid6c_encode,
    raid6c_encode_n,
    raid6c_is_supported_prime,
    raid6c_last_error,
    raid6c_max_prime,
    raid6c_recover_1,
    raid6c_recover_2,
    raid6c_recover_n,
    raid6c_rs_encode_n,
    raid6c_strerror,
    raid6c_tune_clear,
    raid6c_tune_get,
    raid6c_tune_set,
    raid6c_unroll_mask,
    raid6c_vec_mask,
)
from .layout import StripeBatch  # noqa: F401
