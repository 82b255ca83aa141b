"""MI355X (gfx950) implementation of the accelerated shiftable O(1) Gaussian
bilateral filter: Algorithm 2 of Chaudhury's paper behind the C ABI of
include/bf.h (libbf.so), with a thin ctypes binding.
"""
from .bf import (  # noqa: F401
    BFError,
    Plan,
    bf_dynamic_range,
    bf_filter,
    bf_filter_batch,
    bf_last_error_detail,
    bf_plan,
    bf_plan_destroy,
    bf_profile,
    bf_profile_read,
    bf_status_string,
    bilateral_filter,
    make_params,
)
