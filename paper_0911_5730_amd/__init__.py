"""Adaptive-multilevel BDDC on MI355X: Python binding of libbddc.so.

The numerical work runs in the HIP library (paper_0911_5730_amd/libbddc.so);
see include/bddc.h for the C ABI.
"""

from .bddc import (  # noqa: F401
    BDDCError,
    Solver,
    load_library,
    plan,
    status_string,
    timing_start,
    timing_stop,
)
