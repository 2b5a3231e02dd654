"""Cluster-preserving correction of lossy-compressed particle data on MI355X.

The whole correction pass runs in the gfx950 library ``libpcc.so`` behind the
C ABI of ``include/pcc.h``; this package is its ctypes binding.
"""
from ._binding import (  # noqa: F401
    Context, PccError, Server, decode, lib, make_params, version, LIB_PATH, MODES, STAGE_NAMES,
    inject_alloc_failure, alloc_failure_countdown, fof_labels_noalloc_max_n, noalloc_high_water,
)
