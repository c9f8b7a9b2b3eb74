"""MI355X-native projector-algorithm Voronoi / Delaunay engine (HIP, gfx950).

The compute path is the C-ABI library ``libvor.so`` (``include/vor.h``); this package is its thin
Python binding (argument marshalling only).  Importing it loads the library and fails loudly if
it has not been built: there is no CPU fallback.
"""
from ._binding import (  # noqa: F401
    VOR_OK, VOR_PENDING, VOR_E_INVAL, VOR_E_DOMAIN, VOR_E_DUPLICATE, VOR_E_NOMEM, VOR_E_DEVICE,
    VOR_E_TICKET, VOR_E_CAPACITY, VOR_SET_DEVICE, VOR_RESULT_DEVICE, VOR_NO_VERTICES,
    VOR_CHECK_SYMMETRY, VOR_TIME_KERNELS, VOR_PATH_GRID_FIRST, VOR_PATH_TREE, VOR_EXACT_ONLY,
    VOR_FP32_FILTERED, VorError, Result, Stats,
    lib, lib_path, vor_create, vor_destroy, vor_compute, vor_compute_batch, vor_submit,
    vor_poll, vor_result_free, vor_result_to_host, vor_strerror, vor_set_tuning, vor_get_tuning,
    vor_set_size_tuning, vor_ticket_times, vor_ticket_count, vor_footprint,
    vor_version, vor_filter_keys, vor_filter_keys_words, vor_region_diag, vor_lloyd,
    vor_peak_fp32, vor_peak_copy, vor_compute_noalloc, VOR_NOALLOC_MAX_SITES,
    Context,
)
