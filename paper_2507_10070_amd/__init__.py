"""MI355X (gfx950) search hot path of FlashANNS (arXiv 2507.10070).

The compute path is the HIP library ``libflashann.so`` (C ABI declared in
``include/flashann.h``); this package is a thin ctypes binding around it.
Importing the package does not load the library; the first call does, and it
raises if the library has not been built.
"""
from .flashann import (ANN_ERRORS, AnnError, Index, SearchGraph, SearchOptions,  # noqa: F401
                       Server, clock_us, load_library, search, search_noalloc,
                       build_index, save_index, save_records_striped, device_clock_khz, DTYPE_CODES, TIER_HBM,
                       TIER_HOST, TIER_FILE, TRANSPORT_AUTO, TRANSPORT_DIRECT, TRANSPORT_AGENT,
                       SYNC_QUERY, SYNC_KERNEL, NAV_FULL, NAV_PQ, PQ_DROP_NAV, PQ_AUTO, PQ_TABLE,
                       PQ_CACHE)
