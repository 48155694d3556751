"""spotdd: MI355X-native brute-force dedispersion + boxcar single-pulse search.

The compute lives in libspotdd.so (HIP for gfx950, C ABI in include/spotdd.h);
this package is its Python binding."""
from ._capi import SddError, header_functions, lib  # noqa: F401
from .spotdd import (BEST_DTYPE, CAND_DTYPE, FFA_BEST_DTYPE, STATS_DTYPE, Batch,  # noqa: F401
                     FfaOut, Plan, SearchOut, Server, SiftOut, Stream, ffa_search,
                     plane_host, tile_menu)

__all__ = ["Plan", "Batch", "Server", "Stream", "SearchOut", "SiftOut", "SddError", "tile_menu",
           "plane_host", "lib", "header_functions", "CAND_DTYPE", "BEST_DTYPE", "STATS_DTYPE",
           "ffa_search", "FfaOut", "FFA_BEST_DTYPE"]
