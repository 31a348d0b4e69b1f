"""MI355X-native list ranking and connected components by pointer jumping.

The compute lives in libptrjump.so (hand-written HIP for gfx950, C ABI in
include/ptrjump.h); this package is its Python binding.
"""

from ._lib import (PJ_EBADLIST, PJ_EINVAL, PJ_ENOCONV, PJ_OK, PjError, load)  # noqa: F401

__all__ = [
    "load",
    "list_rank",
    "list_rank_batched",
    "list_rank_noalloc",
    "list_rank_weighted",
    "list_rank_weighted_batched",
    "connected_components",
    "connected_components_batched",
    "PjError",
]


def __getattr__(name):
    # torch is imported lazily so that loading the C library (e.g. to list its
    # symbols on a machine without a GPU) does not need it
    if name in ("list_rank", "list_rank_batched", "list_rank_noalloc", "list_rank_weighted",
                "list_rank_weighted_batched", "connected_components",
                "connected_components_batched", "make_opts", "tune_list_rank", "tune_lookup",
                "tune_save", "tune_load", "tune_clear", "graph_cache_clear"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
