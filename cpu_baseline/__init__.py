"""Multi-threaded CPU list ranking by random splitters (ruling_set.c): the
host-core comparison point for the GPU path, as Section 3.2 compares its GPU
ranking with a multi-core CPU.  Timed by the benchmark; not a parity
reference (the tests pin it against the oracle's ranks).

  ruling_set(succ, spacing, nthreads) -> (status, rank)
      status 0, or -4 for input that is not one list; rank int32[n] from the
      head (tail -1 or a self-loop).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcpurs.so")
_lib = None

OK, EINVAL, ENOMEM, EBADLIST = 0, -1, -2, -4


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.cpu_ruling_set_list_rank.argtypes = [i32p, ctypes.c_int64, i32p, ctypes.c_int, ctypes.c_int]
    lib.cpu_ruling_set_list_rank.restype = ctypes.c_int
    _lib = lib
    return lib


def ruling_set(succ, spacing=64, nthreads=None):
    succ = np.ascontiguousarray(succ, dtype=np.int32)
    rank = np.full(succ.shape[0], -1, dtype=np.int32)
    nt = nthreads or min(16, os.cpu_count() or 1)
    p = ctypes.POINTER(ctypes.c_int32)
    rc = _load().cpu_ruling_set_list_rank(succ.ctypes.data_as(p), succ.shape[0],
                                          rank.ctypes.data_as(p), spacing, nt)
    return rc, rank
