"""CPU oracle: the plain definitions of list ranking and connected components.

TEST INFRASTRUCTURE ONLY.  Only the tests, `__graft_entry__.smoke()` and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
imports, links or calls it, and it never imports the GPU library.

The arithmetic lives in `oracle.c` (plain sequential C, built with gcc by
`oracle/build.py`); this module only marshals numpy arrays through ctypes.

  list_rank(succ)          distance from the head, per the list-ranking
                           problem statement (Section 3); tail marked -1 or
                           by a self-loop.
  list_rank_weighted(..)   sum of the weights of the nodes before each node
                           (the weighted splitter list of Section 3.2).
  connected_components(..) smallest vertex id of each component, per the
                           connected-components problem statement (Section 4).
  *_batched                the same per instance of an offset-table batch.

Parity status: pinned (brute force on small inputs, closed forms of the
generators, complete invariants and a library cross-check; see tests/).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, EBADLIST = 0, -1, -2, -4


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_list_rank.argtypes = [i32p, ctypes.c_int64, i32p]
    lib.oracle_list_rank.restype = ctypes.c_int
    lib.oracle_list_rank_weighted.argtypes = [i32p, i32p, ctypes.c_int64, i32p]
    lib.oracle_list_rank_weighted.restype = ctypes.c_int
    lib.oracle_cc.argtypes = [i32p, i32p, ctypes.c_int64, ctypes.c_int64, i32p]
    lib.oracle_cc.restype = ctypes.c_int
    lib.oracle_list_rank_batched.argtypes = [i32p, i64p, ctypes.c_int64, i32p, i32p, ctypes.c_int]
    lib.oracle_list_rank_batched.restype = ctypes.c_int
    lib.oracle_cc_batched.argtypes = [i32p, i32p, i64p, i64p, ctypes.c_int64, i32p, i32p,
                                      ctypes.c_int]
    lib.oracle_cc_batched.restype = ctypes.c_int
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def list_rank_status(succ):
    """(status, rank) for one list; rank is int32[n], distance from the head."""
    succ = _i32(succ)
    rank = np.full(succ.shape[0], -1, dtype=np.int32)
    rc = _load().oracle_list_rank(_p32(succ), succ.shape[0], _p32(rank))
    return rc, rank


def list_rank(succ):
    rc, rank = list_rank_status(succ)
    if rc != OK:
        raise OracleError(rc)
    return rank


def list_rank_weighted(succ, weight):
    """rank[x] = sum of the weights of the nodes before x (int32, wrapping)."""
    succ, weight = _i32(succ), _i32(weight)
    if succ.shape != weight.shape:
        raise ValueError("succ and weight differ in length")
    rank = np.full(succ.shape[0], -1, dtype=np.int32)
    rc = _load().oracle_list_rank_weighted(_p32(succ), _p32(weight), succ.shape[0], _p32(rank))
    if rc != OK:
        raise OracleError(rc)
    return rank


def connected_components(src, dst, n):
    src, dst = _i32(src), _i32(dst)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    label = np.empty(n, dtype=np.int32)
    rc = _load().oracle_cc(_p32(src), _p32(dst), n, src.shape[0], _p32(label))
    if rc != OK:
        raise OracleError(rc)
    return label


def list_rank_batched(succ, offsets, nthreads=None):
    """(status int32[L], rank int32[total]) with local ranks per list."""
    succ = _i32(succ)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    L = offsets.shape[0] - 1
    rank = np.full(succ.shape[0], -1, dtype=np.int32)
    status = np.zeros(max(L, 0), dtype=np.int32)
    nt = nthreads or os.cpu_count() or 1
    rc = _load().oracle_list_rank_batched(_p32(succ), _p64(offsets), L, _p32(rank), _p32(status), nt)
    if rc == EINVAL:
        raise OracleError(rc)
    return status, rank


def connected_components_batched(src, dst, vtx_off, edge_off, nthreads=None):
    src, dst = _i32(src), _i32(dst)
    vtx_off = np.ascontiguousarray(vtx_off, dtype=np.int64)
    edge_off = np.ascontiguousarray(edge_off, dtype=np.int64)
    G = vtx_off.shape[0] - 1
    label = np.full(int(vtx_off[-1]) if G >= 0 else 0, -1, dtype=np.int32)
    status = np.zeros(max(G, 0), dtype=np.int32)
    nt = nthreads or os.cpu_count() or 1
    rc = _load().oracle_cc_batched(_p32(src), _p32(dst), _p64(vtx_off), _p64(edge_off), G,
                                   _p32(label), _p32(status), nt)
    if rc != OK:
        raise OracleError(rc)
    return label
