"""Python handle on the C serving loop (pj_server_*): continuous batching of
list-ranking and components requests under an HBM budget.

Inputs and outputs are host arrays (numpy or CPU torch tensors; pinned torch
tensors keep the copies asynchronous).  The server keeps references to them
until the request is collected.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import PjError, PjServerConfig, PjServerStats


def _host_i32(a, name):
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.is_cuda or a.dtype != torch.int32 or not a.is_contiguous() or a.dim() != 1:
                raise TypeError(f"{name}: contiguous 1-D int32 CPU tensor expected")
            return a, a.data_ptr()
    except ImportError:
        pass
    a = np.ascontiguousarray(a, dtype=np.int32)
    if a.ndim != 1:
        raise ValueError(f"{name}: 1-D array expected")
    return a, a.ctypes.data


def _empty_like_host(n, pinned):
    if pinned:
        import torch
        t = torch.empty(n, dtype=torch.int32, pin_memory=True)
        return t, t.data_ptr()
    a = np.empty(n, dtype=np.int32)
    return a, a.ctypes.data


class Server:
    def __init__(self, hbm_budget=16 << 30, max_inflight=3, max_batch=256, device=-1,
                 pinned_outputs=True, large_items=0, **opt_kw):
        from .api import make_opts
        lib = _lib.load()
        cfg = PjServerConfig()
        cfg.hbm_budget = int(hbm_budget)
        cfg.max_inflight = max_inflight
        cfg.max_batch = max_batch
        cfg.device = device
        cfg.large_items = int(large_items)
        cfg.opts = make_opts(**opt_kw)
        self._h = ctypes.c_void_p()
        rc = lib.pj_server_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if rc != _lib.PJ_OK:
            raise PjError(rc, "pj_server_create")
        self._live = {}
        self._pinned = pinned_outputs

    def submit_list_rank(self, succ):
        succ, p = _host_i32(succ, "succ")
        n = len(succ)
        out, po = _empty_like_host(n, self._pinned)
        rid = ctypes.c_uint64()
        rc = _lib.load().pj_server_submit_list_rank(self._h, ctypes.c_void_p(p), n,
                                                   ctypes.c_void_p(po), ctypes.byref(rid))
        if rc != _lib.PJ_OK:
            raise PjError(rc, "pj_server_submit_list_rank")
        self._live[rid.value] = (succ, out)
        return rid.value

    def submit_cc(self, src, dst, n):
        src, ps = _host_i32(src, "src")
        dst, pd = _host_i32(dst, "dst")
        if len(src) != len(dst):
            raise ValueError("src and dst differ in length")
        out, po = _empty_like_host(n, self._pinned)
        rid = ctypes.c_uint64()
        rc = _lib.load().pj_server_submit_cc(self._h, ctypes.c_void_p(ps), ctypes.c_void_p(pd), n,
                                            len(src), ctypes.c_void_p(po), ctypes.byref(rid))
        if rc != _lib.PJ_OK:
            raise PjError(rc, "pj_server_submit_cc")
        self._live[rid.value] = (src, dst, out)
        return rid.value

    def _collect(self, rid, rc, st, lat):
        if rc == _lib.PJ_EBUSY:
            return None
        if rc != _lib.PJ_OK:
            raise PjError(rc, "pj_server_poll")
        held = self._live.pop(rid)
        out = held[-1]
        out = out.numpy() if hasattr(out, "numpy") else out
        return st.value, lat.value, out

    def poll(self, rid):
        """(status, latency_ms, result) once finished, else None."""
        st, lat = ctypes.c_int32(), ctypes.c_double()
        rc = _lib.load().pj_server_poll(self._h, rid, ctypes.byref(st), ctypes.byref(lat))
        return self._collect(rid, rc, st, lat)

    def wait(self, rid, timeout_s=None):
        st, lat = ctypes.c_int32(), ctypes.c_double()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        rc = _lib.load().pj_server_wait(self._h, rid, ctypes.byref(st), ctypes.byref(lat), us)
        return self._collect(rid, rc, st, lat)

    def drain(self):
        _lib.load().pj_server_drain(self._h)

    def stats(self):
        s = PjServerStats()
        _lib.load().pj_server_get_stats(self._h, ctypes.byref(s))
        return s.to_dict()

    def close(self):
        if self._h:
            _lib.load().pj_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
