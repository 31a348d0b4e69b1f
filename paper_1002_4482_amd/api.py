"""Torch-facing wrappers over the C ABI.

torch supplies device memory and the current HIP stream; these functions only
check shapes and dtypes, build a pj_opts struct and pass raw pointers.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import ALGO, LEVEL0_STATE, PjError, PjOpts, PjStats


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_i32(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda:
        raise TypeError(f"{name} must be an int32 CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _dev_i64(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_cuda:
        raise TypeError(f"{name} must be an int64 CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _host_i64(a, length, name):
    """Host int64 table of exactly `length` entries (None passes through)."""
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.int64)
    if a.ndim != 1 or a.shape[0] != length:
        raise ValueError(f"{name} must hold {length} int64 entries")
    return a


def _need(t, count, name):
    if t.numel() < count:
        raise ValueError(f"{name} holds {t.numel()} elements, {count} needed")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def make_opts(algo="auto", block=0, spacing=0, spacing_up=0, cutoff=0, max_walk=0, seed=None,
              validate=False, to_tail=False, rounds_per_check=0, use_graph=False, status=None,
              workspace=None, h_offsets=None, h_edge_offsets=None, stats=None,
              level0_state="auto", splitters=None):
    """Build a pj_opts.  Host arrays (h_offsets...) and the device `splitters`
    tensor must stay alive for the call."""
    o = PjOpts()
    _lib.load().pj_opts_init(ctypes.byref(o))
    o.algo = ALGO[algo] if isinstance(algo, str) else int(algo)
    o.block = block
    o.spacing = spacing
    o.spacing_up = spacing_up
    o.cutoff = cutoff
    o.max_walk = max_walk
    if seed is not None:
        o.seed = seed
    o.validate = int(bool(validate))
    o.to_tail = int(bool(to_tail))
    o.rounds_per_check = rounds_per_check
    o.use_graph = int(bool(use_graph))
    if status is not None:
        o.d_status = _dev_i32(status, "status").data_ptr()
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if h_offsets is not None:
        o.h_offsets = h_offsets.ctypes.data
    if h_edge_offsets is not None:
        o.h_edge_offsets = h_edge_offsets.ctypes.data
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    o.level0_state = (LEVEL0_STATE[level0_state] if isinstance(level0_state, str)
                      else int(level0_state))
    if splitters is not None:
        splitters = _dev_i32(splitters, "splitters")
        o.d_splitters = splitters.data_ptr() if splitters.numel() else None
        o.n_splitters = splitters.numel()
    return o


def _check(rc, where):
    if rc != _lib.PJ_OK:
        raise PjError(rc, where)


def list_rank(succ, rank=None, *, stream=None, return_stats=False, **kw):
    """Rank one list: rank[i] = distance of node i from the head (or to the
    tail with to_tail=True).  `succ` is int32 on the device, tail -1 or self."""
    succ = _dev_i32(succ, "succ")
    n = succ.numel()
    if rank is None:
        rank = torch.empty_like(succ)
    _dev_i32(rank, "rank")
    _need(rank, n, "rank")
    st = PjStats() if return_stats else None
    o = make_opts(stats=st, **kw)
    rc = _lib.load().pj_list_rank_ex(_ptr(succ), n, _ptr(rank), ctypes.byref(o), _stream_ptr(stream))
    _check(rc, "pj_list_rank")
    return (rank, st.to_dict()) if return_stats else rank


def list_rank_noalloc(succ, rank=None, *, stream=None, **kw):
    """pj_list_rank_noalloc: the same ranks as list_rank, with the workspace
    taken from the library's fixed device scratch (no device allocation in
    the call; `rank` is allocated here by torch when not given)."""
    succ = _dev_i32(succ, "succ")
    n = succ.numel()
    if rank is None:
        rank = torch.empty_like(succ)
    _dev_i32(rank, "rank")
    _need(rank, n, "rank")
    o = make_opts(**kw)
    rc = _lib.load().pj_list_rank_noalloc(_ptr(succ), n, _ptr(rank), ctypes.byref(o),
                                          _stream_ptr(stream))
    _check(rc, "pj_list_rank_noalloc")
    return rank


def list_rank_noalloc_max_bytes():
    return int(_lib.load().pj_list_rank_noalloc_max_bytes())


def list_rank_batched(succ, offsets, rank=None, *, h_offsets=None, stream=None,
                      return_stats=False, **kw):
    """Rank L lists concatenated in `succ` (local ids) with device int64
    offsets[L+1]; `h_offsets` (numpy int64) avoids a device-to-host read."""
    succ = _dev_i32(succ, "succ")
    offsets = _dev_i64(offsets, "offsets")
    L = offsets.numel() - 1
    if rank is None:
        rank = torch.empty_like(succ)
    _dev_i32(rank, "rank")
    _need(rank, succ.numel(), "rank")
    h_offsets = _host_i64(h_offsets, L + 1, "h_offsets")
    if h_offsets is not None and h_offsets[-1] > succ.numel():
        raise ValueError("offsets exceed succ")
    st = PjStats() if return_stats else None
    o = make_opts(stats=st, h_offsets=h_offsets, **kw)
    rc = _lib.load().pj_list_rank_batched_ex(_ptr(succ), _ptr(offsets), L, _ptr(rank),
                                             ctypes.byref(o), _stream_ptr(stream))
    _check(rc, "pj_list_rank_batched")
    return (rank, st.to_dict()) if return_stats else rank


def list_rank_weighted(succ, weight, rank=None, *, stream=None, return_stats=False, **kw):
    """Weighted ranks of one list: rank[i] = sum of the weights of the nodes
    before i (int32 on the device, `weight` beside `succ`)."""
    succ = _dev_i32(succ, "succ")
    weight = _dev_i32(weight, "weight")
    n = succ.numel()
    _need(weight, n, "weight")
    if rank is None:
        rank = torch.empty_like(succ)
    _dev_i32(rank, "rank")
    _need(rank, n, "rank")
    st = PjStats() if return_stats else None
    o = make_opts(stats=st, **kw)
    rc = _lib.load().pj_list_rank_weighted(_ptr(succ), _ptr(weight), n, _ptr(rank),
                                           ctypes.byref(o), _stream_ptr(stream))
    _check(rc, "pj_list_rank_weighted")
    return (rank, st.to_dict()) if return_stats else rank


def list_rank_weighted_batched(succ, weight, offsets, rank=None, *, h_offsets=None, stream=None,
                               return_stats=False, **kw):
    """Weighted ranks of L concatenated lists (local ids, device int64
    offsets[L+1], `weight` laid out like `succ`)."""
    succ = _dev_i32(succ, "succ")
    weight = _dev_i32(weight, "weight")
    _need(weight, succ.numel(), "weight")
    offsets = _dev_i64(offsets, "offsets")
    L = offsets.numel() - 1
    if rank is None:
        rank = torch.empty_like(succ)
    _dev_i32(rank, "rank")
    _need(rank, succ.numel(), "rank")
    h_offsets = _host_i64(h_offsets, L + 1, "h_offsets")
    if h_offsets is not None and h_offsets[-1] > succ.numel():
        raise ValueError("offsets exceed succ")
    st = PjStats() if return_stats else None
    o = make_opts(stats=st, h_offsets=h_offsets, **kw)
    rc = _lib.load().pj_list_rank_weighted_batched(_ptr(succ), _ptr(weight), _ptr(offsets), L,
                                                   _ptr(rank), ctypes.byref(o),
                                                   _stream_ptr(stream))
    _check(rc, "pj_list_rank_weighted_batched")
    return (rank, st.to_dict()) if return_stats else rank


def connected_components(src, dst, n, label=None, *, stream=None, return_stats=False, **kw):
    """label[v] = smallest vertex id in v's component (device int32 pairs)."""
    src = _dev_i32(src, "src")
    dst = _dev_i32(dst, "dst")
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    if label is None:
        label = torch.empty(n, dtype=torch.int32, device=src.device)
    _dev_i32(label, "label")
    if label.numel() < n:
        raise ValueError("label too short")
    st = PjStats() if return_stats else None
    o = make_opts(stats=st, **kw)
    rc = _lib.load().pj_connected_components_ex(_ptr(src), _ptr(dst), n, src.numel(), _ptr(label),
                                                ctypes.byref(o), _stream_ptr(stream))
    _check(rc, "pj_connected_components")
    return (label, st.to_dict()) if return_stats else label


def connected_components_batched(src, dst, vtx_off, edge_off, label=None, *, h_vtx_off=None,
                                 h_edge_off=None, stream=None, return_stats=False, **kw):
    src = _dev_i32(src, "src")
    dst = _dev_i32(dst, "dst")
    vtx_off = _dev_i64(vtx_off, "vtx_off")
    edge_off = _dev_i64(edge_off, "edge_off")
    G = vtx_off.numel() - 1
    if edge_off.numel() != G + 1:
        raise ValueError("vtx_off and edge_off differ in length")
    h_vtx_off = _host_i64(h_vtx_off, G + 1, "h_vtx_off")
    h_edge_off = _host_i64(h_edge_off, G + 1, "h_edge_off")
    total = int(h_vtx_off[-1]) if h_vtx_off is not None else int(vtx_off[-1].item())
    if label is None:
        label = torch.empty(total, dtype=torch.int32, device=src.device)
    _dev_i32(label, "label")
    _need(label, total, "label")
    if h_edge_off is not None and h_edge_off[-1] > src.numel():
        raise ValueError("edge offsets exceed the pair arrays")
    st = PjStats() if return_stats else None
    o = make_opts(stats=st, h_offsets=h_vtx_off, h_edge_offsets=h_edge_off, **kw)
    rc = _lib.load().pj_connected_components_batched_ex(
        _ptr(src), _ptr(dst), _ptr(vtx_off), _ptr(edge_off), G, _ptr(label), ctypes.byref(o),
        _stream_ptr(stream))
    _check(rc, "pj_connected_components_batched")
    return (label, st.to_dict()) if return_stats else label


def tune_list_rank(succ, offsets=None, *, h_offsets=None, stream=None):
    """Autotune the ruling-set parameters on this input (single list when
    `offsets` is None).  Returns (best parameters dict, mean ms)."""
    succ = _dev_i32(succ, "succ")
    best = PjOpts()
    ms = ctypes.c_float(0.0)
    lib = _lib.load()
    if offsets is None:
        rc = lib.pj_tune_list_rank(_ptr(succ), None, 1, None, succ.numel(), ctypes.byref(best),
                                   ctypes.byref(ms), _stream_ptr(stream))
    else:
        offsets = _dev_i64(offsets, "offsets")
        if h_offsets is None:
            h_offsets = offsets.cpu().numpy()
        h_offsets = _host_i64(h_offsets, offsets.numel(), "h_offsets")
        if h_offsets[-1] > succ.numel():
            raise ValueError("offsets exceed succ")
        rc = lib.pj_tune_list_rank(_ptr(succ), _ptr(offsets), offsets.numel() - 1,
                                   ctypes.c_void_p(h_offsets.ctypes.data), 0, ctypes.byref(best),
                                   ctypes.byref(ms), _stream_ptr(stream))
    _check(rc, "pj_tune_list_rank")
    return ({"spacing": best.spacing, "spacing_up": best.spacing_up, "cutoff": best.cutoff,
             "max_walk": best.max_walk, "block": best.block}, float(ms.value))


def tune_lookup(n, L=1):
    o = PjOpts()
    rc = _lib.load().pj_tune_lookup(n, L, ctypes.byref(o))
    if rc != _lib.PJ_OK:
        return None
    return {"spacing": o.spacing, "spacing_up": o.spacing_up, "cutoff": o.cutoff,
            "max_walk": o.max_walk, "block": o.block}


def tune_save(path):
    _check(_lib.load().pj_tune_save(str(path).encode()), "pj_tune_save")


def tune_load(path):
    _check(_lib.load().pj_tune_load(str(path).encode()), "pj_tune_load")


def tune_clear():
    _lib.load().pj_tune_clear()


def graph_cache_clear():
    _lib.load().pj_graph_cache_clear()
