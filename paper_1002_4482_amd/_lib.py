"""ctypes binding of libptrjump.so (the C ABI of include/ptrjump.h).

Argument marshalling only: every step of every solve runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built; there
is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libptrjump.so")

PJ_OK = 0
PJ_EINVAL = -1
PJ_ENOMEM = -2
PJ_EHIP = -3
PJ_EBADLIST = -4
PJ_ENOCONV = -5
PJ_EBUDGET = -6
PJ_ENOTFOUND = -7
PJ_EBUSY = -8
PJ_ESHUTDOWN = -9
PJ_ESCRATCH = -10

ALGO = {"auto": 0, "wyllie": 1, "ruling_set": 2, "sv": 3}
LEVEL0_STATE = {"auto": 0, "separate": 1}
PJ_MAX_PHASES = 16
PJ_MAX_LEVELS = 8


class PjStats(ctypes.Structure):
    _fields_ = [
        ("algo", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("base_kind", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("level_nodes", ctypes.c_int64 * (PJ_MAX_LEVELS + 1)),
        ("nphases", ctypes.c_int32),
        ("phase_name", (ctypes.c_char * 24) * PJ_MAX_PHASES),
        ("phase_ms", ctypes.c_float * PJ_MAX_PHASES),
        ("status", ctypes.c_int32),
        ("max_sublist0", ctypes.c_int32),
        ("sublists0", ctypes.c_int64),
        ("cuts0", ctypes.c_int64),
    ]

    def to_dict(self):
        return {
            "algo": self.algo,
            "levels": self.levels,
            "base_kind": self.base_kind,
            "rounds": self.rounds,
            "level_nodes": [int(v) for v in self.level_nodes][: max(self.levels + 1, 1)],
            "phases": {self.phase_name[i].value.decode(): float(self.phase_ms[i])
                       for i in range(self.nphases)},
            "phase_list": [(self.phase_name[i].value.decode(), float(self.phase_ms[i]))
                           for i in range(self.nphases)],
            "status": self.status,
            "max_sublist0": self.max_sublist0,
            "sublists0": int(self.sublists0),
            "cuts0": int(self.cuts0),
        }


class PjOpts(ctypes.Structure):
    _fields_ = [
        ("algo", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("spacing", ctypes.c_int32),
        ("spacing_up", ctypes.c_int32),
        ("cutoff", ctypes.c_int32),
        ("max_walk", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("validate", ctypes.c_int32),
        ("to_tail", ctypes.c_int32),
        ("rounds_per_check", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("d_status", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("h_offsets", ctypes.c_void_p),
        ("h_edge_offsets", ctypes.c_void_p),
        ("stats", ctypes.POINTER(PjStats)),
        ("level0_state", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("d_splitters", ctypes.c_void_p),
        ("n_splitters", ctypes.c_int64),
    ]


class PjServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("max_inflight", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("opts", PjOpts),
        ("large_items", ctypes.c_int64),
    ]


class PjServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("ticks", ctypes.c_int64),
        ("inflight_peak", ctypes.c_int64),
        ("budget_waits", ctypes.c_int64),
        ("bytes_peak", ctypes.c_size_t),
        ("bytes_in_use", ctypes.c_size_t),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double),
        ("wall_s", ctypes.c_double),
        ("req_per_s", ctypes.c_double),
        ("items_per_s", ctypes.c_double),
        ("large_ticks", ctypes.c_int64),
    ]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PjError(RuntimeError):
    def __init__(self, code, where=""):
        lib = load()
        msg = lib.pj_strerror(code).decode()
        if code == PJ_EHIP:
            msg += ": " + lib.pj_last_hip_error().decode()
        super().__init__(f"{where}: {msg} ({code})" if where else f"{msg} ({code})")
        self.code = code


_lib = None

# (name, restype, argtypes) of every exported entry point
_VP, _I64, _I32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
SIGNATURES = [
    ("pj_opts_init", None, [_VP]),
    ("pj_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("pj_last_hip_error", ctypes.c_char_p, []),
    ("pj_version", ctypes.c_int, []),
    ("pj_list_rank", ctypes.c_int, [_VP, _I64, _VP, _VP]),
    ("pj_list_rank_ex", ctypes.c_int, [_VP, _I64, _VP, _VP, _VP]),
    ("pj_list_rank_batched", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP]),
    ("pj_list_rank_batched_ex", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP, _VP]),
    ("pj_list_rank_workspace_bytes", _SZ, [_I64, _I64, _VP]),
    ("pj_list_rank_noalloc", ctypes.c_int, [_VP, _I64, _VP, _VP, _VP]),
    ("pj_list_rank_noalloc_max_bytes", _SZ, []),
    ("pj_list_rank_weighted", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP, _VP]),
    ("pj_list_rank_weighted_batched", ctypes.c_int, [_VP, _VP, _VP, _I64, _VP, _VP, _VP]),
    ("pj_list_rank_weighted_workspace_bytes", _SZ, [_I64, _I64, _VP]),
    ("pj_connected_components", ctypes.c_int, [_VP, _VP, _I64, _I64, _VP, _VP]),
    ("pj_connected_components_ex", ctypes.c_int, [_VP, _VP, _I64, _I64, _VP, _VP, _VP]),
    ("pj_connected_components_batched", ctypes.c_int, [_VP, _VP, _VP, _VP, _I64, _VP, _VP]),
    ("pj_connected_components_batched_ex", ctypes.c_int,
     [_VP, _VP, _VP, _VP, _I64, _VP, _VP, _VP]),
    ("pj_cc_workspace_bytes", _SZ, [_I64, _I64, _I64, _VP]),
    ("pj_graph_cache_clear", None, []),
    ("pj_tune_list_rank", ctypes.c_int, [_VP, _VP, _I64, _VP, _I64, _VP, _VP, _VP]),
    ("pj_tune_lookup", ctypes.c_int, [_I64, _I64, _VP]),
    ("pj_tune_save", ctypes.c_int, [ctypes.c_char_p]),
    ("pj_tune_load", ctypes.c_int, [ctypes.c_char_p]),
    ("pj_tune_clear", None, []),
    ("pj_server_create", ctypes.c_int, [_VP, _VP]),
    ("pj_server_submit_list_rank", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP]),
    ("pj_server_submit_cc", ctypes.c_int, [_VP, _VP, _VP, _I64, _I64, _VP, _VP]),
    ("pj_server_poll", ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP]),
    ("pj_server_wait", ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, _I64]),
    ("pj_server_drain", ctypes.c_int, [_VP]),
    ("pj_server_get_stats", ctypes.c_int, [_VP, _VP]),
    ("pj_server_destroy", ctypes.c_int, [_VP]),
]


def load():
    """Load libptrjump.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_names():
    return [name for name, _, _ in SIGNATURES]
