"""The C ABI: the built library loads without a GPU and exports every entry
point include/ptrjump.h declares; the Python binding knows them all; the
header's struct layouts match the binding's ctypes mirrors."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ptrjump.h")
LIB = os.path.join(ROOT, "paper_1002_4482_amd", "libptrjump.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pj_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libptrjump.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pj_list_rank", "pj_connected_components", "pj_list_rank_batched",
                 "pj_connected_components_batched", "pj_strerror"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1002_4482_amd import _lib
    assert set(_lib.exported_names()) == set(declared_functions())


def test_exports_are_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in declared_functions():
        assert n in syms, f"{n} is not an unmangled export"


def test_host_only_calls(lib):
    from paper_1002_4482_amd import _lib
    L = _lib.load()
    assert L.pj_strerror(0) == b"ok"
    assert L.pj_strerror(-4).startswith(b"input is not")
    assert L.pj_version() >= 10000
    o = _lib.PjOpts()
    L.pj_opts_init(ctypes.byref(o))
    assert o.algo == 0 and o.seed != 0
    # workspace sizing is host arithmetic
    plain = L.pj_list_rank_workspace_bytes(1 << 20, 1, None)
    assert 0 < plain < 64 * (1 << 20)
    o.validate = 1
    assert L.pj_list_rank_workspace_bytes(1 << 20, 1, ctypes.byref(o)) >= plain + 4 * (1 << 20)
    assert L.pj_cc_workspace_bytes(1 << 20, 1 << 22, 1, None) >= 8 * (1 << 20)


def _c_sizeof(struct, field=None):
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"ptrjump.h\"\n"
           f"int main(void){{printf(\"%zu\", {'offsetof(' + struct + ',' + field + ')' if field else 'sizeof(' + struct + ')'});return 0;}}\n")
    return src


def test_struct_layout_matches_ctypes(tmp_path):
    from paper_1002_4482_amd import _lib
    checks = []
    for cname, cls in (("pj_opts", _lib.PjOpts), ("pj_stats", _lib.PjStats),
                       ("pj_server_config", _lib.PjServerConfig),
                       ("pj_server_stats", _lib.PjServerStats)):
        checks.append((cname, None, ctypes.sizeof(cls)))
        for f, _ in cls._fields_:
            checks.append((cname, f, getattr(cls, f).offset))
    for i, (s, f, want) in enumerate(checks):
        c = tmp_path / f"t{i}.c"
        c.write_text(_c_sizeof(s, f))
        exe = tmp_path / f"t{i}"
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                       check=True)
        got = int(subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout)
        assert got == want, (s, f, got, want)


def test_python_layer_rejects_short_outputs_and_bad_tables():
    """Argument checks in the Python binding that keep the library from
    writing past a caller's buffer (run on the CPU: the checks come before any
    device call)."""
    torch = pytest.importorskip("torch")
    from paper_1002_4482_amd import api
    with pytest.raises(ValueError):
        api._host_i64(np.zeros(3, np.int64), 4, "h")
    with pytest.raises(ValueError):
        api._host_i64(np.zeros((2, 2), np.int64), 4, "h")
    assert api._host_i64([0, 1, 5], 3, "h").dtype == np.int64
    with pytest.raises(ValueError):
        api._need(torch.empty(3, dtype=torch.int32), 4, "rank")
    api._need(torch.empty(4, dtype=torch.int32), 4, "rank")


def test_argument_checks_before_any_device_work(lib):
    # these calls are refused by host-side checks before any HIP call, so they
    # run without a GPU; the pointers are host memory and never dereferenced
    from paper_1002_4482_amd import _lib
    L = _lib.load()
    EINVAL = -1
    buf = np.zeros(64, dtype=np.int32)
    p = buf.ctypes.data
    o = _lib.PjOpts()
    L.pj_opts_init(ctypes.byref(o))
    assert L.pj_list_rank_ex(p, -1, p + 4 * 32, ctypes.byref(o), None) == EINVAL
    assert L.pj_list_rank_ex(None, 16, p, ctypes.byref(o), None) == EINVAL
    # partial overlap of rank and succ
    assert L.pj_list_rank_ex(p, 16, p + 8, ctypes.byref(o), None) == EINVAL
    # in place is allowed, but not with the full output check
    o.validate = 1
    assert L.pj_list_rank_ex(p, 16, p, ctypes.byref(o), None) == EINVAL
    o.validate = 0
    # weighted: weights required, no Wyllie, no to-tail form, no full check,
    # and rank must not overlap the weights
    w = p + 4 * 16
    r = p + 4 * 32
    assert L.pj_list_rank_weighted(p, None, 16, r, ctypes.byref(o), None) == EINVAL
    for field, value in (("algo", 1), ("to_tail", 1), ("validate", 1)):
        L.pj_opts_init(ctypes.byref(o))
        setattr(o, field, value)
        assert L.pj_list_rank_weighted(p, w, 16, r, ctypes.byref(o), None) == EINVAL, field
    L.pj_opts_init(ctypes.byref(o))
    assert L.pj_list_rank_weighted(p, w, 16, w + 4, ctypes.byref(o), None) == EINVAL
    assert L.pj_list_rank_weighted_batched(p, None, p, 1, r, ctypes.byref(o), None) == EINVAL
    # weighted workspace is larger than the packed form's
    assert (L.pj_list_rank_weighted_workspace_bytes(1 << 20, 1, None)
            > L.pj_list_rank_workspace_bytes(1 << 20, 1, None))


def test_noalloc_refusals_before_any_device_work(lib):
    """pj_list_rank_noalloc refuses, on the host and before any HIP call, an
    input whose workspace exceeds its fixed scratch, and the options that
    would allocate or read back through host memory."""
    from paper_1002_4482_amd import _lib
    L = _lib.load()
    buf = np.zeros(64, dtype=np.int32)
    p = buf.ctypes.data
    assert L.pj_list_rank_noalloc_max_bytes() == 64 << 20
    assert L.pj_list_rank_workspace_bytes(1 << 24, 1, None) <= L.pj_list_rank_noalloc_max_bytes()
    assert L.pj_list_rank_noalloc(p, 1 << 25, p, None, None) == _lib.PJ_ESCRATCH
    assert L.pj_list_rank_noalloc(p, -1, p, None, None) == _lib.PJ_EINVAL
    assert L.pj_strerror(_lib.PJ_ESCRATCH).startswith(b"input needs more workspace")
    st = _lib.PjStats()
    for field, value in (("use_graph", 1), ("validate", 1), ("workspace", p),
                         ("stats", ctypes.pointer(st))):
        o = _lib.PjOpts()
        L.pj_opts_init(ctypes.byref(o))
        setattr(o, field, value)
        assert L.pj_list_rank_noalloc(p, 16, p + 4 * 32, ctypes.byref(o), None) == \
            _lib.PJ_EINVAL, field
