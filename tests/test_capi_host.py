"""The C-ABI library on the host: it loads, exports every symbol the public
header declares, and rejects bad arguments before touching a device (no
compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hisq.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hisq_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def hisq():
    from paper_2302_09224_amd import hisq as h
    if not os.path.exists(h.LIB_PATH):
        pytest.fail("libhisq.so is not built (run __graft_entry__.build())")
    h.load()
    return h


def test_header_symbols_exported(hisq):
    names = declared_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(hisq.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_sizes(hisq):
    dims = (4, 6, 8, 10)
    V = 4 * 6 * 8 * 10
    assert hisq.hisq_gauge_bytes(dims, hisq.GAUGE_FIX16) == 4 * V * 36
    assert hisq.hisq_gauge_bytes(dims, hisq.GAUGE_F64) == 4 * V * 144
    assert hisq.hisq_spinor_bytes(V // 2, hisq.SPINOR_INT20) == V // 2 * 16
    assert hisq.hisq_spinor_bytes(V // 2, hisq.SPINOR_INT30) == V // 2 * 24
    assert hisq.hisq_gauge_bytes((5, 4, 4, 4), 0) == 0          # odd extent
    assert hisq.hisq_gauge_bytes((2, 4, 4, 4), 0) == 0          # extent below 4
    assert hisq.hisq_spinor_bytes(10, 9) == 0                   # unknown format
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX16, 18) == 4 * V * 36
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX16, 12) == 4 * V * 24
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_F64, 12) == 4 * V * 96
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX32, 12) == 4 * V * 48
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_F32, 8) == 0  # unknown storage
    p = hisq.hisq_solver_params_default()
    assert p.delta == 0.1 and p.grad_buffer == 4 and p.pr_beta == 1 and p.reproject == 1
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.fmt("half"), p) > 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.hisq_fmt(2, 1, 32), p) == 0   # unsupported triplet
    assert hisq.hisq_multishift_workspace_bytes(dims, 33, hisq.fmt("single"), hisq.fmt("half"), p) == 0


def test_argument_errors(hisq):
    lib = hisq.load()
    g = hisq.hisq_gauge()
    for k, v in enumerate((4, 4, 4, 4)):
        g.dims[k] = v
    g.fmt = hisq.GAUGE_F32
    g.fat = 4096
    g.lng = 8192
    f = hisq.fmt("single")
    # wrong parity, unsupported triplet, gauge/triplet mismatch, unaligned, aliasing: all before any launch
    assert lib.hisq_dslash(4096 * 3, 4096 * 4, ctypes.byref(g), 2, f, None) == -1
    assert lib.hisq_dslash(4096 * 3, 4096 * 4, ctypes.byref(g), 0, hisq.hisq_fmt(1, 2, 32), None) == -1
    assert lib.hisq_dslash(4096 * 3, 4096 * 4, ctypes.byref(g), 0, hisq.fmt("half"), None) == -1
    assert lib.hisq_dslash(4096 * 3 + 4, 4096 * 4, ctypes.byref(g), 0, f, None) == -2
    assert lib.hisq_dslash(4096 * 3, 4096 * 3, ctypes.byref(g), 0, f, None) == -1
    assert "alias" in hisq.hisq_last_error()
    assert lib.hisq_dslash_batched(4096 * 3, 4096 * 4, ctypes.byref(g), 0, f, 17, None) == -1
    g.dims[0] = 5
    assert lib.hisq_dslash(4096 * 3, 4096 * 4, ctypes.byref(g), 0, f, None) == -1
    assert lib.hisq_spinor_pack(None, 4096, 10, 1, None) == -1
    assert lib.hisq_spinor_pack(4096 + 8, 4096, 10, 1, None) == -2
    dims = (ctypes.c_int * 4)(4, 4, 4, 3)
    assert lib.hisq_gauge_pack(ctypes.byref(g), 4096, 4096, 4096, 4096, dims, 0, None) == -1
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.hisq_gauge_pack_recon(ctypes.byref(g), 4096, 4096, 4096, 4096, dims, 0, 9, None) == -1
