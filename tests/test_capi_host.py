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
    assert hisq.hisq_spinor_bytes(V // 2, hisq.SPINOR_INT24) == V // 2 * 20
    assert hisq.hisq_spinor_bytes(V // 2, 6) == 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.fmt("int24"), hisq.hisq_solver_params_default()) > 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.hisq_fmt(3, 5, 64), hisq.hisq_solver_params_default()) == 0
    assert hisq.hisq_bicgstab_workspace_bytes(dims, 4, hisq.fmt("int24")) > 0
    assert hisq.hisq_gauge_bytes(dims, hisq.GAUGE_SX24) == 4 * V * 60
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_SX24, 12) == 4 * V * 40
    assert hisq.hisq_gauge_bytes(dims, 5) == 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.fmt("sx24"), hisq.hisq_solver_params_default()) > 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.hisq_fmt(4, 3, 32), hisq.hisq_solver_params_default()) == 0
    # SX24 links with 30-bit spinors: FP64 arithmetic only
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.fmt("sx24_int30"), hisq.hisq_solver_params_default()) > 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.hisq_fmt(4, 4, 32), hisq.hisq_solver_params_default()) == 0
    assert hisq.hisq_gauge_bytes((5, 4, 4, 4), 0) == 0          # odd extent
    assert hisq.hisq_gauge_bytes((2, 4, 4, 4), 0) == 0          # extent below 4
    assert hisq.hisq_spinor_bytes(10, 9) == 0                   # unknown format
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX16, 18) == 4 * V * 36
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX16, 12) == 4 * V * 24
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_F64, 12) == 4 * V * 96
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX32, 12) == 4 * V * 48
    assert hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_F32, 8) == 0  # unknown storage
    p = hisq.hisq_solver_params_default()
    assert p.delta == 0.1 and p.grad_buffer == 8 and p.pr_beta == 1 and p.reproject == 1
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.fmt("half"), p) > 0
    assert hisq.hisq_cg_workspace_bytes(dims, hisq.hisq_fmt(2, 1, 32), p) == 0   # unsupported triplet
    assert hisq.hisq_multishift_workspace_bytes(dims, 33, hisq.fmt("single"), hisq.fmt("half"), p) == 0
    assert hisq.hisq_bicgstab_workspace_bytes(dims, 4, hisq.fmt("int20")) > 0
    assert hisq.hisq_bicgstab_workspace_bytes(dims, 0, hisq.fmt("int20")) == 0
    assert hisq.hisq_bicgstab_workspace_bytes(dims, 9, hisq.fmt("int20")) == 0
    assert p.batch_refine == 3
    p.batch_refine = 1
    wb = hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int20"), p)
    p.batch_refine = 0
    ws = hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int20"), p)
    assert wb > ws > 0                                           # room for a block of 11 shifted systems
    p.batch_refine = 1
    assert hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int24"), p) > ws
    p.batch_refine = 0
    # refinement in FIX32/INT30/FP32 has no batched form: no extra room
    p.batch_refine = 1
    a = hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int30_fp32"), p)
    p.batch_refine = 0
    assert a == hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int30_fp32"), p)
    p.batch_refine = 2                                           # the batch overlapping the base: same room
    assert hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int20"), p) == wb
    p.batch_refine = 3                                           # the base joins the block: room for 12
    assert hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int20"), p) > wb
    p.batch_refine = 4
    assert hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int20"), p) == 0
    p.batch_refine = 1
    p.ru_estimate = 2
    assert hisq.hisq_multishift_workspace_bytes(dims, 12, hisq.fmt("int30"), hisq.fmt("int20"), p) == 0


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
    # several lattices in one launch: count, null and aliasing checks before any launch
    for k, v in enumerate((4, 4, 4, 4)):
        g.dims[k] = v
    g.fmt = hisq.GAUGE_F32
    outs = (ctypes.c_void_p * 2)(4096 * 3, 4096 * 3)
    ins = (ctypes.c_void_p * 2)(4096 * 4, 4096 * 5)
    gp = (ctypes.POINTER(hisq.hisq_gauge) * 2)(ctypes.pointer(g), ctypes.pointer(g))
    assert lib.hisq_dslash_multi(0, outs, ins, gp, 0, f, None) == -1
    assert lib.hisq_dslash_multi(9, outs, ins, gp, 0, f, None) == -1
    assert lib.hisq_dslash_multi(2, outs, ins, gp, 0, f, None) == -1     # two lattices write one field
    assert "alias" in hisq.hisq_last_error()
    assert lib.hisq_dslash_multi(2, outs, ins, None, 0, f, None) == -1


def test_tune_set_validation(hisq):
    dims = (8, 8, 8, 16)
    hisq.hisq_tune_clear()
    hisq.hisq_tune_set("half", dims, 1, 1, 1, 4, 128, 0)
    hisq.hisq_tune_set("half", dims, 1, 1, 1, 2, 128, 0, long_recon=12)
    hisq.hisq_tune_set("double", dims, 4, 2, 2, 1, 256, 2048, sweep=1)
    hisq.hisq_tune_set("int24", dims, 4, 4, 1, 1, 256, 0)
    hisq.hisq_tune_set("int30", dims, 1, 1, 1, -2, 256, 0)
    hisq.hisq_tune_set("int20", dims, 16, 4, 4, 5, 256, 0)      # matrix-core path, four lanes per site
    hisq.hisq_tune_set("int20", dims, 8, 4, 2, -1, 256, 0)      # double-buffered hops, 4 right-hand sides per lane
    hisq.hisq_tune_set("int30", dims, 1, 1, 1, -2, 256, 0, long_recon=8)   # eight-parameter long links
    rep = hisq.hisq_tune_report()
    assert "recon 18 lattice 8x8x8x16 rhs-block 4: nr 2 rg 2 stage 1 block 256 grid 2048 sweep 1" in rep
    assert "recon 12 lattice 8x8x8x16 rhs-block 1: nr 1 rg 1 stage 2 block 128 grid 0 sweep 0" in rep
    assert "triplet 341 recon 8 lattice 8x8x8x16 rhs-block 1: nr 1 rg 1 stage -2 block 256 grid 0 sweep 0" in rep
    bad = [("half", dims, 3, 1, 3, 1, 256, 0),          # block of 3 right-hand sides
           ("half", dims, 4, 2, 1, 1, 256, 0),          # nr*rg != block
           ("half", dims, 1, 1, 1, 3, 256, 0),          # stage
           ("half", dims, 2, 2, 1, 2, 256, 0),          # stages only with one right-hand side per lane
           ("half", dims, 16, 16, 1, -1, 256, 0),       # double-buffered stages: at most 8 right-hand sides per lane
           ("half", dims, 2, 2, 1, -2, 256, 0),         # two-hop double-buffered stages: one right-hand side only
           ("half", dims, 1, 1, 1, -4, 256, 0),         # double-buffered stages of 1 or 2 hops
           ("half", dims, 16, 8, 2, 5, 256, 0),         # matrix-core path needs four lanes per site
           ("double", dims, 16, 4, 4, 5, 256, 0),       # matrix-core path is FP32 only
           ("half", dims, 1, 1, 1, 1, 192, 0),          # block size
           ("half", dims, 1, 1, 1, 1, 256, 12),         # grid not a multiple of 8
           ("int30_fp32", dims, 2, 1, 2, 1, 256, 0),    # no batched form
           ("half", (8, 8, 8, 7), 1, 1, 1, 1, 256, 0),  # odd extent
           ("half", dims, 1, 1, 1, 1, 256, 0, 3),       # sweep order
           ("half", dims, 1, 1, 1, 1, 256, 0, 0, 9),    # long-link storage
           ("half", dims, 1, 1, 1, 1, 256, 0, 0, 8),    # eight parameters: FP64 triplets only
           ("double", dims, 2, 1, 2, 1, 256, 0, 0, 8)]  # eight parameters: one right-hand side
    for args in bad:
        with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
            hisq.hisq_tune_set(*args)
    # blocks of right-hand sides: hisq_tune_set pins the fused-reduction shape too,
    # hisq_tune_set_fused only that one
    rep = hisq.hisq_tune_report()
    assert "recon 18 lattice 8x8x8x16 rhs-block 4 reduction: nr 2 rg 2 stage 1 block 256 grid 2048 sweep 1" in rep
    assert "rhs-block 1 reduction" not in rep
    hisq.hisq_tune_set_fused("double", dims, 4, 4, 1, 1, 128, 0)
    rep = hisq.hisq_tune_report()
    assert "recon 18 lattice 8x8x8x16 rhs-block 4 reduction: nr 4 rg 1 stage 1 block 128 grid 0 sweep 0" in rep
    assert "recon 18 lattice 8x8x8x16 rhs-block 4: nr 2 rg 2 stage 1 block 256 grid 2048 sweep 1" in rep
    for args in [("half", dims, 1, 1, 1, 1, 256, 0),       # one right-hand side has a single shape
                 ("half", dims, 4, 2, 1, 1, 256, 0),       # nr*rg != block
                 ("int30_fp32", dims, 2, 1, 2, 1, 256, 0)]:  # no batched form
        with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
            hisq.hisq_tune_set_fused(*args)
    hisq.hisq_tune_clear()
    assert hisq.hisq_tune_report() == ""


def test_tune_cache_needs_a_device(hisq, tmp_path):
    """without a HIP device the tune cache calls report HISQ_EHIP and touch no file"""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(hisq.HisqError, match="HISQ_EHIP"):
        hisq.hisq_tune_save(tmp_path / "t.txt")
    with pytest.raises(hisq.HisqError, match="HISQ_EHIP"):
        hisq.hisq_tune_load(tmp_path / "t.txt")
    assert not (tmp_path / "t.txt").exists()
    assert hisq.load().hisq_tune_save(None) == -1
    assert hisq.load().hisq_tune_load(None, None) == -1


def test_noalloc_rejects_oversize_before_device_work(hisq):
    """the allocation-free normal operator refuses a lattice whose odd-parity
    intermediate exceeds its scratch array, before any device call (the
    pointers here are never dereferenced)"""
    import ctypes
    lib = hisq.load()
    g = hisq.hisq_gauge()
    for k, v in enumerate((48, 48, 48, 96)):          # F64 intermediate: 255 MB > 128 MiB
        g.dims[k] = v
    g.fmt, g.fat, g.lng, g.fat_max, g.long_max, g.long_recon, g.long_coeff = hisq.GAUGE_F64, 4096, 8192, 1, 1, 18, 1
    st = lib.hisq_normal_op_noalloc(ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.byref(g), 0.1, 0.0,
                                    hisq.fmt("double"), None)
    assert st == -1 and "scratch" in hisq.hisq_last_error()
    g.dims[3] = 48                                     # 127 MB: within the array, but unaligned pointers
    st = lib.hisq_normal_op_noalloc(ctypes.c_void_p((1 << 20) + 8), ctypes.c_void_p(2 << 20), ctypes.byref(g), 0.1,
                                    0.0, hisq.fmt("double"), None)
    assert st == -2


def test_workspace_too_small_is_reported_before_any_device_work(hisq):
    """every solver checks its workspace before touching the device (pointers
    here are never dereferenced)"""
    import ctypes
    lib = hisq.load()
    dims = (4, 4, 4, 4)
    fake = 1 << 20

    def gauge(fmt):
        g = hisq.hisq_gauge()
        for k in range(4):
            g.dims[k] = dims[k]
        g.fmt, g.fat, g.lng, g.fat_max, g.long_max = fmt, fake, fake, 1.0, 1.0
        g.long_recon, g.long_coeff = 18, 1.0
        return g

    g64, g16 = gauge(hisq.GAUGE_F64), gauge(hisq.GAUGE_FIX16)
    p = hisq.hisq_solver_params_default()
    st = hisq.hisq_solver_stats()
    half = hisq.fmt("half")
    assert lib.hisq_cg_solve(fake, fake, g64, g16, 0.1, 0.0, 1e-10, half, p, fake, 16, ctypes.byref(st), None) == -6
    shifts = (ctypes.c_double * 2)(0.0, 0.1)
    tols = (ctypes.c_double * 2)(1e-10, 1e-10)
    xs = (ctypes.c_void_p * 2)(fake, fake)
    assert lib.hisq_multishift_cg_solve(xs, fake, shifts, 2, tols, g64, g16, g16, 0.1, half, half, p, fake, 16,
                                        ctypes.byref(st), None) == -6
    assert lib.hisq_cg_solve_batched(fake, fake, 4, g64, g16, 0.1, 0.0, 1e-10, half, p, fake, 16,
                                     ctypes.byref(st), None) == -6
    assert lib.hisq_bicgstab_solve(fake, fake, g64, g16, 0.1, 1e-10, 4, half, p, fake, 16, ctypes.byref(st),
                                   None) == -6
    assert "workspace" in hisq.hisq_last_error()
