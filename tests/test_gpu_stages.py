"""Every load-stage schedule of the single-RHS Dslash (1, 2, 4, 8 hops per
stage, and the double-buffered -1, -2 that issue the next stage's loads
before the current stage's arithmetic) computes the same per-site arithmetic
in the same order: outputs are bit-identical, and the tuned launch matches
the oracle (checked elsewhere), so every schedule does."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import need_gpu
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

DIMS = (6, 8, 10, 12)       # Vh = 2880: a ragged last tile


@pytest.mark.parametrize("recon", [18, 12, 8])
def test_stage_schedules_bit_identical(recon):
    hisq = need_gpu()
    fat, lng = inputs.make_links(DIMS, "near_unit", seed=inputs.GAUGE_SEED + 80, device="cuda")
    vh = oracle.volume(DIMS) // 2
    psi = inputs.gaussian_spinor(vh, 81, device="cuda")
    names = ("double", "single", "half", "int20", "int30", "int30_fp32", "int24", "sx24", "sx24_int30")
    try:
        for name in (("double", "int30") if recon == 8 else names):
            f = hisq.fmt(name)
            pg = hisq.pack_gauge(fat, lng, DIMS, f.gauge, long_recon=recon)
            pin = hisq.pack_spinor(psi, f.spinor)
            ref = None
            for stage in (1, 2, 4, 8, -1, -2):
                for block, grid, sweep in ((256, 0, 1), (128, 16, 0), (256, 0, 2), (128, 16, 2)):
                    hisq.hisq_tune_set(name, DIMS, 1, 1, 1, stage, block, grid, sweep=sweep, long_recon=recon)
                    y = hisq.dslash(pin, pg, 0, f)
                    if ref is None:
                        ref = y.clone()
                    assert torch.equal(y, ref), (name, recon, stage, block, grid, sweep)
    finally:
        hisq.hisq_tune_clear()


def test_pipelined_stage_in_solver():
    """CG with the double-buffered schedules fixed for both operators"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 82)
    ev = oracle.parity_sites(dims, 0)
    b = inputs.gaussian_spinor(ev.size, 83).numpy()
    try:
        for name, stage in (("double", -1), ("half", -2)):
            hisq.hisq_tune_set(name, dims, 1, 1, 1, stage, 256, 0, sweep=1)
        g64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_F64)
        g16 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_FIX16)
        x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), g64, g16, mass, tol=1e-10, sloppy="half")
        assert st["status"] == "HISQ_OK", st
        full_x = np.zeros((oracle.volume(dims), 3), complex)
        full_b = np.zeros_like(full_x)
        full_x[ev], full_b[ev] = x.cpu().numpy(), b
        assert oracle.true_residual(fat.numpy(), lng.numpy(), full_x, full_b, dims, mass) <= 1e-10 * (1 + 1e-6)
    finally:
        hisq.hisq_tune_clear()


SF_NAME = {0: "f64", 1: "f32", 2: "half16", 3: "int20", 4: "int30", 5: "int24"}
DIMS_M = (6, 6, 6, 6)       # Vh = 648: four lanes per site leave a partial last tile of 256 lanes


@pytest.mark.parametrize("recon", [18, 12])
@pytest.mark.parametrize("nrhs", [4, 8, 16])
def test_matrix_core_block_matches_single(recon, nrhs):
    """the 4x4x1 MFMA path (four lanes per site, stage 5) against one FMA
    Dslash per right-hand side: equal to within one output quantum plus FP32
    rounding of the accumulation (the product order differs)"""
    hisq = need_gpu()
    fat, lng = inputs.make_links(DIMS_M, "near_unit", seed=inputs.GAUGE_SEED + 84, device="cuda")
    vh = oracle.volume(DIMS_M) // 2
    try:
        for name in ("single", "half", "int20", "int24", "sx24"):
            f = hisq.fmt(name)
            pg = hisq.pack_gauge(fat, lng, DIMS_M, f.gauge, long_recon=recon)
            nb = hisq.hisq_spinor_bytes(vh, f.spinor)
            packed = [hisq.pack_spinor(inputs.gaussian_spinor(vh, 90 + j, device="cuda"), f.spinor)
                      for j in range(nrhs)]
            pin = torch.cat([pk[:nb] for pk in packed]).contiguous()
            for grid, sweep in ((0, 1), (16, 0)):
                hisq.hisq_tune_set(name, DIMS_M, nrhs, nrhs // 4, 4, 5, 256, grid, sweep=sweep, long_recon=recon)
                pout = torch.empty_like(pin)
                hisq.hisq_dslash_batched(pout, pin, pg.desc, 1, f, nrhs)
                for j in range(nrhs):
                    yb = hisq.unpack_spinor(pout[j * nb:(j + 1) * nb].contiguous(), vh, f.spinor).cpu().numpy()
                    ys = hisq.unpack_spinor(hisq.dslash(packed[j], pg, 1, f), vh, f.spinor).cpu().numpy()
                    q = oracle.spinor_quantum(ys, SF_NAME[f.spinor])[:, None]
                    d = yb - ys
                    bound = q + 1e-6 * np.abs(ys).max()
                    assert (np.maximum(np.abs(d.real), np.abs(d.imag)) <= bound).all(), (name, recon, nrhs, j)
            del pg, pin, packed
    finally:
        hisq.hisq_tune_clear()


def test_matrix_core_block_in_batched_cg():
    hisq = need_gpu()
    dims, mass, nrhs = (8, 8, 8, 8), 0.05, 16
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 85)
    ev = oracle.parity_sites(dims, 0)
    bs = inputs.gaussian_spinor(ev.size, 86, nrhs=nrhs).numpy()
    try:
        for c in (4, 8, 16):
            hisq.hisq_tune_set("int20", dims, c, c // 4, 4, 5, 256, 0, sweep=1)
        g64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_F64)
        g16 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_FIX16)
        x, st = hisq.cg_solve_batched(torch.from_numpy(bs).cuda(), g64, g16, mass, tol=1e-10, sloppy="int20")
        assert st["status"] == "HISQ_OK", st
        x = x.cpu().numpy()
        for j in range(nrhs):
            fx = np.zeros((oracle.volume(dims), 3), complex)
            fb = np.zeros_like(fx)
            fx[ev], fb[ev] = x[j], bs[j]
            assert oracle.true_residual(fat.numpy(), lng.numpy(), fx, fb, dims, mass) <= 1e-10 * (1 + 1e-6), j
    finally:
        hisq.hisq_tune_clear()
