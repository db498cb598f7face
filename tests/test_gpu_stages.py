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


@pytest.mark.parametrize("recon", [18, 12])
def test_stage_schedules_bit_identical(recon):
    hisq = need_gpu()
    fat, lng = inputs.make_links(DIMS, "near_unit", seed=inputs.GAUGE_SEED + 80, device="cuda")
    vh = oracle.volume(DIMS) // 2
    psi = inputs.gaussian_spinor(vh, 81, device="cuda")
    try:
        for name in ("double", "single", "half", "int20", "int30", "int30_fp32", "int24", "sx24"):
            f = hisq.fmt(name)
            pg = hisq.pack_gauge(fat, lng, DIMS, f.gauge, long_recon=recon)
            pin = hisq.pack_spinor(psi, f.spinor)
            ref = None
            for stage in (1, 2, 4, 8, -1, -2):
                for block, grid, sweep in ((256, 0, 1), (128, 16, 0)):
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
