"""Dslash launches on a persistent grid (fewer blocks than tiles: every block
sweeps several tiles and writes one reduction partial) inside the solvers.
The launch shapes are fixed with hisq_tune_set, so the solvers' reductions
must count exactly the partials such a launch writes."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import need_gpu
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8, 16)      # Vh = 4096: 16 tiles of 256 lanes per right-hand side; grid 8 = 2+ tiles per block
MASS = 0.05


@pytest.fixture
def persistent():
    hisq = need_gpu()
    hisq.hisq_tune_clear()
    for name in ("double", "single", "half", "int20", "int30"):
        for recon in (18, 12):
            hisq.hisq_tune_set(name, DIMS, 1, 1, 1, 8, 256, 8, sweep=recon % 2, long_recon=recon)
            for c in (2, 4, 8, 16):
                hisq.hisq_tune_set(name, DIMS, c, 1, c, 1, 256, 8, sweep=c % 3 % 2, long_recon=recon)
    yield hisq
    hisq.hisq_tune_clear()


def _setup():
    fat, lng = inputs.make_links(DIMS, "near_unit", seed=inputs.GAUGE_SEED + 21)
    ev = oracle.parity_sites(DIMS, 0)
    return fat, lng, ev


def _full(ev, v):
    f = np.zeros((oracle.volume(DIMS), 3), dtype=np.complex128)
    f[ev] = v
    return f


def test_persistent_dslash_matches_tiled(persistent):
    hisq = persistent
    fat, lng, ev = _setup()
    psi = inputs.gaussian_spinor(ev.size, 31).numpy()
    for name in ("double", "half"):
        f = hisq.fmt(name)
        pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, f.gauge)
        pin = hisq.pack_spinor(torch.from_numpy(psi).cuda(), f.spinor)
        yp = hisq.dslash(pin, pg, 1, f).clone()
        for grid, sweep in ((0, 0), (0, 1), (8, 1)):
            hisq.hisq_tune_set(name, DIMS, 1, 1, 1, 8, 256, grid, sweep=sweep)
            yt = hisq.dslash(pin, pg, 1, f)
            assert torch.equal(yp, yt), (name, grid, sweep)   # same arithmetic per site, only the schedule differs
        hisq.hisq_tune_set(name, DIMS, 1, 1, 1, 8, 256, 8)


def test_persistent_cg(persistent):
    hisq = persistent
    fat, lng, ev = _setup()
    b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED).numpy()
    p64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_F64)
    ph = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_FIX16)
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), p64, ph, MASS, tol=1e-10, sloppy="half")
    assert st["status"] == "HISQ_OK", st
    res = oracle.true_residual(fat.numpy(), lng.numpy(), _full(ev, x.cpu().numpy()), _full(ev, b), DIMS, MASS)
    assert res <= 1e-10 * (1 + 1e-6) and abs(res - st["true_resid"]) <= 1e-3 * res, (res, st)


def test_persistent_batched_cg(persistent):
    hisq = persistent
    fat, lng, ev = _setup()
    bs = inputs.gaussian_spinor(ev.size, inputs.RHS_SEED, nrhs=5).numpy()
    p64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_F64)
    ph = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_FIX16)
    x, st = hisq.cg_solve_batched(torch.from_numpy(bs).cuda(), p64, ph, MASS, tol=1e-10, sloppy="int20")
    assert st["status"] == "HISQ_OK", st
    x = x.cpu().numpy()
    for j in range(5):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), _full(ev, x[j]), _full(ev, bs[j]), DIMS, MASS)
        assert res <= 1e-10 * (1 + 1e-6) and abs(res - st["shift_resid"][j]) <= 1e-3 * res, (j, res)


def test_persistent_multishift(persistent):
    hisq = persistent
    fat, lng, ev = _setup()
    b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED).numpy()
    shifts = [1e-4, 1e-3, 1e-2, 0.1, 1.0, 10.0]
    p64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_F64)
    p32 = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_FIX32)
    p16 = hisq.pack_gauge(fat.cuda(), lng.cuda(), DIMS, hisq.GAUGE_FIX16)
    xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, [1e-10] * 6, p64, p32, p16, MASS,
                                      ms_fmt="int30", ref_fmt="int20")
    assert st["status"] == "HISQ_OK", st
    for i, s in enumerate(shifts):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), _full(ev, xs[i].cpu().numpy()), _full(ev, b), DIMS,
                                   MASS, s)
        assert res <= 1e-10 * (1 + 1e-6) and abs(res - st["shift_resid"][i]) <= 1e-3 * res, (i, res, st)
