"""Sec. 3.1 / Fig. 1 analog: at a light mass on rough links, double-half CG with
reliable updates alone (Fletcher-Reeves beta, no gradient re-projection) stalls,
while the stabilised double-half CG (Polak-Ribiere beta, re-projection, FP64
buffered solution) converges within a small factor of the FP64 iteration count.
The stabilised solution is checked with the oracle's FP64 operator."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import need_gpu
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu


def test_stabilised_cg_converges_where_naive_stalls():
    hisq = need_gpu()
    dims, mass, tol = (16, 16, 16, 16), 0.001, 1e-10
    fat, lng = inputs.make_links(dims, "haar", seed=inputs.GAUGE_SEED + 60)
    ev = oracle.parity_sites(dims, 0)
    b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED + 60).numpy()
    bt = torch.from_numpy(b).cuda()
    g64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_F64)
    g16 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_FIX16)
    _, s64 = hisq.cg_solve(bt, g64, g64, mass, tol=tol, sloppy="double", delta=0.0)
    assert s64["status"] == "HISQ_OK"
    cap = int(1.6 * s64["iters"])
    x, stab = hisq.cg_solve(bt, g64, g16, mass, tol=tol, sloppy="half", maxiter=cap)
    assert stab["status"] == "HISQ_OK", stab
    _, naive = hisq.cg_solve(bt, g64, g16, mass, tol=tol, sloppy="half", maxiter=cap, pr_beta=0, reproject=0)
    assert naive["status"] == "HISQ_ENOCONV" and naive["true_resid"] > 1e3 * tol, naive
    full_x = np.zeros((oracle.volume(dims), 3), dtype=np.complex128)
    full_b = np.zeros_like(full_x)
    full_x[ev], full_b[ev] = x.cpu().numpy(), b
    assert oracle.true_residual(fat.numpy(), lng.numpy(), full_x, full_b, dims, mass) <= tol * (1 + 1e-6)
