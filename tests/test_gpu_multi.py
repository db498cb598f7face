"""Several lattices in one launch (hisq_dslash_multi) against the oracle's
emulated Dslash of each lattice, and bit for bit against one hisq_dslash per
lattice (same per-site arithmetic, only the schedule differs)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import need_gpu
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

TRIPLETS = ["double", "single", "half", "int20", "int30", "int30_fp32", "int24", "sx24", "sx24_int30"]
SF_NAME = {0: "f64", 1: "f32", 2: "half16", 3: "int20", 4: "int30", 5: "int24"}
GF_NAME = {0: "f64", 1: "f32", 2: "fix16", 3: "fix32", 4: "sx24"}
# the uneven batch of the block-solver workload plus a non-cubic one
LATTICES = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (4, 6, 4, 8)]


def _fields(dims, k):
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 40 + k)
    V = oracle.volume(dims)
    psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 40 + k).numpy()
    return fat, lng, psi


@pytest.mark.parametrize("name", TRIPLETS)
@pytest.mark.parametrize("recon", [18, 12])
def test_multi_matches_single_and_oracle(name, recon):
    hisq = need_gpu()
    f = hisq.fmt(name)
    parity = 0
    data, outs, ins, gauges = [], [], [], []
    for k, dims in enumerate(LATTICES):
        fat, lng, psi = _fields(dims, k)
        pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge, long_recon=recon)
        src = oracle.parity_sites(dims, 1 - parity)
        pin = hisq.pack_spinor(torch.from_numpy(psi[src]).cuda(), f.spinor)
        data.append((dims, fat, lng, psi, pg, pin))
        outs.append(torch.empty_like(pin))
        ins.append(pin)
        gauges.append(pg.desc)
    hisq.hisq_dslash_multi(outs, ins, gauges, parity, f)
    torch.cuda.synchronize()
    for (dims, fat, lng, psi, pg, pin), out in zip(data, outs):
        single = hisq.dslash(pin, pg, parity, f)
        assert torch.equal(out, single), (name, recon, dims)
        dst, src = oracle.parity_sites(dims, parity), oracle.parity_sites(dims, 1 - parity)
        y = hisq.unpack_spinor(out, dst.size, f.spinor).cpu().numpy()
        full = np.zeros_like(psi)
        full[src] = psi[src]
        ref = oracle.emulated_dslash(fat.numpy(), lng.numpy(), full, dims, parity, GF_NAME[f.gauge],
                                     SF_NAME[f.spinor], f.compute, long_recon=recon)[dst]
        q = oracle.spinor_quantum(ref, SF_NAME[f.spinor])[:, None]
        eps = 1e-6 if f.compute == 32 else 1e-13
        bound = 0.5 * q * (1 + 1e-3) + 2 * eps * np.abs(ref).max()
        d = y - ref
        assert (np.maximum(np.abs(d.real), np.abs(d.imag)) <= bound).all(), (name, recon, dims)


def test_multi_rejects_mixed_long_storage():
    hisq = need_gpu()
    f = hisq.fmt("half")
    outs, ins, gauges = [], [], []
    for k, (dims, recon) in enumerate(zip(LATTICES[:2], (18, 12))):
        fat, lng, psi = _fields(dims, k)
        pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge, long_recon=recon)
        pin = hisq.pack_spinor(torch.from_numpy(psi[oracle.parity_sites(dims, 1)]).cuda(), f.spinor)
        outs.append(torch.empty_like(pin))
        ins.append(pin)
        gauges.append(pg.desc)
    with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
        hisq.hisq_dslash_multi(outs, ins, gauges, 0, f)
