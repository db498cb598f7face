"""The allocation-free normal operator against hisq_normal_op (and the
oracle): two calls in a row on one device, the second on a smaller lattice,
each bit-identical to the entry point with a caller-provided tmp field."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import format_bounds, need_gpu, rel_inf
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

SF_NAME = {0: "f64", 1: "f32", 2: "half16", 3: "int20", 4: "int30", 5: "int24"}


@pytest.mark.parametrize("name,recon", [("int20", 12), ("double", 18), ("int30", 12)])
def test_noalloc_normal_op_matches(name, recon):
    hisq = need_gpu()
    f = hisq.fmt(name)
    mass, shift = 0.05, 0.01
    bound = format_bounds()[name][1]
    for k, dims in enumerate([(8, 8, 8, 12), (6, 6, 4, 8)]):       # the second call: a smaller lattice
        fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 90 + k)
        pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge, long_recon=recon)
        ev = oracle.parity_sites(dims, 0)
        p = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED + 90 + k).numpy()
        pin = hisq.pack_spinor(torch.from_numpy(p).cuda(), f.spinor)
        want = torch.empty_like(pin)
        tmp = torch.empty_like(pin)
        hisq.hisq_normal_op(want, pin, tmp, pg.desc, mass, shift, f)
        got = torch.full_like(pin, 0x5A)
        hisq.hisq_normal_op_noalloc(got, pin, pg.desc, mass, shift, f)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (name, dims)
        y = hisq.unpack_spinor(got, ev.size, f.spinor).cpu().numpy()
        full = np.zeros((oracle.volume(dims), 3), dtype=np.complex128)
        full[ev] = p
        ref = oracle.normal_op(fat.numpy(), lng.numpy(), full, dims, mass, shift)[ev]
        assert rel_inf(y, ref) <= bound, (name, dims, rel_inf(y, ref))

