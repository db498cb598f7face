"""The workloads the method is measured on, each as a parity case at its own
size (the oracle checks what it can compute: whole fields at 16^4 and 32^4,
sampled sites of the 48^3x96 solve):

* 16^4, near-unit links: the FP64 and FP32 Dslash (18-real links) against the
  FP64 oracle; double-single CG with reliable updates (delta = 0.1, m = 0.05)
  to a 1e-10 true residual, against the plain FP64 CG on the same GPU.
* 32^4, near-unit links, m = 0.01: every storage triplet's Dslash error
  against the unquantised FP64 oracle, and the mixed-precision CG of each to
  a 1e-10 true residual (measured by the oracle's FP64 operator).
* 48^3x96, near-unit links, m = 0.005: the mixed 12-shift solve (shifts
  log-spaced 1e-5..10, two-row long links, multi-shift in FIX32/INT30/FP64,
  refinement in FIX16/INT20/FP32): every shift's true residual <= 1e-10, the
  residual vector checked against the oracle at sampled sites, and each
  shift's solution against a lone CG solve of that shift.
* 32^3x64, near-unit links, m = 0.01: 16 right-hand sides solved together
  in INT20 storage, each to a 1e-10 true residual (oracle), and the uneven
  batch of lattices 8^4, 12^4, 16^4, 24^4 in one Dslash launch.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import need_gpu, rel_inf
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

# ||D|| <= sum_mu 2 (||F_mu|| + ||L_mu||) <= 8 (1 + 1/24) for these links
# (F = 0.6 U + 0.4 U' with U, U' unitary, L = -U1 U2 U3 / 24), so the
# spectrum of -D_eo D_oe lies in [0, LAMBDA_D]
LAMBDA_D = (8.0 * (1.0 + 1.0 / 24.0)) ** 2


def kappa(mass, shift):
    """condition number bound of 4m^2 + shift - D_eo D_oe"""
    c = 4.0 * mass * mass + shift
    return (c + LAMBDA_D) / c


def host_links(dims, seed):
    fat, lng = inputs.make_links(dims, "near_unit", seed=seed, device="cuda")
    return fat, lng, fat.cpu().numpy(), lng.cpu().numpy()


def full_even(dims, ev, v):
    f = np.zeros((oracle.volume(dims), 3), dtype=np.complex128)
    f[ev] = v
    return f


def test_config_16():
    hisq = need_gpu()
    dims, mass = (16, 16, 16, 16), 0.05
    fat, lng, fat_h, lng_h = host_links(dims, inputs.GAUGE_SEED + 11)
    V = oracle.volume(dims)
    ev, od = oracle.parity_sites(dims, 0), oracle.parity_sites(dims, 1)
    psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 11).numpy()
    src = np.zeros_like(psi)
    src[od] = psi[od]
    ref = oracle.dslash(fat_h, lng_h, src, dims, 0)[ev]
    pgs = {}
    for name, tol in (("double", 1e-13), ("single", 1e-6)):
        f = hisq.fmt(name)
        pgs[name] = hisq.pack_gauge(fat, lng, dims, f.gauge)
        pin = hisq.pack_spinor(torch.from_numpy(psi[od]).cuda(), f.spinor)
        y = hisq.unpack_spinor(hisq.dslash(pin, pgs[name], 0, f), ev.size, f.spinor).cpu().numpy()
        assert rel_inf(y, ref) <= tol, (name, rel_inf(y, ref))
    b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED + 12).numpy()
    bd = torch.from_numpy(b).cuda()
    x64, s64 = hisq.cg_solve(bd, pgs["double"], pgs["double"], mass, tol=1e-10, sloppy="double")
    xm, sm = hisq.cg_solve(bd, pgs["double"], pgs["single"], mass, tol=1e-10, sloppy="single", delta=0.1)
    assert s64["status"] == "HISQ_OK" and sm["status"] == "HISQ_OK", (s64, sm)
    assert sm["reliable_updates"] >= 1
    for x in (x64, xm):
        res = oracle.true_residual(fat_h, lng_h, full_even(dims, ev, x.cpu().numpy()), full_even(dims, ev, b), dims,
                                   mass)
        assert res <= 1e-10 * (1 + 1e-6), res
    d = (xm - x64).norm() / x64.norm()
    assert float(d) <= 2e-10 * kappa(mass, 0.0), float(d)
    # the mixed solve needs about as many iterations as the FP64 one
    assert sm["iters"] <= 1.25 * s64["iters"], (sm["iters"], s64["iters"])


# max-norm relative Dslash error against the unquantised FP64 oracle, per
# triplet: FP64 rounding; FP32 rounding; the fixed-point links (2^-31 or 2^-15
# of the field maximum), the shared-exponent link rows (2^-23 of the row
# maximum) and the spinor quantum of each format
DSLASH_TOL = {"double": 1e-13, "single": 1e-6, "int30": 1e-8, "int30_fp32": 2e-6, "int24": 2e-6, "sx24": 2e-6,
              "sx24_int30": 5e-7, "int20": 3e-4, "half": 3e-4}


def test_config_32_formats():
    hisq = need_gpu()
    dims, mass = (32, 32, 32, 32), 0.01
    fat, lng, fat_h, lng_h = host_links(dims, inputs.GAUGE_SEED + 13)
    V = oracle.volume(dims)
    ev, od = oracle.parity_sites(dims, 0), oracle.parity_sites(dims, 1)
    psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 13).numpy()
    src = np.zeros_like(psi)
    src[od] = psi[od]
    ref = oracle.dslash(fat_h, lng_h, src, dims, 0)[ev]
    b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED + 14).numpy()
    bd, bfull = torch.from_numpy(b).cuda(), full_even(dims, ev, b)
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64)
    err, iters = {}, {}
    for name in ("double", "single", "int30", "int30_fp32", "int24", "sx24", "sx24_int30", "int20", "half"):
        f = hisq.fmt(name)
        pg = g64 if f.gauge == hisq.GAUGE_F64 else hisq.pack_gauge(fat, lng, dims, f.gauge)
        pin = hisq.pack_spinor(torch.from_numpy(psi[od]).cuda(), f.spinor)
        y = hisq.unpack_spinor(hisq.dslash(pin, pg, 0, f), ev.size, f.spinor).cpu().numpy()
        err[name] = rel_inf(y, ref)
        x, st = hisq.cg_solve(bd, g64, pg, mass, tol=1e-10, sloppy=name)
        assert st["status"] == "HISQ_OK", (name, st)
        res = oracle.true_residual(fat_h, lng_h, full_even(dims, ev, x.cpu().numpy()), bfull, dims, mass)
        assert res <= 1e-10 * (1 + 1e-6), (name, res)
        iters[name] = st["iters"]
        del pg, pin, x
        torch.cuda.empty_cache()
    print("\n32^4 m=0.01 per-Dslash error vs FP64 oracle / CG iterations to 1e-10:",
          {k: (f"{err[k]:.2e}", iters[k]) for k in err})
    for name, e in err.items():
        assert e <= DSLASH_TOL[name], (name, e)
    # at equal bit width the 20-bit spinor is the more accurate one (Sec. 4)
    assert err["int20"] <= err["half"], err
    assert iters["int20"] <= 1.02 * iters["half"], iters


def _neighbours(sites, dims):
    """lexicographic sites at +-1, +-3 hops of each site, per (mu, hop)"""
    X, Y, Z, T = dims
    c = [sites % X, (sites // X) % Y, (sites // (X * Y)) % Z, sites // (X * Y * Z)]
    out = []
    for mu in range(4):
        for h in (1, -1, 3, -3):
            cc = [v.copy() for v in c]
            cc[mu] = (cc[mu] + h) % dims[mu]
            out.append((mu, h, ((cc[3] * Z + cc[2]) * Y + cc[1]) * X + cc[0]))
    return out


class SampledOperator:
    """the oracle's (4m^2 + s - D_eo D_oe) x at a few even sites of a large
    lattice: only the links and solution entries those sites reach are
    copied from the device into lazily allocated full-size arrays"""

    def __init__(self, fat, lng, dims, samp_cb):
        V = oracle.volume(dims)
        self.dims, self.V = dims, V
        self.ev = oracle.parity_sites(dims, 0)
        self.S = self.ev[samp_cb]
        self.samp_cb = samp_cb
        n1 = np.unique(np.concatenate([nb for _, _, nb in _neighbours(self.S, dims)]))
        n2 = np.unique(np.concatenate([nb for _, _, nb in _neighbours(n1, dims)]))
        self.n1, self.n2 = n1, n2
        links = set()
        for sites in (self.S, n1):
            for mu, h, nb in _neighbours(sites, dims):
                links.update((mu * V + (sites if h > 0 else nb)).tolist())
        lidx = np.array(sorted(links))
        li = torch.from_numpy(lidx).cuda()
        self.fat = np.zeros((4 * V, 3, 3), dtype=np.complex128)
        self.lng = np.zeros((4 * V, 3, 3), dtype=np.complex128)
        self.fat[lidx] = fat.reshape(4 * V, 3, 3)[li].cpu().numpy()
        self.lng[lidx] = lng.reshape(4 * V, 3, 3)[li].cpu().numpy()
        self.n2_cb = torch.from_numpy(np.searchsorted(self.ev, n2)).cuda()
        self.x = np.zeros((V, 3), dtype=np.complex128)
        self.y = np.zeros((V, 3), dtype=np.complex128)

    def apply(self, x_dev, c):
        self.x[self.n2] = x_dev[self.n2_cb].cpu().numpy()
        f4 = (self.fat.reshape(4, self.V, 3, 3), self.lng.reshape(4, self.V, 3, 3))
        self.y[self.n1] = oracle.dslash_sites(*f4, self.x, self.dims, self.n1)
        return c * self.x[self.S] - oracle.dslash_sites(*f4, self.y, self.dims, self.S)


def test_config_48_multishift():
    hisq = need_gpu()
    dims, mass = (48, 48, 48, 96), 0.005
    shifts = list(np.logspace(-5, 1, 12))
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED, device="cuda")
    vh = oracle.volume(dims) // 2
    b = inputs.gaussian_spinor(vh, inputs.SOURCE_SEED, device="cuda")
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64, long_recon=12)
    gms = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_FIX32, long_recon=12)
    gref = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_FIX16, long_recon=12)
    xs, st = hisq.multishift_cg_solve(b, shifts, 1e-10, g64, gms, gref, mass, ms_fmt="int30", ref_fmt="int20")
    assert st["status"] == "HISQ_OK", st
    samp_cb = np.unique(np.concatenate([np.random.default_rng(7).integers(0, vh, 400), [0, vh - 1]]))
    op = SampledOperator(fat, lng, dims, samp_cb)
    del fat, lng
    torch.cuda.empty_cache()
    f64 = hisq.fmt("double")
    bp = hisq.pack_spinor(b, hisq.SPINOR_F64)
    b_s = b[torch.from_numpy(samp_cb).cuda()].cpu().numpy()
    bn = float(b.norm())
    for i, (s, x) in enumerate(zip(shifts, xs)):
        c = 4 * mass * mass + s
        # the whole residual with the library's FP64 operator ...
        xp = hisq.pack_spinor(x, hisq.SPINOR_F64)
        ax, tmp = torch.empty_like(xp), torch.empty_like(xp)
        hisq.hisq_normal_op(ax, xp, tmp, g64.desc, mass, s, f64)
        r = b - hisq.unpack_spinor(ax, vh, hisq.SPINOR_F64)
        res = float(r.norm()) / bn
        assert res <= 1e-10 * (1 + 1e-6), (i, s, res)
        assert abs(res - st["shift_resid"][i]) <= 1e-3 * res, (i, res, st["shift_resid"][i])
        # ... is the oracle's at the sampled sites, up to FP64 rounding of b - A x
        r_or = b_s - op.apply(x, c)
        r_gpu = r[torch.from_numpy(samp_cb).cuda()].cpu().numpy()
        scale = np.abs(b_s).max() + (c + LAMBDA_D) * float(x.abs().max())
        assert np.abs(r_or - r_gpu).max() <= 1e-13 * scale, (i, np.abs(r_or - r_gpu).max(), scale)
        # the sampled sites carry no more than their share of the residual
        assert np.sqrt(np.mean(np.abs(r_or) ** 2) * vh) <= 4 * 1e-10 * bn, i
        # a lone CG on this shift reaches the same solution, to what the condition number allows
        xc, sc = hisq.cg_solve(b, g64, gref, mass, shift=s, tol=1e-10, sloppy="int20")
        assert sc["status"] == "HISQ_OK", (i, sc)
        d = float((xc - x).norm() / xc.norm())
        assert d <= 2e-10 * kappa(mass, s), (i, s, d)
        del xp, ax, tmp, r, xc


def test_config_32x64_batched():
    hisq = need_gpu()
    dims, mass, nrhs = (32, 32, 32, 64), 0.01, 16
    fat, lng, fat_h, lng_h = host_links(dims, inputs.GAUGE_SEED + 15)
    ev = oracle.parity_sites(dims, 0)
    bs = inputs.gaussian_spinor(ev.size, inputs.RHS_SEED, nrhs=nrhs, device="cuda")
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64, long_recon=12)
    g16 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_FIX16, long_recon=12)
    x, st = hisq.cg_solve_batched(bs, g64, g16, mass, tol=1e-10, sloppy="int20")
    assert st["status"] == "HISQ_OK", st
    for j in range(nrhs):
        res = oracle.true_residual(fat_h, lng_h, full_even(dims, ev, x[j].cpu().numpy()),
                                   full_even(dims, ev, bs[j].cpu().numpy()), dims, mass)
        assert res <= 1e-10 * (1 + 1e-6), (j, res)
    for j in (0, nrhs - 1):
        xc, sc = hisq.cg_solve(bs[j].contiguous(), g64, g64, mass, tol=1e-10, sloppy="double")
        assert float((xc - x[j]).norm() / xc.norm()) <= 2e-10 * kappa(mass, 0.0)


def test_config_uneven_lattices_one_launch():
    """8^4 + 12^4 + 16^4 + 24^4 in one launch (FIX16/INT20/FP32, two-row long
    links) against the unquantised oracle Dslash of each lattice"""
    hisq = need_gpu()
    f = hisq.fmt("int20")
    lat = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (24, 24, 24, 24)]
    data, outs, ins, gauges = [], [], [], []
    for k, dims in enumerate(lat):
        fat, lng, fat_h, lng_h = host_links(dims, inputs.GAUGE_SEED + 60 + k)
        V = oracle.volume(dims)
        psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 60 + k).numpy()
        od = oracle.parity_sites(dims, 1)
        pg = hisq.pack_gauge(fat, lng, dims, f.gauge, long_recon=12)
        pin = hisq.pack_spinor(torch.from_numpy(psi[od]).cuda(), f.spinor)
        data.append((dims, fat_h, lng_h, psi, pg))
        outs.append(torch.empty_like(pin))
        ins.append(pin)
        gauges.append(pg.desc)
    hisq.hisq_dslash_multi(outs, ins, gauges, 0, f)
    for (dims, fat_h, lng_h, psi, pg), out in zip(data, outs):
        ev, od = oracle.parity_sites(dims, 0), oracle.parity_sites(dims, 1)
        src = np.zeros_like(psi)
        src[od] = psi[od]
        ref = oracle.dslash(fat_h, lng_h, src, dims, 0)[ev]
        y = hisq.unpack_spinor(out, ev.size, f.spinor).cpu().numpy()
        assert rel_inf(y, ref) <= DSLASH_TOL["int20"], (dims, rel_inf(y, ref))
