"""Long links stored as eight parameters (Sec. 1, "Compression": eight real
degrees of freedom of a special unitary matrix) for the triplets with FP64
arithmetic: the packing bit for bit against the oracle's encoder, the Dslash
against the oracle's emulation of the same storage element by element, and
the solvers with such links against the oracle's FP64 operator.

The rebuild of a link divides by N = |U01|^2 + |U02|^2 and takes the root of
|U20|^2 = N - |U10|^2, so the rounding of its arithmetic is amplified by about
kappa = 1/min(N, |U20|^2) (pinned on the oracle's rebuild).  The Dslash bound
is therefore the bound of the other storage forms (half an output quantum
plus the FP64 allowance) plus, per output site, 1000 eps_64 kappa |c| |psi|
summed over its eight long-link hops and three colours."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import long8_records, need_gpu
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

TRIPLETS8 = ["double", "int30"]
SF_NAME = {0: "f64", 1: "f32", 2: "half16", 3: "int20", 4: "int30", 5: "int24"}
GF_NAME = {0: "f64", 1: "f32", 2: "fix16", 3: "fix32", 4: "sx24"}


def rebuild_allowance(lng, psi_full, dims):
    """per site of the lattice: the first-order bound of the FP64 rebuild's
    rounding in the Dslash output at that site"""
    c, u = oracle.long_link_split(lng, dims)
    n = np.minimum(np.abs(u[..., 0, 1]) ** 2 + np.abs(u[..., 0, 2]) ** 2, np.abs(u[..., 2, 0]) ** 2)
    kap = 1.0 / n                                                   # [4, V]
    X, Y, Z, T = dims
    m = np.maximum(np.abs(psi_full.real), np.abs(psi_full.imag)).max(axis=1).reshape(T, Z, Y, X)
    tot = np.zeros((T, Z, Y, X))
    for mu in range(4):
        ax = 3 - mu
        k4 = kap[mu].reshape(T, Z, Y, X)
        tot += k4 * np.roll(m, -3, axis=ax)                         # L(x) psi(x + 3mu)
        tot += np.roll(k4 * m, 3, axis=ax)                          # L(x - 3mu)^dag psi(x - 3mu)
    return 3 * 1000 * 2.0 ** -52 * abs(c) * tot.reshape(-1)


@pytest.mark.parametrize("name", TRIPLETS8)
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 8, 4)])
def test_pack_recon8_bit_exact(name, dims):
    hisq = need_gpu()
    f = hisq.fmt(name)
    for kind in ("near_unit", "haar"):
        fat, lng = inputs.make_links(dims, kind, seed=inputs.GAUGE_SEED + 31)
        pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge, long_recon=hisq.RECON_8)
        assert pg.desc.long_recon == 8 and abs(pg.desc.long_coeff + 1 / 24) < 1e-14
        assert pg.desc.long_max == oracle.field_absmax(lng.numpy())
        assert pg.lng.numel() >= hisq.hisq_gauge_long_bytes(dims, f.gauge, 8) == 4 * oracle.volume(dims) * (
            64 if f.gauge == hisq.GAUGE_F64 else 32)
        got = long8_records(pg.lng.cpu().numpy(), dims, f.gauge)
        want = oracle.long_recon8_encode(lng.numpy(), dims, GF_NAME[f.gauge])
        if f.gauge == hisq.GAUGE_F64:
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), kind
        else:
            assert np.array_equal(got, want), kind


@pytest.mark.parametrize("name", TRIPLETS8)
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 8, 10, 12), (4, 6, 4, 8)])
def test_dslash_recon8(name, dims):
    hisq = need_gpu()
    f = hisq.fmt(name)
    for kind in ("near_unit", "haar"):
        fat, lng = inputs.make_links(dims, kind, seed=inputs.GAUGE_SEED + 32)
        V = oracle.volume(dims)
        psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 32).numpy()
        pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge, long_recon=hisq.RECON_8)
        for parity in (0, 1):
            src, dst = oracle.parity_sites(dims, 1 - parity), oracle.parity_sites(dims, parity)
            pin = hisq.pack_spinor(torch.from_numpy(psi[src]).cuda(), f.spinor)
            y = hisq.unpack_spinor(hisq.dslash(pin, pg, parity, f), dst.size, f.spinor).cpu().numpy()
            full = np.zeros_like(psi)
            full[src] = psi[src]
            ref = oracle.emulated_dslash(fat.numpy(), lng.numpy(), full, dims, parity, GF_NAME[f.gauge],
                                         SF_NAME[f.spinor], 64, long_recon=8)[dst]
            q = oracle.spinor_quantum(ref, SF_NAME[f.spinor])[:, None]
            bound = (0.5 * q * (1 + 1e-3) + 2e-13 * np.abs(ref).max()
                     + rebuild_allowance(lng.numpy(), full, dims)[dst][:, None])
            d = y - ref
            worst = float((np.maximum(np.abs(d.real), np.abs(d.imag)) / bound).max())
            assert worst <= 1.0, f"{name} {dims} {kind} parity {parity}: max err/bound {worst:.3f}"


def test_solvers_with_recon8_links():
    """CG with FIX32/INT30/FP64 sloppy links and an FP64 operator both stored
    as eight parameters, and the multi-shift CG with them as its operator,
    each to a 1e-10 true residual of the oracle's unquantised FP64 operator"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 12), 0.02
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 33)
    ev = oracle.parity_sites(dims, 0)
    b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED + 33).numpy()
    bd = torch.from_numpy(b).cuda()
    g64_8 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_F64, long_recon=hisq.RECON_8)
    g64 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_F64, long_recon=hisq.RECON_12)
    g32_8 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_FIX32, long_recon=hisq.RECON_8)
    g16 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_FIX16, long_recon=hisq.RECON_12)
    V = oracle.volume(dims)

    def resid(x, s=0.0):
        fx, fb = np.zeros((V, 3), complex), np.zeros((V, 3), complex)
        fx[ev], fb[ev] = x.cpu().numpy(), b
        return oracle.true_residual(fat.numpy(), lng.numpy(), fx, fb, dims, mass, shift=s)

    x, st = hisq.cg_solve(bd, g64_8, g32_8, mass, tol=1e-10, sloppy="int30")
    assert st["status"] == "HISQ_OK" and resid(x) <= 1e-10 * (1 + 1e-6), (st, resid(x))
    shifts = [0.0, 0.01, 0.1, 1.0]
    xs, sm = hisq.multishift_cg_solve(bd, shifts, 1e-10, g64, g32_8, g16, mass, ms_fmt="int30", ref_fmt="int20")
    assert sm["status"] == "HISQ_OK", sm
    for s, xv in zip(shifts, xs):
        assert resid(xv, s) <= 1e-10 * (1 + 1e-6), (s, resid(xv, s))


def test_recon8_rejections():
    hisq = need_gpu()
    dims = (4, 4, 4, 4)
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 34)
    for gf in (hisq.GAUGE_F32, hisq.GAUGE_FIX16, hisq.GAUGE_SX24):      # no eight-parameter storage
        with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
            hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, gf, long_recon=hisq.RECON_8)
    g8 = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, hisq.GAUGE_FIX32, long_recon=hisq.RECON_8)
    vh = oracle.volume(dims) // 2
    for name in ("int30_fp32", "int24"):                                  # FP32 arithmetic on FIX32 links
        f = hisq.fmt(name)
        pin = hisq.pack_spinor(inputs.gaussian_spinor(vh, 5, device="cuda"), f.spinor)
        with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
            hisq.dslash(pin, g8, 0, f)
    f = hisq.fmt("int30")
    nb = hisq.hisq_spinor_bytes(vh, f.spinor)
    pin = torch.cat([hisq.pack_spinor(inputs.gaussian_spinor(vh, 6 + j, device="cuda"), f.spinor)[:nb]
                     for j in range(4)]).contiguous()
    with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
        hisq.hisq_dslash_batched(torch.empty_like(pin), pin, g8.desc, 0, f, 4)
    with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
        hisq.hisq_dslash_multi([torch.empty_like(pin[:nb])], [pin[:nb]], [g8.desc], 0, f)
    with pytest.raises(hisq.HisqError, match="HISQ_EINVAL"):
        hisq.hisq_tune_set("int30", dims, 4, 4, 1, 1, 256, 0, long_recon=8)


@pytest.mark.parametrize("name", TRIPLETS8)
def test_full_size_sampled_recon8(name):
    """48^3x96 (the benchmark lattice) with the multi-shift operator's long-link
    storage, eight parameters, in the autotuned launch shape the benchmark
    times: sampled output sites against the oracle's emulation of the same
    storage, evaluated site by site, within the bound of test_dslash_recon8"""
    hisq = need_gpu()
    dims = (48, 48, 48, 96)
    V = oracle.volume(dims)
    X, Y, Z, T = dims
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 3, device="cuda")
    psi = inputs.gaussian_spinor(V // 2, inputs.SOURCE_SEED + 3, device="cuda")
    f = hisq.fmt(name)
    gname, sname = GF_NAME[f.gauge], SF_NAME[f.spinor]
    parity = 0
    out_sites, in_sites = oracle.parity_sites(dims, parity), oracle.parity_sites(dims, 1 - parity)
    rng = np.random.default_rng(2)
    samp_cb = np.unique(np.concatenate([rng.integers(0, V // 2, 3000), [0, V // 2 - 1]]))
    samp = out_sites[samp_cb]
    co = [samp % X, (samp // X) % Y, (samp // (X * Y)) % Z, samp // (X * Y * Z)]
    need_links, need_sp, long_hops = set(), set(), []
    for mu in range(4):
        for h in (1, -1, 3, -3):
            cc = [v.copy() for v in co]
            cc[mu] = (cc[mu] + h) % dims[mu]
            nb = ((cc[3] * Z + cc[2]) * Y + cc[1]) * X + cc[0]
            li = mu * V + (samp if h > 0 else nb)
            need_sp.update(nb.tolist())
            need_links.update(li.tolist())
            if abs(h) == 3:
                long_hops.append((li, nb))
    lidx, sidx = np.array(sorted(need_links)), np.array(sorted(need_sp))
    fat_h = fat.reshape(4 * V, 3, 3)[torch.from_numpy(lidx).cuda()].cpu().numpy()
    lng_h = lng.reshape(4 * V, 3, 3)[torch.from_numpy(lidx).cuda()].cpu().numpy()
    psi_h = psi[torch.from_numpy(np.searchsorted(in_sites, sidx)).cuda()].cpu().numpy()
    fmax = float(torch.view_as_real(fat).abs().amax())
    lmax = float(torch.view_as_real(lng).abs().amax())
    c = -1.0 / 24.0                                           # the generator's long-link constant
    pg = hisq.pack_gauge(fat, lng, dims, f.gauge, long_recon=hisq.RECON_8)
    assert abs(pg.desc.long_coeff - c) < 1e-14 and pg.desc.long_max == lmax
    pin = hisq.pack_spinor(psi, f.spinor)
    y = hisq.unpack_spinor(hisq.dslash(pin, pg, parity, f), V // 2, f.spinor)
    y = y[torch.from_numpy(samp_cb).cuda()].cpu().numpy()
    del pg, pin, fat, lng, psi
    torch.cuda.empty_cache()
    full_fat = np.zeros((4 * V, 3, 3), dtype=np.complex128)   # lazily allocated; only touched entries used
    full_lng = np.zeros((4 * V, 3, 3), dtype=np.complex128)
    full_psi = np.zeros((V, 3), dtype=np.complex128)
    if gname == "fix32":
        qf, _ = oracle.fix_encode(fat_h, 32, absmax=fmax)
        full_fat[lidx] = oracle.fix_decode(qf, fmax, 64, shape=fat_h.shape)
    else:
        full_fat[lidx] = oracle.gauge_roundtrip(fat_h, gname, 64)
    ph = oracle.long_phases(dims).reshape(4 * V)[lidx]
    full_lng[lidx] = oracle.long8_links_roundtrip(lng_h, ph, c, lmax, gname)
    full_psi[sidx] = oracle.spinor_roundtrip(psi_h, sname)
    ref = oracle.dslash_sites(full_fat.reshape(4, V, 3, 3), full_lng.reshape(4, V, 3, 3), full_psi, dims, samp)
    # the FP64 rebuild's rounding, amplified by kappa of each long link, per sampled site
    u = lng_h / (c * ph)[:, None, None]
    kap = 1.0 / np.minimum(np.abs(u[:, 0, 1]) ** 2 + np.abs(u[:, 0, 2]) ** 2, np.abs(u[:, 2, 0]) ** 2)
    allow = np.zeros(samp.size)
    for li, nb in long_hops:
        m = np.maximum(np.abs(full_psi[nb].real), np.abs(full_psi[nb].imag)).max(axis=1)
        allow += kap[np.searchsorted(lidx, li)] * m
    allow *= 3 * 1000 * 2.0 ** -52 * abs(c)
    q = oracle.spinor_quantum(ref, sname)[:, None]
    bound = 0.5 * q * (1 + 1e-3) + 2e-13 * np.abs(ref).max() + allow[:, None]
    d = y - ref
    worst = float((np.maximum(np.abs(d.real), np.abs(d.imag)) / bound).max())
    assert worst <= 1.0, f"{name}: max err/bound {worst:.3f}"
