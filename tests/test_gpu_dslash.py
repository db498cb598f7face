"""HIP Dslash against the FP64 oracle, element by element.

Reference for a triplet gauge/fermion/compute: the oracle's FP64 Dslash of
the inputs exactly as the storage formats hold them (links and spinor after
an encode/decode round trip in the oracle's own codecs).  The kernel then
differs from it only by (a) its own rounding in the compute precision and
(b) the quantisation of the packed output, so per component
  |y_gpu - y_ref| <= q_site/2 * (1 + 1e-3) + eps_c * max|y_ref|
with q_site the output format's quantum at that site and eps_c = 1e-6 for
FP32 compute (the FP32 tolerance of the Dslash, 16 mat-vecs of O(1)
entries) and 1e-13 for FP64 compute.
Pure FP64 and FP32 triplets are also checked against the unquantised FP64
oracle at the tolerances 1e-13 and 1e-6 (max-norm relative).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import format_bounds, need_gpu, rel_inf
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

TRIPLETS = ["double", "single", "half", "int20", "int30", "int30_fp32", "int24", "sx24", "sx24_int30"]
SF_NAME = {0: "f64", 1: "f32", 2: "half16", 3: "int20", 4: "int30", 5: "int24"}
GF_NAME = {0: "f64", 1: "f32", 2: "fix16", 3: "fix32", 4: "sx24"}
# 4^4: x+3mu and x-mu coincide; (6,8,10,12): Vh = 2880, a ragged last block;
# (8,8,8,8): Vh = 2048, whole blocks; (4,6,4,8) non-cubic
DIMS = [(4, 4, 4, 4), (6, 8, 10, 12), (8, 8, 8, 8), (4, 6, 4, 8)]
_cache = {}


def fields(dims, kind):
    key = (dims, kind)
    if key not in _cache:
        fat, lng = inputs.make_links(dims, kind, seed=inputs.GAUGE_SEED + 7)
        V = oracle.volume(dims)
        psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 7).numpy()
        psi[::53] = 0.0                                   # some all-zero sites
        _cache[key] = (fat, lng, psi)
    return _cache[key]


def eps_c(compute):
    return 1e-6 if compute == 32 else 1e-13


def check_against_emulation(hisq, name, dims, kind, parity):
    f = hisq.fmt(name)
    fat, lng, psi = fields(dims, kind)
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    src_sites = oracle.parity_sites(dims, 1 - parity)
    out_sites = oracle.parity_sites(dims, parity)
    pin = hisq.pack_spinor(torch.from_numpy(psi[src_sites]).cuda(), f.spinor)
    pout = hisq.dslash(pin, pg, parity, f)
    y = hisq.unpack_spinor(pout, out_sites.size, f.spinor).cpu().numpy()
    psi_in = np.zeros_like(psi)
    psi_in[src_sites] = psi[src_sites]
    ref = oracle.emulated_dslash(fat.numpy(), lng.numpy(), psi_in, dims, parity,
                                 GF_NAME[f.gauge], SF_NAME[f.spinor], f.compute)[out_sites]
    q = oracle.spinor_quantum(ref, SF_NAME[f.spinor])[:, None]
    bound = 0.5 * q * (1 + 1e-3) + eps_c(f.compute) * np.abs(ref).max()
    d = y - ref
    err = np.maximum(np.abs(d.real), np.abs(d.imag))
    worst = float((err / bound).max())
    assert worst <= 1.0, f"{name} {dims} {kind} parity {parity}: max err/bound {worst:.3f}"
    return y, ref


@pytest.mark.parametrize("name", TRIPLETS)
@pytest.mark.parametrize("dims", DIMS)
def test_dslash_triplet(name, dims):
    hisq = need_gpu()
    for kind in ("near_unit", "haar"):
        for parity in (0, 1):
            check_against_emulation(hisq, name, dims, kind, parity)


@pytest.mark.parametrize("name,tol", [("double", 1e-13), ("single", 1e-6)])
def test_ieee_triplets_vs_pure_fp64(name, tol):
    hisq = need_gpu()
    dims = (6, 8, 10, 12)
    f = hisq.fmt(name)
    fat, lng, psi = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    for parity in (0, 1):
        src, dst = oracle.parity_sites(dims, 1 - parity), oracle.parity_sites(dims, parity)
        pin = hisq.pack_spinor(torch.from_numpy(psi[src]).cuda(), f.spinor)
        y = hisq.unpack_spinor(hisq.dslash(pin, pg, parity, f), dst.size, f.spinor).cpu().numpy()
        full = np.zeros_like(psi)
        full[src] = psi[src]
        ref = oracle.dslash(fat.numpy(), lng.numpy(), full, dims, parity)[dst]
        assert rel_inf(y, ref) <= tol


@pytest.mark.parametrize("name", ["double", "single", "half"])
def test_xpay(name):
    hisq = need_gpu()
    dims = (6, 8, 10, 12)
    f = hisq.fmt(name)
    fat, lng, psi = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    parity = 0
    src, dst = oracle.parity_sites(dims, 1), oracle.parity_sites(dims, 0)
    xv = inputs.gaussian_spinor(dst.size, 99).numpy()
    pin = hisq.pack_spinor(torch.from_numpy(psi[src]).cuda(), f.spinor)
    px = hisq.pack_spinor(torch.from_numpy(xv).cuda(), f.spinor)
    out = torch.empty_like(px)
    a, b = 0.37, -1.25
    hisq.hisq_dslash_xpay(out, pin, pg.desc, parity, f, a, px, b)
    y = hisq.unpack_spinor(out, dst.size, f.spinor).cpu().numpy()
    full = np.zeros_like(psi)
    full[src] = psi[src]
    ref = a * oracle.spinor_roundtrip(xv, SF_NAME[f.spinor]) + b * oracle.emulated_dslash(
        fat.numpy(), lng.numpy(), full, dims, parity, GF_NAME[f.gauge], SF_NAME[f.spinor], f.compute)[dst]
    q = oracle.spinor_quantum(ref, SF_NAME[f.spinor])[:, None]
    bound = 0.5 * q * (1 + 1e-3) + 2 * eps_c(f.compute) * np.abs(ref).max()
    d = y - ref
    assert (np.maximum(np.abs(d.real), np.abs(d.imag)) <= bound).all()


@pytest.mark.parametrize("name", ["single", "int20"])
def test_xpay_in_place_on_first_application(name):
    """out = a*out + b*D(in) with out == x, on the first application of its
    launch-shape key (the autotuner times its candidates then; they must not
    write the caller's output, which is also the x operand)"""
    hisq = need_gpu()
    dims = (6, 8, 10, 12)
    f = hisq.fmt(name)
    fat, lng, psi = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    src, dst = oracle.parity_sites(dims, 1), oracle.parity_sites(dims, 0)
    xv = inputs.gaussian_spinor(dst.size, 98).numpy()
    pin = hisq.pack_spinor(torch.from_numpy(psi[src]).cuda(), f.spinor)
    px = hisq.pack_spinor(torch.from_numpy(xv).cuda(), f.spinor)
    a, b = -0.61, 0.83
    hisq.hisq_tune_clear()
    hisq.hisq_dslash_xpay(px, pin, pg.desc, 0, f, a, px, b)
    assert "lattice 6x8x10x12 rhs-block 1" in hisq.hisq_tune_report()
    y = hisq.unpack_spinor(px, dst.size, f.spinor).cpu().numpy()
    full = np.zeros_like(psi)
    full[src] = psi[src]
    ref = a * oracle.spinor_roundtrip(xv, SF_NAME[f.spinor]) + b * oracle.emulated_dslash(
        fat.numpy(), lng.numpy(), full, dims, 0, GF_NAME[f.gauge], SF_NAME[f.spinor], f.compute)[dst]
    q = oracle.spinor_quantum(ref, SF_NAME[f.spinor])[:, None]
    bound = 0.5 * q * (1 + 1e-3) + 2 * eps_c(f.compute) * np.abs(ref).max()
    d = y - ref
    assert (np.maximum(np.abs(d.real), np.abs(d.imag)) <= bound).all()


def test_tune_cache_file_round_trip(tmp_path):
    """shapes saved, cleared and loaded again give the same table and the same
    results; HISQ_TUNE_CACHE appends every newly tuned shape"""
    import os
    hisq = need_gpu()
    dims = (8, 8, 8, 8)
    f = hisq.fmt("int20")
    fat, lng, psi = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    src = oracle.parity_sites(dims, 1)
    pin = hisq.pack_spinor(torch.from_numpy(psi[src]).cuda(), f.spinor)
    cache = tmp_path / "tune.txt"
    hisq.hisq_tune_clear()
    os.environ["HISQ_TUNE_CACHE"] = str(cache)
    try:
        y0 = hisq.dslash(pin, pg, 0, f).cpu()
    finally:
        del os.environ["HISQ_TUNE_CACHE"]
    lines = [ln for ln in cache.read_text().splitlines() if ln.startswith("hisq-tune")]
    assert len(lines) == 1 and " 8 8 8 8 1 0 : " in lines[0]
    rep = hisq.hisq_tune_report()
    saved = tmp_path / "saved.txt"
    hisq.hisq_tune_save(saved)
    hisq.hisq_tune_clear()
    assert hisq.hisq_tune_report() == ""
    assert hisq.hisq_tune_load(saved) == 1
    shape = lambda r: r.split(": ", 1)[1].split(" (")[0]          # noqa: E731
    assert shape(hisq.hisq_tune_report()) == shape(rep)
    y1 = hisq.dslash(pin, pg, 0, f).cpu()
    assert torch.equal(y0, y1)
    # a line for another architecture is skipped; a malformed line loads nothing
    other = tmp_path / "other.txt"
    other.write_text(lines[0].replace("hisq-tune 1 gfx950", "hisq-tune 1 gfx000") + "\n")
    assert hisq.hisq_tune_load(other) == 0
    bad = tmp_path / "bad.txt"
    bad.write_text(lines[0] + "\nhisq-tune 1 gfx950 garbage\n")
    hisq.hisq_tune_clear()
    with pytest.raises(hisq.HisqError, match="HISQ_EIO"):
        hisq.hisq_tune_load(bad)
    assert hisq.hisq_tune_report() == ""
    hisq.hisq_tune_clear()


_PIN_CHILD = """
import sys, torch
sys.path.insert(0, {root!r})
from paper_2302_09224_amd import hisq, inputs
dims = (8, 8, 8, 8)
f = hisq.fmt("int20")
if {pin}:
    hisq.hisq_tune_set(f, dims, 1, 1, 1, 2, 256, 0, sweep=1)
fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED, device="cuda")
pg = hisq.pack_gauge(fat, lng, dims, f.gauge)
pin = hisq.pack_spinor(inputs.gaussian_spinor(2048, 5, device="cuda"), f.spinor)
hisq.dslash(pin, pg, 0, f)
torch.cuda.synchronize()
print("REPORT " + hisq.hisq_tune_report().strip().replace(chr(10), " | "), flush=True)
"""


def test_tune_cache_keeps_pinned_shapes(tmp_path):
    """HISQ_TUNE_CACHE is read at the first shape lookup of a process: it fills
    the keys without a shape, and a shape fixed before (hisq_tune_set) stays.
    Each case runs in a fresh process, since the file is read once per process."""
    import os
    import subprocess
    import sys
    hisq = need_gpu()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    dims = (8, 8, 8, 8)
    f = hisq.fmt("int20")
    cache = tmp_path / "tune.txt"
    hisq.hisq_tune_clear()
    try:
        hisq.hisq_tune_set(f, dims, 1, 1, 1, 1, 128, 0, sweep=0)     # the file's shape: stage 1, block 128
        hisq.hisq_tune_save(cache)
    finally:
        hisq.hisq_tune_clear()
    env = dict(os.environ, HISQ_TUNE_CACHE=str(cache))
    shapes = {}
    for pin in (False, True):
        print(f"child process, pinned {pin}", flush=True)
        r = subprocess.run([sys.executable, "-c", _PIN_CHILD.format(root=root, pin=pin)], env=env,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        rep = [ln for ln in r.stdout.splitlines() if ln.startswith("REPORT ")][0]
        shapes[pin] = rep
    assert "stage 1 block 128 grid 0 sweep 0" in shapes[False], shapes[False]
    assert "stage 2 block 256 grid 0 sweep 1" in shapes[True], shapes[True]


@pytest.mark.parametrize("name", ["double", "single", "int30", "int20", "half", "int24", "sx24", "sx24_int30"])
def test_normal_op(name):
    """(4m^2+s) p - D_eo D_oe p; the intermediate D_oe p is stored in the
    sloppy format, so the bound is the format's precision (max-norm relative):
    FP64 and FP32 rounding of two applications for the IEEE triplets, the
    oracle-derived bound of golden/format_bounds.txt for the others"""
    tol = {"double": 1e-13, "single": 2e-6}.get(name) or format_bounds()[name][1]
    hisq = need_gpu()
    dims = (6, 8, 10, 12)
    f = hisq.fmt(name)
    fat, lng, psi = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    ev = oracle.parity_sites(dims, 0)
    p = psi[ev]
    pin = hisq.pack_spinor(torch.from_numpy(p).cuda(), f.spinor)
    out = torch.empty_like(pin)
    tmp = torch.empty_like(pin)
    mass, shift = 0.05, 0.01
    hisq.hisq_normal_op(out, pin, tmp, pg.desc, mass, shift, f)
    y = hisq.unpack_spinor(out, ev.size, f.spinor).cpu().numpy()
    full = np.zeros_like(psi)
    full[ev] = p
    ref = oracle.normal_op(fat.numpy(), lng.numpy(), full, dims, mass, shift)[ev]
    assert rel_inf(y, ref) <= tol


@pytest.mark.parametrize("name", ["double", "single", "half", "int20", "int30", "int24", "sx24", "sx24_int30"])
@pytest.mark.parametrize("nrhs", [1, 3, 16])
def test_batched_matches_single(name, nrhs):
    """one link load for a block of right-hand sides gives every right-hand
    side the same result as its own Dslash"""
    hisq = need_gpu()
    dims = (6, 8, 10, 12)
    f = hisq.fmt(name)
    fat, lng, _ = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    odd = oracle.parity_sites(dims, 1)
    vh = odd.size
    srcs = inputs.gaussian_spinor(vh, 500, nrhs=nrhs).numpy()
    packed = [hisq.pack_spinor(torch.from_numpy(srcs[j]).cuda(), f.spinor) for j in range(nrhs)]
    nb = hisq.hisq_spinor_bytes(vh, f.spinor)
    pin = torch.cat([pk[:nb] for pk in packed]).contiguous()
    pout = torch.empty_like(pin)
    hisq.hisq_dslash_batched(pout, pin, pg.desc, 0, f, nrhs)
    for j in range(nrhs):
        single = hisq.dslash(packed[j], pg, 0, f)
        yb = hisq.unpack_spinor(pout[j * nb:(j + 1) * nb].contiguous(), vh, f.spinor).cpu().numpy()
        ys = hisq.unpack_spinor(single, vh, f.spinor).cpu().numpy()
        q = oracle.spinor_quantum(ys, SF_NAME[f.spinor])[:, None]
        d = yb - ys
        assert (np.maximum(np.abs(d.real), np.abs(d.imag)) <= q + eps_c(f.compute) * np.abs(ys).max()).all()


@pytest.mark.parametrize("name,shape", [("int20", (1, 16, 1)), ("int20", (4, 4, 1)), ("int20", (16, 1, 1)),
                                        ("int20", (4, 4, 5)), ("half", (2, 8, 1)), ("sx24_int30", (4, 4, 1))])
def test_batched_padding_columns_untouched(name, shape):
    """11 right-hand sides in a block of 16: the five padding columns are
    neither written (a sentinel after the last field survives) nor change the
    live ones, for several lane layouts (nr, rg, stage; stage 5 = matrix cores)"""
    hisq = need_gpu()
    dims, nrhs = (6, 8, 10, 12), 11
    f = hisq.fmt(name)
    fat, lng, _ = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge)
    vh = oracle.parity_sites(dims, 1).size
    srcs = inputs.gaussian_spinor(vh, 510, nrhs=nrhs).numpy()
    packed = [hisq.pack_spinor(torch.from_numpy(srcs[j]).cuda(), f.spinor) for j in range(nrhs)]
    nb = hisq.hisq_spinor_bytes(vh, f.spinor)
    pin = torch.cat([pk[:nb] for pk in packed]).contiguous()
    pout = torch.full((16 * nb,), 0xA5, dtype=torch.uint8, device="cuda")
    hisq.hisq_tune_clear()
    try:
        hisq.hisq_tune_set(name, dims, 16, shape[0], shape[1], shape[2], 256, 0)
        hisq.hisq_dslash_batched(pout, pin, pg.desc, 0, f, nrhs)
        torch.cuda.synchronize()
    finally:
        hisq.hisq_tune_clear()
    assert bool((pout[nrhs * nb:] == 0xA5).all()), "a padding column was written"
    for j in range(nrhs):
        single = hisq.dslash(packed[j], pg, 0, f)
        yb = hisq.unpack_spinor(pout[j * nb:(j + 1) * nb].contiguous(), vh, f.spinor).cpu().numpy()
        ys = hisq.unpack_spinor(single, vh, f.spinor).cpu().numpy()
        q = oracle.spinor_quantum(ys, SF_NAME[f.spinor])[:, None]
        d = yb - ys
        assert (np.maximum(np.abs(d.real), np.abs(d.imag)) <= q + eps_c(f.compute) * np.abs(ys).max()).all(), j


# every lane layout the autotuner may choose for a block of 16 right-hand
# sides: (nr, rg, stage) with stage 5 the matrix-core path (FP32 compute
# only), and (grid, sweep) for tile-per-block and persistent grids in the
# three tile orders
SHAPES_16 = [((1, 16, 1), (0, 1)), ((1, 16, 2), (0, 1)), ((2, 8, 1), (0, 1)), ((4, 4, 1), (0, 1)),
             ((4, 4, 1), (2048, 0)), ((8, 2, 1), (0, 1)), ((16, 1, 1), (0, 1)), ((16, 1, 1), (2048, 0)),
             ((4, 4, 5), (0, 1)), ((4, 4, 5), (2048, 0)), ((1, 16, 1), (0, 2)), ((4, 4, 1), (0, 2)),
             ((16, 1, 1), (2048, 2)), ((4, 4, 5), (0, 2))]


@pytest.mark.parametrize("recon", [18, 12])
@pytest.mark.parametrize("name", ["double", "single", "half", "int20", "int30", "int24", "sx24", "sx24_int30"])
def test_batched_shapes_vs_emulation(name, recon):
    """13 right-hand sides (a block of 16 with padding) at 16^4 in every lane
    layout, each column against the oracle's format emulation element by
    element, at the bound of check_against_emulation"""
    hisq = need_gpu()
    dims, nrhs = (16, 16, 16, 16), 13
    f = hisq.fmt(name)
    gf, sf = GF_NAME[f.gauge], SF_NAME[f.spinor]
    fat, lng, _ = fields(dims, "near_unit")
    pg = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, f.gauge, long_recon=recon)
    ev, od = oracle.parity_sites(dims, 0), oracle.parity_sites(dims, 1)
    srcs = inputs.gaussian_spinor(od.size, 520, nrhs=nrhs).numpy()
    srcs[3, ::37] = 0.0                                         # all-zero sites in one column
    nb = hisq.hisq_spinor_bytes(od.size, f.spinor)
    pin = torch.cat([hisq.pack_spinor(torch.from_numpy(srcs[j]).cuda(), f.spinor)[:nb]
                     for j in range(nrhs)]).contiguous()
    fq = oracle.gauge_roundtrip(fat.numpy(), gf, f.compute)
    lq = (oracle.long_recon_roundtrip(lng.numpy(), dims, gf, f.compute) if recon == 12
          else oracle.gauge_roundtrip(lng.numpy(), gf, f.compute))
    refs = [oracle.dslash(fq, lq, oracle.to_full(oracle.spinor_roundtrip(srcs[j], sf), dims, 1), dims, 0)[ev]
            for j in range(nrhs)]
    try:
        for (nr, rg, stage), (grid, sweep) in SHAPES_16:
            if stage == 5 and f.compute != 32:
                continue
            hisq.hisq_tune_set(name, dims, 16, nr, rg, stage, 256, grid, sweep=sweep, long_recon=recon)
            pout = torch.empty_like(pin)
            hisq.hisq_dslash_batched(pout, pin, pg.desc, 0, f, nrhs)
            for j in range(nrhs):
                y = hisq.unpack_spinor(pout[j * nb:(j + 1) * nb].contiguous(), ev.size, f.spinor).cpu().numpy()
                q = oracle.spinor_quantum(refs[j], sf)[:, None]
                bound = 0.5 * q * (1 + 1e-3) + eps_c(f.compute) * np.abs(refs[j]).max()
                d = y - refs[j]
                worst = float((np.maximum(np.abs(d.real), np.abs(d.imag)) / bound).max())
                assert worst <= 1.0, (name, recon, nr, rg, stage, grid, j, worst)
    finally:
        hisq.hisq_tune_clear()


@pytest.mark.parametrize("recon", [18, 12])
def test_full_size_sampled(recon):
    """48^3x96 (the benchmark lattice), launch configuration of the benchmark
    (autotuned shapes; the benchmark's solvers use two-row long links): sampled
    output sites against the oracle evaluated site by site"""
    hisq = need_gpu()
    dims = (48, 48, 48, 96)
    V = oracle.volume(dims)
    fat, lng = inputs.make_links(dims, "near_unit", seed=inputs.GAUGE_SEED + 3, device="cuda")
    psi = inputs.gaussian_spinor(V // 2, inputs.SOURCE_SEED + 3, device="cuda")
    rng = np.random.default_rng(1)
    parity = 0
    out_sites = oracle.parity_sites(dims, parity)
    odd_sites = oracle.parity_sites(dims, 1)
    samp_cb = np.unique(np.concatenate([rng.integers(0, V // 2, 3000), [0, V // 2 - 1]]))
    samp = out_sites[samp_cb]
    # every link and neighbour the sampled sites touch, gathered on the device
    X, Y, Z, T = dims
    c = [samp % X, (samp // X) % Y, (samp // (X * Y)) % Z, samp // (X * Y * Z)]
    need_links, need_sp = set(), set()
    for mu in range(4):
        for h in (1, -1, 3, -3):
            cc = [v.copy() for v in c]
            cc[mu] = (cc[mu] + h) % dims[mu]
            nb = ((cc[3] * Z + cc[2]) * Y + cc[1]) * X + cc[0]
            need_sp.update(nb.tolist())
            if h > 0:
                need_links.update((mu * V + samp).tolist())
            else:
                need_links.update((mu * V + nb).tolist())
    lidx = np.array(sorted(need_links))
    sidx = np.array(sorted(need_sp))
    full_fat = np.zeros((4 * V, 3, 3), dtype=np.complex128)   # lazily allocated; only touched entries used
    full_lng = np.zeros((4 * V, 3, 3), dtype=np.complex128)
    full_psi = np.zeros((V, 3), dtype=np.complex128)
    fat_h = fat.reshape(4 * V, 3, 3)[torch.from_numpy(lidx).cuda()].cpu().numpy()
    lng_h = lng.reshape(4 * V, 3, 3)[torch.from_numpy(lidx).cuda()].cpu().numpy()
    pos = np.searchsorted(odd_sites, sidx)                     # cb index of each needed odd site
    psi_h = psi[torch.from_numpy(pos).cuda()].cpu().numpy()
    fmax = float(torch.view_as_real(fat).abs().amax())
    lmax = float(torch.view_as_real(lng).abs().amax())
    if recon == 12:
        # the stored rows of U = L / (c * phase), c = -1/24 for these links; their scale is max |U|
        ph = torch.from_numpy(oracle.long_phases(dims)).cuda().reshape(4, V, 1, 1)
        U = lng / (-1.0 / 24.0 * ph)
        umax = float(torch.view_as_real(U).abs().amax())
        del U
        u_h = lng_h / (-1.0 / 24.0 * oracle.long_phases(dims).reshape(4 * V)[lidx, None, None])
    for name in ("half", "int20", "int30", "int24", "sx24", "single", "double"):
        f = hisq.fmt(name)
        pg = hisq.pack_gauge(fat, lng, dims, f.gauge, long_recon=recon)
        pin = hisq.pack_spinor(psi, f.spinor)
        y = hisq.unpack_spinor(hisq.dslash(pin, pg, parity, f), V // 2, f.spinor)[torch.from_numpy(samp_cb).cuda()]
        y = y.cpu().numpy()
        del pg, pin
        gname, sname = GF_NAME[f.gauge], SF_NAME[f.spinor]
        if gname in ("fix16", "fix32"):
            bits = 16 if gname == "fix16" else 32
            qf, _ = oracle.fix_encode(fat_h, bits, absmax=fmax)
            full_fat[lidx] = oracle.fix_decode(qf, fmax, f.compute, shape=fat_h.shape)
            if recon == 18:
                ql, _ = oracle.fix_encode(lng_h, bits, absmax=lmax)
                full_lng[lidx] = oracle.fix_decode(ql, lmax, f.compute, shape=lng_h.shape)
        else:
            full_fat[lidx] = oracle.gauge_roundtrip(fat_h, gname, f.compute)
            if recon == 18:
                full_lng[lidx] = oracle.gauge_roundtrip(lng_h, gname, f.compute)
        if recon == 12:
            # two stored rows in the format, the third rebuilt, times c * phase (the oracle's reading)
            rows = np.ascontiguousarray(u_h[:, :2, :])
            if gname in ("fix16", "fix32"):
                q, _ = oracle.fix_encode(rows, 16 if gname == "fix16" else 32, absmax=umax)
                rows = oracle.fix_decode(q, umax, f.compute, shape=rows.shape)
            elif gname == "sx24":
                rows = oracle.gauge_roundtrip(rows, "sx24", f.compute)
            elif gname == "f32" or f.compute == 32:
                rows = rows.astype(np.complex64).astype(np.complex128)
            full3 = np.concatenate([rows, oracle.su3_third_row(rows)[:, None, :]], axis=1)
            full_lng[lidx] = (-1.0 / 24.0) * oracle.long_phases(dims).reshape(4 * V)[lidx, None, None] * full3
        full_psi[sidx] = oracle.spinor_roundtrip(psi_h, sname)
        ref = oracle.dslash_sites(full_fat.reshape(4, V, 3, 3), full_lng.reshape(4, V, 3, 3), full_psi, dims, samp)
        q = oracle.spinor_quantum(ref, sname)[:, None]
        bound = 0.5 * q * (1 + 1e-3) + (2 if recon == 12 else 1) * eps_c(f.compute) * np.abs(ref).max()
        d = y - ref
        worst = float((np.maximum(np.abs(d.real), np.abs(d.imag)) / bound).max())
        assert worst <= 1.0, f"{name} recon {recon}: max err/bound {worst:.3f}"
        torch.cuda.empty_cache()
