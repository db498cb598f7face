"""HIP solvers against the oracle: the solution of (4m^2 + s - D_eo D_oe) x = b
is unique, so every mixed-precision solve must reach the requested true
residual (measured by the oracle's FP64 operator) and agree with the
oracle's FP64 solve to the accuracy the condition number allows."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import need_gpu
from paper_2302_09224_amd import inputs

pytestmark = pytest.mark.gpu

_cache = {}


def setup(dims, kind, seed=inputs.GAUGE_SEED):
    key = (dims, kind, seed)
    if key not in _cache:
        fat, lng = inputs.make_links(dims, kind, seed)
        ev = oracle.parity_sites(dims, 0)
        b = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED).numpy()
        _cache[key] = (fat, lng, ev, b)
    return _cache[key]


def packed(hisq, fat, lng, dims, names):
    out = {}
    for n in names:
        g = hisq.fmt(n).gauge
        if g not in out:
            out[g] = hisq.pack_gauge(fat.cuda(), lng.cuda(), dims, g)
    return out


def full(dims, ev, v):
    f = np.zeros((oracle.volume(dims), 3), dtype=np.complex128)
    f[ev] = v
    return f


def test_cg_config0_dense():
    """4^4 rough links, m = 0.1, FP64 CG against a dense LAPACK solve"""
    hisq = need_gpu()
    import pins
    dims, mass = (4, 4, 4, 4), 0.1
    fat, lng, ev, b = setup(dims, "haar")
    pg = packed(hisq, fat, lng, dims, ["double"])
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), pg[0], pg[0], mass, tol=1e-10, sloppy="double")
    x = x.cpu().numpy()
    A = pins.dense_normal(fat.numpy(), lng.numpy(), dims, mass)
    xd = np.linalg.solve(A, b.ravel())
    assert st["status"] == "HISQ_OK"
    assert np.linalg.norm(x.ravel() - xd) / np.linalg.norm(xd) < 1e-8
    assert oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x), full(dims, ev, b), dims, mass) <= 1e-10


@pytest.mark.parametrize("sloppy", ["double", "single", "half", "int20", "int30", "int30_fp32", "int24", "sx24",
                                    "sx24_int30"])
@pytest.mark.parametrize("dims,kind,mass", [((8, 8, 8, 8), "near_unit", 0.05), ((6, 8, 10, 12), "haar", 0.2)])
def test_cg_mixed(sloppy, dims, kind, mass):
    hisq = need_gpu()
    fat, lng, ev, b = setup(dims, kind)
    pg = packed(hisq, fat, lng, dims, ["double", sloppy])
    gs = pg[hisq.fmt(sloppy).gauge]
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), pg[0], gs, mass, tol=1e-10, sloppy=sloppy)
    x = x.cpu().numpy()
    assert st["status"] == "HISQ_OK", st
    res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x), full(dims, ev, b), dims, mass)
    assert res <= 1e-10 * (1 + 1e-6), (res, st)
    assert abs(res - st["true_resid"]) <= 1e-3 * res + 1e-15
    xo, it, ores, _ = oracle.cg(fat.numpy(), lng.numpy(), full(dims, ev, b), dims, mass, tol=1e-12)
    assert np.linalg.norm(x - xo[ev]) / np.linalg.norm(xo[ev]) < 1e-8


@pytest.mark.parametrize("opts", [dict(grad_buffer=1), dict(grad_buffer=8), dict(use_graph=0),
                                  dict(pr_beta=0), dict(reproject=0), dict(poll_every=3, grad_buffer=2),
                                  dict(delta=0.5)])
def test_cg_options(opts):
    hisq = need_gpu()
    dims, mass = (6, 8, 10, 12), 0.1
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "half"])
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), pg[0], pg[2], mass, tol=1e-10, sloppy="half", **opts)
    res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x.cpu().numpy()), full(dims, ev, b), dims, mass)
    assert st["status"] == "HISQ_OK" and res <= 1e-10 * (1 + 1e-6), (opts, st, res)


def test_cg_initial_guess_and_zero_rhs():
    hisq = need_gpu()
    dims, mass = (6, 8, 10, 12), 0.1
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "single"])
    xo, *_ = oracle.cg(fat.numpy(), lng.numpy(), full(dims, ev, b), dims, mass, tol=1e-13)
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), pg[0], pg[1], mass, tol=1e-10, sloppy="single",
                          x0=torch.from_numpy(xo[ev]).cuda())
    assert st["status"] == "HISQ_OK" and st["iters"] == 0
    z = torch.zeros((ev.size, 3), dtype=torch.complex128, device="cuda")
    x, st = hisq.cg_solve(z, pg[0], pg[1], mass, tol=1e-10, sloppy="single")
    assert st["status"] == "HISQ_OK" and float(x.abs().max()) == 0.0


def test_cg_maxiter_reports_noconv():
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.01
    fat, lng, ev, b = setup(dims, "haar")
    pg = packed(hisq, fat, lng, dims, ["double", "single"])
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), pg[0], pg[1], mass, tol=1e-12, sloppy="single", maxiter=5)
    assert st["status"] == "HISQ_ENOCONV" and st["iters"] >= 5
    res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x.cpu().numpy()), full(dims, ev, b), dims, mass)
    assert abs(res - st["true_resid"]) <= 1e-6 * res


@pytest.mark.parametrize("ms,ref,batch", [("single", "half", 1), ("int30", "int20", 1), ("double", "double", 1),
                                          ("single", "single", 1), ("int30", "int20", 0), ("single", "half", 0),
                                          ("int30", "int30_fp32", 1), ("int30", "int24", 1),
                                          ("sx24_int30", "int20", 1), ("int30", "int20", 2), ("single", "half", 2),
                                          ("int30", "int30_fp32", 2), ("int30", "int20", 3), ("single", "half", 3),
                                          ("int30", "int30_fp32", 3)])
def test_multishift(ms, ref, batch):
    """batch: refine the shifted systems together (1), together while the
    base is refined concurrently (2), together with the base continuing its
    gradient vector in the same block (3), or one after another (0);
    int30_fp32 has no batched form, so it refines one after another either way"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    shifts = [1e-4, 1e-3, 1e-2, 0.1, 1.0, 10.0]
    tol = [1e-10] * len(shifts)
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", ms, ref])
    xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, tol, pg[0], pg[hisq.fmt(ms).gauge],
                                      pg[hisq.fmt(ref).gauge], mass, ms_fmt=ms, ref_fmt=ref, batch_refine=batch)
    assert st["status"] == "HISQ_OK", st
    out = oracle.multishift_cg(fat.numpy(), lng.numpy(), full(dims, ev, b), dims, mass, shifts, 1e-12)
    for i, s in enumerate(shifts):
        x = xs[i].cpu().numpy()
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x), full(dims, ev, b), dims, mass, s)
        assert res <= tol[i] * (1 + 1e-6), (i, res, st)
        xo = out["x"][i][ev]
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8


@pytest.mark.parametrize("ms,ref", [("double", "double"), ("single", "half")])
def test_multishift_block_size_invariance(ms, ref):
    """The shifted systems are updated once per block of grad_buffer
    iterations, replaying the block's recurrences from its base residuals; with
    IEEE storage of the multi-shift vectors (nothing is quantised between
    iterations) the arithmetic and its order do not depend on where the blocks
    end.  So the solutions, iterations and reliable updates are bit-identical
    for every block size, chunk length (where the host looks) and with or
    without graph replay, also when shifts stop and reliable updates fall
    inside a block."""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.02
    shifts = [1e-4, 1e-3, 1e-2, 0.1, 1.0, 10.0]
    tol = [1e-10, 1e-9, 1e-10, 1e-8, 1e-10, 1e-11]
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", ms, ref])
    runs = []
    for opts in (dict(grad_buffer=8), dict(grad_buffer=1), dict(grad_buffer=3, poll_every=7),
                 dict(grad_buffer=16), dict(grad_buffer=5, use_graph=0)):
        xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, tol, pg[0], pg[hisq.fmt(ms).gauge],
                                          pg[hisq.fmt(ref).gauge], mass, ms_fmt=ms, ref_fmt=ref, **opts)
        assert st["status"] == "HISQ_OK", (opts, st)
        runs.append((opts, [x.cpu().numpy() for x in xs], st))
    opts0, x0, st0 = runs[0]
    assert st0["reliable_updates"] > 1 and len(set(st0["shift_iters"][1:len(shifts)])) > 1, st0
    for opts, xs, st in runs[1:]:
        assert st["iters"] == st0["iters"] and st["refine_iters"] == st0["refine_iters"], (opts, st, st0)
        assert st["reliable_updates"] == st0["reliable_updates"], (opts, st, st0)
        for i in range(len(shifts)):
            assert np.array_equal(xs[i].view(np.uint64), x0[i].view(np.uint64)), (opts, i)
    for i, s in enumerate(shifts):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x0[i]), full(dims, ev, b), dims, mass, s)
        assert res <= tol[i] * (1 + 1e-6), (i, res)


@pytest.mark.parametrize("nb", [1, 3, 16])
def test_multishift_quantised_block_sizes(nb):
    """30-bit multi-shift vectors (the benchmark's format) with blocks of 1, 3
    (shifts stop and reliable updates fall inside blocks) and 16 iterations:
    every shift still reaches its true residual and the oracle's solution"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    shifts = [1e-4, 1e-3, 1e-2, 0.1, 1.0, 10.0]
    tol = [1e-10] * len(shifts)
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "int30", "int20"])
    xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, tol, pg[0], pg[hisq.fmt("int30").gauge],
                                      pg[hisq.fmt("int20").gauge], mass, ms_fmt="int30", ref_fmt="int20",
                                      grad_buffer=nb, poll_every=7)
    assert st["status"] == "HISQ_OK", st
    out = oracle.multishift_cg(fat.numpy(), lng.numpy(), full(dims, ev, b), dims, mass, shifts, 1e-12)
    for i, s in enumerate(shifts):
        x = xs[i].cpu().numpy()
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x), full(dims, ev, b), dims, mass, s)
        assert res <= tol[i] * (1 + 1e-6), (nb, i, res, st)
        xo = out["x"][i][ev]
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8, (nb, i)


def test_multishift_explicit_floor():
    """An explicit stopping floor above the tolerance (the INT30 epsilon) ends
    the multi-shift phase sooner and leaves more to the refinement; every
    shift still reaches its tolerance and the oracle's solution. Without a
    floor (FP64 arithmetic) the shifts stop at their tolerance in the
    multi-shift phase itself."""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    shifts = [1e-4, 1e-3, 1e-2, 0.1, 1.0, 10.0]
    tol = [1e-10] * len(shifts)
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "int30", "int20"])
    runs = {}
    for floor in (0.0, 2.0 ** -29):
        xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, tol, pg[0], pg[hisq.fmt("int30").gauge],
                                          pg[hisq.fmt("int20").gauge], mass, ms_fmt="int30", ref_fmt="int20",
                                          shift_floor=floor)
        assert st["status"] == "HISQ_OK", (floor, st)
        runs[floor] = (xs, st)
    out = oracle.multishift_cg(fat.numpy(), lng.numpy(), full(dims, ev, b), dims, mass, shifts, 1e-12)
    for floor, (xs, st) in runs.items():
        for i, s in enumerate(shifts):
            x = xs[i].cpu().numpy()
            res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x), full(dims, ev, b), dims, mass, s)
            assert res <= tol[i] * (1 + 1e-6), (floor, i, res, st)
            xo = out["x"][i][ev]
            assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8, (floor, i)
    st0, st1 = runs[0.0][1], runs[2.0 ** -29][1]
    assert st1["iters"] < st0["iters"], (st0["iters"], st1["iters"])
    assert sum(st1["refine_iters"]) > sum(st0["refine_iters"]), (st0["refine_iters"], st1["refine_iters"])


def test_multishift_per_shift_tolerances():
    """RHMC-like: every shift has its own target (Sec. 6.2 footnote)"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    shifts = [1e-5, 3e-4, 1e-2, 0.3, 10.0]
    tol = [1e-6, 1e-8, 1e-10, 1e-11, 1e-12]
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "int30", "int20"])
    xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, tol, pg[0], pg[3], pg[2], mass,
                                      ms_fmt="int30", ref_fmt="int20")
    assert st["status"] == "HISQ_OK", st
    for i, s in enumerate(shifts):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, xs[i].cpu().numpy()), full(dims, ev, b),
                                   dims, mass, s)
        assert res <= tol[i] * (1 + 1e-6), (i, res)


def test_multishift_many_shifts_two_blocks():
    """18 shifts: the batched refinement runs the 17 shifted systems as a block
    of 16 and a block of 1; per-shift targets differ inside a block; with the
    base refined concurrently (batch_refine 2) as well, and with the base in
    the first block (batch_refine 3: blocks of 16 and 2)"""
    hisq = need_gpu()
    dims, mass = (6, 8, 10, 12), 0.05
    shifts = [10.0 ** (-4 + 5 * i / 17) for i in range(18)]
    tol = [1e-9 if i % 3 == 1 else 1e-10 for i in range(18)]
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "single", "half"])
    for batch in (1, 2, 3):
        xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, tol, pg[0], pg[1], pg[2], mass,
                                          ms_fmt="single", ref_fmt="half", batch_refine=batch)
        assert st["status"] == "HISQ_OK", st
        for i, s in enumerate(shifts):
            res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, xs[i].cpu().numpy()),
                                       full(dims, ev, b), dims, mass, s)
            assert res <= tol[i] * (1 + 1e-6), (batch, i, res)
            assert abs(res - st["shift_resid"][i]) <= 1e-3 * res + 1e-15


def test_multishift_single_shift():
    hisq = need_gpu()
    dims, mass = (6, 8, 10, 12), 0.1
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "single", "half"])
    xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), [0.02], [1e-10], pg[0], pg[1], pg[2], mass)
    res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, xs[0].cpu().numpy()), full(dims, ev, b),
                               dims, mass, 0.02)
    assert st["status"] == "HISQ_OK" and res <= 1e-10 * (1 + 1e-6)


@pytest.mark.parametrize("sloppy", ["half", "int20", "single", "double", "int24", "sx24"])
@pytest.mark.parametrize("nrhs", [1, 4, 16])
def test_batched_cg(sloppy, nrhs):
    hisq = need_gpu()
    dims, mass = (6, 8, 10, 12), 0.1
    fat, lng, ev, _ = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", sloppy])
    bs = inputs.gaussian_spinor(ev.size, inputs.RHS_SEED, nrhs=nrhs).numpy()
    bs[nrhs // 2] *= 1e-3          # right-hand sides of very different norms
    x, st = hisq.cg_solve_batched(torch.from_numpy(bs).cuda(), pg[0], pg[hisq.fmt(sloppy).gauge], mass, tol=1e-10,
                                  sloppy=sloppy)
    assert st["status"] == "HISQ_OK", st
    x = x.cpu().numpy()
    for j in range(nrhs):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x[j]), full(dims, ev, bs[j]), dims, mass)
        assert res <= 1e-10 * (1 + 1e-6), (j, res)


@pytest.mark.parametrize("plain,fused", [((4, 4), (8, 2)), ((16, 1), (2, 8)), ((8, 2), (4, 4))])
def test_batched_cg_fused_shape_differs(plain, fused):
    """the launches that fuse a reduction on another nr x rg than the plain ones:
    each has its own column map, and the partial sums follow the fused shape"""
    hisq = need_gpu()
    dims, mass, nrhs, sloppy = (6, 8, 10, 12), 0.1, 11, "int20"
    fat, lng, ev, _ = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", sloppy])
    bs = inputs.gaussian_spinor(ev.size, inputs.RHS_SEED + 5, nrhs=nrhs).numpy()
    bs[3] *= 1e-3
    hisq.hisq_tune_clear()
    try:
        for f, recon in ((sloppy, 18), ("double", 18)):
            hisq.hisq_tune_set(f, dims, 16, plain[0], plain[1], 1, 256, 0, long_recon=recon)
            hisq.hisq_tune_set_fused(f, dims, 16, fused[0], fused[1], 1, 256, 0, long_recon=recon)
        x, st = hisq.cg_solve_batched(torch.from_numpy(bs).cuda(), pg[0], pg[hisq.fmt(sloppy).gauge], mass,
                                      tol=1e-10, sloppy=sloppy)
    finally:
        hisq.hisq_tune_clear()
    assert st["status"] == "HISQ_OK", st
    x = x.cpu().numpy()
    for j in range(nrhs):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x[j]), full(dims, ev, bs[j]), dims, mass)
        assert res <= 1e-10 * (1 + 1e-6), (j, res)


@pytest.mark.parametrize("sloppy", ["half", "int20", "single", "int30", "int24"])
def test_cg_error_estimate_reliable_updates(sloppy):
    """reliable updates triggered by the residual-deviation estimate instead of delta"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.02
    fat, lng, ev, b = setup(dims, "haar")
    pg = packed(hisq, fat, lng, dims, ["double", sloppy])
    x, st = hisq.cg_solve(torch.from_numpy(b).cuda(), pg[0], pg[hisq.fmt(sloppy).gauge], mass, tol=1e-10,
                          sloppy=sloppy, ru_estimate=1)
    assert st["status"] == "HISQ_OK" and st["reliable_updates"] >= 1, st
    res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, x.cpu().numpy()), full(dims, ev, b), dims, mass)
    assert res <= 1e-10 * (1 + 1e-6), (res, st)


def test_multishift_error_estimate_reliable_updates():
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    shifts = [1e-4, 1e-2, 1.0]
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "int30", "int20"])
    xs, st = hisq.multishift_cg_solve(torch.from_numpy(b).cuda(), shifts, [1e-10] * 3, pg[0], pg[3], pg[2], mass,
                                      ms_fmt="int30", ref_fmt="int20", ru_estimate=1)
    assert st["status"] == "HISQ_OK", st
    for i, s in enumerate(shifts):
        res = oracle.true_residual(fat.numpy(), lng.numpy(), full(dims, ev, xs[i].cpu().numpy()), full(dims, ev, b),
                                   dims, mass, s)
        assert res <= 1e-10 * (1 + 1e-6), (i, res)


def test_iteration_caps_report_enoconv():
    """an iteration cap ends every solver with HISQ_ENOCONV, its stats filled
    and the best iterate finite"""
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.01
    fat, lng, ev, b = setup(dims, "haar")
    pg = packed(hisq, fat, lng, dims, ["double", "half"])
    bt = torch.from_numpy(b).cuda()
    xs, st = hisq.multishift_cg_solve(bt, [0.0, 0.01, 0.1], 1e-12, pg[0], pg[2], pg[2], mass, ms_fmt="half",
                                      ref_fmt="half", maxiter=10)
    assert st["status"] == "HISQ_ENOCONV" and st["iters"] >= 10, st
    assert all(bool(torch.isfinite(torch.view_as_real(x)).all()) for x in xs)
    bs = inputs.gaussian_spinor(ev.size, inputs.RHS_SEED, nrhs=4).cuda()
    x, st = hisq.cg_solve_batched(bs, pg[0], pg[2], mass, tol=1e-12, sloppy="half", maxiter=6)
    assert st["status"] == "HISQ_ENOCONV", st
    assert bool(torch.isfinite(torch.view_as_real(x)).all())


def test_nonfinite_source_is_a_breakdown():
    hisq = need_gpu()
    dims, mass = (8, 8, 8, 8), 0.05
    fat, lng, ev, b = setup(dims, "near_unit")
    pg = packed(hisq, fat, lng, dims, ["double", "single"])
    bad = b.copy()
    bad[17, 1] = complex(float("nan"), 0.0)
    with pytest.raises(hisq.HisqError) as e:
        hisq.cg_solve(torch.from_numpy(bad).cuda(), pg[0], pg[1], mass, tol=1e-10, sloppy="single")
    assert e.value.status == -5
