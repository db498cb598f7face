"""Benchmark: mixed-precision multi-shift CG on the HISQ operator (one MI355X).

Workload (one "step" = one pass of the whole hot path): 48^3x96 lattice,
near-unit links, m = 0.005, 12 shifts log-spaced from 1e-5 to 10, every shift
solved to a 1e-10 true relative residual.  A step packs the FP64 links (already
resident in HBM) into the solver's storage formats and runs the multi-shift
solve: multi-shift phase in 32-bit links / 30-bit fermions / FP64 compute with
FP64 reliable updates, then CG refinement in 16-bit links / 20-bit fermions /
FP32 compute (the paper's improved variant, Sec. 6.2).  The multi-shift
operator keeps each long link as the eight parameters of its SU(3) matrix
(--ms-recon 8), the refinement and FP64 operators as two rows (--recon 12).

Printed (one JSON line): whole-step algorithmic HBM GB/s (value), the
per-triplet Dslash GB/s and GFLOP/s measured with HIP events (the Fig. 3
analog), the roofline of the dominant kernel, the FP64 GPU multi-shift
comparator (time to the same residuals), and the FP64 CPU oracle timed on the
host cores as a reported baseline.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-fp64] [--no-cpu] [--no-stability]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FLOP_PER_SITE = 1146


COUNTERS = os.path.join(ROOT, "profiles", "dslash_int30_r8_48x48x48x96_counters.txt")
COUNTER_SOURCES = ["hisq_dslash_kernels.h", "hisq_device.h", "hisq_dslash_t_int30.hip"]


def counter_traffic(kernel, dims, recon):
    """HBM bytes per launch of the dominant Dslash from the committed rocprofv3
    counter passes (FETCH_SIZE + WRITE_SIZE, calibrated with a 1 GiB copy), or
    None when that file covers another kernel or its sources have changed."""
    import hashlib
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    for line in open(COUNTERS):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    want = f"{kernel} long_recon {recon} lattice {'x'.join(map(str, dims))}"
    if kv.get("kernel") != want:
        return None
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, "paper_2302_09224_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != kv.get("kernel_sha256"):
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_batched(args, hisq, inputs, torch, dev, dims=(32, 32, 32, 64), nrhs=16, reps=10,
                  names=("half", "int20", "single"), recon=18, shapes=None):
    """Block of nrhs right-hand sides (one link load per site for the block)
    against nrhs single-right-hand-side applications (default 16 on 32^3x64).
    shapes: launch shapes (nr, rg, stage, sweep) to pin one after another with
    hisq_tune_set and time (2 warm-up and `reps` timed launches each), in place
    of the autotuned one."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    vh = V // 2
    fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED + 4, device=dev)
    srcs = inputs.gaussian_spinor(vh, inputs.RHS_SEED, device=dev, nrhs=nrhs)
    out = {}
    stream = torch.cuda.current_stream()
    for name in names:
        f = hisq.fmt(name)
        pg = hisq.pack_gauge(fat, lng, dims, f.gauge, long_recon=recon)
        nb = hisq.hisq_spinor_bytes(vh, f.spinor)
        pin = torch.cat([hisq.pack_spinor(srcs[j], f.spinor)[:nb] for j in range(nrhs)]).contiguous()
        pout = torch.empty_like(pin)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if shapes:
            block = 1
            while block < nrhs:
                block <<= 1
            pinned = {}
            for nr, rg, stage, sweep in shapes:
                hisq.hisq_tune_set(name, dims, block, nr, rg, stage, 256, 0, sweep=sweep, long_recon=recon)
                for _ in range(2):
                    hisq.hisq_dslash_batched(pout, pin, pg.desc, 1, f, nrhs)
                e0.record(stream)
                for _ in range(reps):
                    hisq.hisq_dslash_batched(pout, pin, pg.desc, 1, f, nrhs)
                e1.record(stream)
                torch.cuda.synchronize()
                pinned[f"{nr},{rg},{stage},{sweep}"] = round(e0.elapsed_time(e1) / reps * 1e3, 1)
                log(f"[bench] batched {name} {dims} x{nrhs} shape nr {nr} rg {rg} stage {stage} order {sweep}: "
                    f"{pinned[f'{nr},{rg},{stage},{sweep}']} us")
            hisq.hisq_tune_clear()
            out[name] = dict(dims=list(dims), nrhs=nrhs, long_recon=recon, us_per_shape=pinned)
            del pg, pin, pout
            continue
        for _ in range(2):
            hisq.hisq_dslash_batched(pout, pin, pg.desc, 1, f, nrhs)
        e0.record(stream)
        for _ in range(reps):
            hisq.hisq_dslash_batched(pout, pin, pg.desc, 1, f, nrhs)
        e1.record(stream)
        torch.cuda.synchronize()
        tb = e0.elapsed_time(e1) / reps
        # 16 single-right-hand-side applications: kernel time of one application x 16
        one_in, one_out = pin[:nb], pout[:nb]
        hisq.hisq_dslash(one_out, one_in, pg.desc, 1, f)
        e0.record(stream)
        for _ in range(reps * 4):
            hisq.hisq_dslash(one_out, one_in, pg.desc, 1, f)
        e1.record(stream)
        torch.cuda.synchronize()
        ts = e0.elapsed_time(e1) / (reps * 4) * nrhs
        nbytes = vh * (8 * hisq.GAUGE_BYTES[f.gauge] + 8 * long_link_bytes(hisq, f.gauge, recon)
                       + nrhs * 2 * hisq.SPINOR_BYTES[f.spinor])
        out[name] = dict(dims=list(dims), nrhs=nrhs, long_recon=recon, us_batched=round(tb * 1e3, 1),
                         us_single_x_nrhs=round(ts * 1e3, 1),
                         speedup=round(ts / tb, 2), gbs=round(nbytes / tb / 1e6, 1),
                         gflops=round(nrhs * FLOP_PER_SITE * vh / tb / 1e6, 1))
        log(f"[bench] batched {name:6s} {out[name]}")
        del pg, pin, pout
    del fat, lng, srcs
    torch.cuda.empty_cache()
    return out


def bench_batched_cg(hisq, inputs, torch, dev, dims=(32, 32, 32, 64), nrhs=16, mass=0.01, tol=1e-10):
    """16 right-hand sides on 32^3x64: one batched mixed-precision CG (FIX16/INT20
    sloppy, two-row long links; every Dslash shared by the block) against 16
    independent FP64 CG solves; solves per second of each."""
    import numpy as np
    V = dims[0] * dims[1] * dims[2] * dims[3]
    fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED + 4, device=dev)
    bs = inputs.gaussian_spinor(V // 2, inputs.RHS_SEED, device=dev, nrhs=nrhs)
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64)
    gs = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_FIX16, long_recon=12)
    del fat, lng
    hisq.cg_solve_batched(bs, g64, gs, mass, tol=tol, sloppy="int20")          # warm-up (launch shapes)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, sb = hisq.cg_solve_batched(bs, g64, gs, mass, tol=tol, sloppy="int20")
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    hisq.cg_solve(bs[0], g64, g64, mass, tol=tol, sloppy="double", delta=0.0)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    iters64 = []
    for j in range(nrhs):
        _, s64 = hisq.cg_solve(bs[j], g64, g64, mass, tol=tol, sloppy="double", delta=0.0)
        iters64.append(s64["iters"])
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t
    out = dict(lattice=list(dims), nrhs=nrhs, mass=mass, tol=tol, batched_triplet="fix16/int20/fp32",
               batched_seconds=round(tb, 3), batched_iters=sb["iters"], batched_resid_max=max(sb["shift_resid"][:nrhs]),
               fp64_seconds=round(t64, 3), fp64_iters_mean=float(np.mean(iters64)),
               solves_per_s_batched=round(nrhs / tb, 2), solves_per_s_fp64=round(nrhs / t64, 2),
               speedup=round(t64 / tb, 2))
    log(f"[bench] batched CG {out}")
    del g64, gs, bs
    torch.cuda.empty_cache()
    return out


def bench_multi(hisq, inputs, torch, dev, reps=50):
    """8^4 + 12^4 + 16^4 + 24^4 in one launch against one launch per lattice
    (HIP events; FIX16/INT20/FP32, two-row long links)."""
    lattices = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (24, 24, 24, 24)]
    f = hisq.fmt("int20")
    outs, ins, gauges, keep = [], [], [], []
    nbytes = 0
    for k, dims in enumerate(lattices):
        vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
        fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED + 50 + k, device=dev)
        pg = hisq.pack_gauge(fat, lng, dims, f.gauge, long_recon=12)
        pin = hisq.pack_spinor(inputs.gaussian_spinor(vh, inputs.SOURCE_SEED + 50 + k, device=dev), f.spinor)
        outs.append(torch.empty_like(pin))
        ins.append(pin)
        gauges.append(pg.desc)
        keep.append(pg)
        nbytes += vh * (8 * 36 + 8 * 24 + 2 * 16)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def one_launch():
        hisq.hisq_dslash_multi(outs, ins, gauges, 0, f)

    def per_lattice():
        for o, i, g in zip(outs, ins, gauges):
            hisq.hisq_dslash(o, i, g, 0, f)

    res = {}
    for name, fn in (("one_launch", one_launch), ("per_lattice", per_lattice)):
        for _ in range(3):
            fn()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps * 1e3
    out = dict(lattices=["x".join(map(str, d)) for d in lattices], triplet="fix16/int20/fp32", long_recon=12,
               us_one_launch=round(res["one_launch"], 1), us_per_lattice=round(res["per_lattice"], 1),
               speedup=round(res["per_lattice"] / res["one_launch"], 2),
               gbs_one_launch=round(nbytes / res["one_launch"] / 1e3, 1))
    log(f"[bench] multi-lattice {out}")
    del outs, ins, gauges, keep
    torch.cuda.empty_cache()
    return out


def bench_cg_stability(hisq, inputs, torch, dev, dims=(16, 16, 16, 16), masses=(0.01, 0.001), tol=1e-10,
                       maxiter=40000):
    """Fig. 1 analog (Sec. 3.1): CG on rough (Haar) links at light masses, FP64
    vs double-half with reliable updates only (Fletcher-Reeves beta, no gradient
    re-projection) vs the stabilised double-half (Polak-Ribiere beta,
    re-projection; the FP64 buffered solution in both mixed variants)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    fat, lng = inputs.make_links(dims, "haar", inputs.GAUGE_SEED + 60, device=dev)
    b = inputs.gaussian_spinor(V // 2, inputs.SOURCE_SEED + 60, device=dev)
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64)
    g16 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_FIX16)
    out = {}
    for m in masses:
        row = {}
        for name, gs, sl, kw in (("double", g64, "double", dict(delta=0.0)),
                                 ("double-half naive", g16, "half", dict(pr_beta=0, reproject=0)),
                                 ("double-half stabilised", g16, "half", {}),
                                 ("double-half stabilised, error-estimate updates", g16, "half",
                                  dict(ru_estimate=1))):
            torch.cuda.synchronize()
            t = time.perf_counter()
            try:
                _, st = hisq.cg_solve(b, g64, gs, m, tol=tol, sloppy=sl, maxiter=maxiter, **kw)
                status = st["status"]
            except hisq.HisqError as e:      # iteration cap: report it
                st, status = None, str(e).split(":")[1].strip()
            torch.cuda.synchronize()
            row[name] = dict(status=status, iters=st["iters"] if st else maxiter,
                             reliable_updates=st["reliable_updates"] if st else None,
                             true_resid=st["true_resid"] if st else None, seconds=round(time.perf_counter() - t, 3))
            log(f"[bench] CG stability m={m} {name}: {row[name]['iters']} it, {status}, {row[name]['seconds']} s")
        out[f"m={m}"] = row
        log(f"[bench] CG stability {dims} Haar m={m}: " +
            ", ".join(f"{k} {v['iters']} it ({v['status']})" for k, v in row.items()))
    del g64, g16, fat, lng
    torch.cuda.empty_cache()
    return out


def bench_bicgstab(hisq, inputs, torch, dev, dims, mass, kind="near_unit", tol=1e-10, l=4, maxiter=200000):
    """Table 2 analog (Sec. 6.1): BiCGStab(4) for the whole-lattice operator
    2m + D in pure double and double-{single, int30, int24, sx24, int20, half}."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    fat, lng = inputs.make_links(dims, kind, inputs.GAUGE_SEED + 90, device=dev)
    b = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 90, device=dev)
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64)
    del fat, lng
    out = {}
    for name in ("double", "single", "int30", "int24", "sx24", "int20", "half"):
        f = hisq.fmt(name)
        gs = g64 if name == "double" else _pack_like(hisq, inputs, dims, f.gauge, dev, kind)
        kw = dict(delta=0.0) if name == "double" else {}
        hisq.bicgstab_solve(b, g64, gs, mass, tol=tol, l=l, sloppy=name, maxiter=16, **kw)   # tune the shapes
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = hisq.bicgstab_solve(b, g64, gs, mass, tol=tol, l=l, sloppy=name, maxiter=maxiter, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[f"double-{name}" if name != "double" else "pure double"] = dict(
            status=st["status"], operator_applications=st["iters"], reliable_updates=st["reliable_updates"],
            true_resid=st["true_resid"], seconds=round(dt, 3))
        log(f"[bench] BiCGStab({l}) {dims} {kind} m={mass} {name}: {st['iters']} applications, {dt:.2f}s, "
            f"resid {st['true_resid']:.2e} ({st['status']})")
        del gs
        torch.cuda.empty_cache()
    return dict(lattice=list(dims), links=kind, mass=mass, tol=tol, l=l, solvers=out)


def bench_formats(hisq, inputs, torch, dev, reps, dims=(32, 32, 32, 32), mass=0.01, tol=1e-10):
    """Per-triplet table on 32^4 (near-unit links, m = 0.01): Dslash time and
    algorithmic GB/s (18-real links), and the mixed CG to a 1e-10 true residual
    with that triplet as the sloppy one (iterations, reliable updates, time)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    vh = V // 2
    fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED + 13, device=dev)
    psi = inputs.gaussian_spinor(vh, inputs.SOURCE_SEED + 13, device=dev)
    b = inputs.gaussian_spinor(vh, inputs.SOURCE_SEED + 14, device=dev)
    g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64)
    stream = torch.cuda.current_stream()
    out = {}
    for name in ("double", "single", "int30", "int30_fp32", "int24", "sx24", "sx24_int30", "int20", "half"):
        f = hisq.fmt(name)
        pg = g64 if f.gauge == hisq.GAUGE_F64 else hisq.pack_gauge(fat, lng, dims, f.gauge)
        pin = hisq.pack_spinor(psi, f.spinor)
        y = torch.empty_like(pin)
        for _ in range(3):
            hisq.hisq_dslash(y, pin, pg.desc, 0, f)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            hisq.hisq_dslash(y, pin, pg.desc, 0, f)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        nbytes = vh * (16 * hisq.GAUGE_BYTES[f.gauge] + 2 * hisq.SPINOR_BYTES[f.spinor])
        hisq.cg_solve(b, g64, pg, mass, tol=tol, sloppy=name)            # launch shapes tuned here
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = hisq.cg_solve(b, g64, pg, mass, tol=tol, sloppy=name)
        torch.cuda.synchronize()
        out[name] = dict(triplet=repr(f), dslash_us=round(us, 1), gbs=round(nbytes / us / 1e3, 1),
                         cg_iters=st["iters"], reliable_updates=st["reliable_updates"],
                         true_resid=float(f"{st['true_resid']:.3g}"), cg_seconds=round(time.perf_counter() - t, 4))
        log(f"[bench] 32^4 {name:10s} dslash {us:7.1f} us {out[name]['gbs']:7.1f} GB/s; CG {st['iters']} it, "
            f"{out[name]['cg_seconds']:.3f} s")
        del pin, y
        if pg is not g64:
            del pg
        torch.cuda.empty_cache()
    del g64, fat, lng
    torch.cuda.empty_cache()
    return dict(lattice=list(dims), mass=mass, tol=tol, triplets=out)


def long_link_bytes(hisq, gf, recon):
    """bytes of one stored long link: 18 reals, two rows, or eight parameters"""
    if recon == 8:
        return {hisq.GAUGE_F64: 64, hisq.GAUGE_FIX32: 32}[gf]
    return hisq.GAUGE_BYTES[gf] * 2 // 3 if recon == 12 else hisq.GAUGE_BYTES[gf]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(np, dims, fat, lng, b, shifts, tols, mass, kernels, fp64_iters, gpu_seconds):
    """The FP64 oracle on the host cores, on bounded samples of the benchmark's
    own lattice and fields (about 25 s in all):
    * its Dslash at 2^20 random output sites, repeated for ~6 s, with all the
      threads the oracle uses, and at 2^16 sites for ~3 s on one thread;
    * its FP64 multi-shift CG of the same 12-shift system for one and for two
      iterations (final residuals skipped), the difference being the time of
      one iteration; times the FP64 multi-shift's iteration count on the GPU
      (the same algorithm) it gives the oracle's extrapolated time to solution."""
    import oracle
    olib = oracle.load()
    nthr = oracle.threads(olib)
    log(f"[bench] CPU oracle baseline ({nthr} threads, {cpu_model()})")
    V = dims[0] * dims[1] * dims[2] * dims[3]
    fat_h = fat.cpu().numpy()
    lng_h = lng.cpu().numpy()
    i = np.arange(V)
    par = ((i % dims[0]) + (i // dims[0]) % dims[1] + (i // (dims[0] * dims[1])) % dims[2]
           + i // (dims[0] * dims[1] * dims[2])) % 2
    odd, even = np.nonzero(par == 1)[0], np.nonzero(par == 0)[0]
    full = np.zeros((V, 3), dtype=np.complex128)
    full[odd] = b.cpu().numpy()
    rng = np.random.default_rng(0)

    def dslash_rate(nsites, seconds):
        sample = np.sort(rng.choice(even, size=min(even.size, nsites), replace=False))
        done, tc = 0, 0.0
        while tc < seconds:
            t2 = time.perf_counter()
            oracle.dslash_sites(fat_h, lng_h, full, dims, sample, lib=olib)
            tc += time.perf_counter() - t2
            done += sample.size
        return done * (16 * 144 + 2 * 48) / tc / 1e9, sample.size, done // sample.size, tc

    gbs, n_s, reps, tc = dslash_rate(1 << 20, 6.0)
    oracle.set_threads(1, olib)
    try:
        gbs1, n_s1, reps1, tc1 = dslash_rate(1 << 16, 3.0)
    finally:
        oracle.set_threads(nthr, olib)
    log(f"[bench]   oracle Dslash {gbs:.2f} GB/s on {nthr} threads, {gbs1:.2f} GB/s on 1 thread")
    # one iteration of the oracle's FP64 multi-shift CG on the whole lattice
    bfull = np.zeros((V, 3), dtype=np.complex128)
    bfull[even] = full[odd]
    tms = []
    for k in (1, 2):
        t2 = time.perf_counter()
        oracle.multishift_cg(fat_h, lng_h, bfull, dims, mass, shifts, tols, maxiter=k, lib=olib, residuals=False)
        tms.append(time.perf_counter() - t2)
    t_iter = tms[1] - tms[0]
    extrap = t_iter * fp64_iters if fp64_iters else None
    log(f"[bench]   oracle multi-shift: {t_iter:.2f} s per iteration"
        + (f", x {fp64_iters} iterations = {extrap:.0f} s (extrapolated)" if extrap else ""))
    del fat_h, lng_h, full, bfull
    return dict(value=round(gbs, 3), unit="GB/s", cores=nthr, kind="oracle", cpu_model=cpu_model(),
                sample=f"FP64 oracle Dslash at {n_s} random even sites of the {dims} lattice, repeated {reps}x "
                       f"({tc:.1f}s); algorithmic bytes 2400/site",
                value_1thread=round(gbs1, 3),
                sample_1thread=f"{n_s1} random even sites, repeated {reps1}x ({tc1:.1f}s), one thread",
                vs_gpu_fp64_dslash=round(kernels["double"]["gbs"] / gbs, 1),
                multishift_seconds_per_iteration=round(t_iter, 3),
                multishift_iterations=fp64_iters,
                multishift_seconds_extrapolated=round(extrap, 1) if extrap else None,
                multishift_sample=("oracle FP64 multi-shift CG of the same 12-shift system: 2 minus 1 iterations "
                                   "timed (final residuals skipped), times the FP64 multi-shift iteration count "
                                   "(extrapolated; the oracle's vector updates are single-threaded)"),
                vs_gpu_mixed_solve=round(extrap / gpu_seconds, 1) if extrap else None)


def cg_time_to_solution(np, hisq, inputs, torch, dev, batched_cg, tol=1e-10):
    """The FP64 oracle's CG time to solution on the host beside the GPU's, on the
    smaller workloads: 4^4 (Haar links, m = 0.1) and 16^4 (near-unit, m = 0.05)
    to completion; 32^4 (near-unit, m = 0.01) and the 32^3x64 block of 16
    systems (m = 0.01) as the oracle's time per iteration (the difference of two
    short runs, setup and final residual cancelling) times the GPU FP64 CG's
    iteration count (extrapolated; the same algorithm).  GPU: plain FP64 CG
    and the mixed CG (double-single on the first two, double-int20 with two-row
    long links on 32^4), each timed after a warm-up solve, excluding the pack."""
    import oracle
    olib = oracle.load()
    rows = []

    def gpu_solve(b, g64, gs, mass, sloppy, **kw):
        hisq.cg_solve(b, g64, gs, mass, tol=tol, sloppy=sloppy, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = hisq.cg_solve(b, g64, gs, mass, tol=tol, sloppy=sloppy, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t, st

    def oracle_per_iter(fat_h, lng_h, bfull, dims, mass, k0, k1):
        ts = []
        for k in (k0, k1):
            t = time.perf_counter()
            oracle.cg(fat_h, lng_h, bfull, dims, mass, tol=tol, maxiter=k, lib=olib)
            ts.append(time.perf_counter() - t)
        return (ts[1] - ts[0]) / (k1 - k0)

    cases = [((4, 4, 4, 4), "haar", 0.1, 0, "single", True),
             ((16, 16, 16, 16), "near_unit", 0.05, 1, "single", True),
             ((32, 32, 32, 32), "near_unit", 0.01, 2, "int20", False)]
    for dims, kind, mass, k, sloppy, complete in cases:
        V = dims[0] * dims[1] * dims[2] * dims[3]
        fat, lng = inputs.make_links(dims, kind, inputs.GAUGE_SEED + k, device=dev)
        ev = np.nonzero(((np.arange(V) % dims[0]) + (np.arange(V) // dims[0]) % dims[1]
                         + (np.arange(V) // (dims[0] * dims[1])) % dims[2]
                         + np.arange(V) // (dims[0] * dims[1] * dims[2])) % 2 == 0)[0]
        bh = inputs.gaussian_spinor(ev.size, inputs.SOURCE_SEED + k).numpy()
        b = torch.from_numpy(bh).to(dev)
        fs = hisq.fmt(sloppy)
        recon = 12 if sloppy == "int20" else 18
        g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64)
        gs = hisq.pack_gauge(fat, lng, dims, fs.gauge, long_recon=recon)
        t64, s64 = gpu_solve(b, g64, g64, mass, "double", delta=0.0)
        tmx, smx = gpu_solve(b, g64, gs, mass, sloppy)
        fat_h, lng_h = fat.cpu().numpy(), lng.cpu().numpy()
        bfull = np.zeros((V, 3), dtype=np.complex128)
        bfull[ev] = bh
        row = dict(lattice=list(dims), links=kind, mass=mass, tol=tol,
                   gpu_fp64_seconds=round(t64, 4), gpu_fp64_iters=s64["iters"],
                   gpu_mixed=f"double-{sloppy}", gpu_mixed_seconds=round(tmx, 4), gpu_mixed_iters=smx["iters"],
                   gpu_mixed_resid=float(f"{smx['true_resid']:.3g}"))
        if complete:
            t = time.perf_counter()
            _, it, res, _ = oracle.cg(fat_h, lng_h, bfull, dims, mass, tol=tol, lib=olib)
            row.update(oracle_seconds=round(time.perf_counter() - t, 3), oracle_iters=it,
                       oracle_resid=float(f"{res:.3g}"), extrapolated=False)
        else:
            per = oracle_per_iter(fat_h, lng_h, bfull, dims, mass, 2, 6)
            row.update(oracle_seconds=round(per * s64["iters"], 1), oracle_seconds_per_iter=round(per, 4),
                       oracle_iters=s64["iters"], extrapolated=True)
        row["oracle_over_gpu_mixed"] = round(row["oracle_seconds"] / tmx, 1)
        rows.append(row)
        log(f"[bench]   CG {dims} m={mass}: oracle {row['oracle_seconds']} s"
            f"{' (extrapolated)' if not complete else ''}, GPU FP64 {t64:.3f} s, GPU double-{sloppy} {tmx:.3f} s")
        del fat, lng, g64, gs, fat_h, lng_h, bfull, b
        torch.cuda.empty_cache()
    if batched_cg:
        dims, mass, nrhs = tuple(batched_cg["lattice"]), batched_cg["mass"], batched_cg["nrhs"]
        V = dims[0] * dims[1] * dims[2] * dims[3]
        fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED + 4, device=dev)
        fat_h, lng_h = fat.cpu().numpy(), lng.cpu().numpy()
        del fat, lng
        ev = np.nonzero(((np.arange(V) % dims[0]) + (np.arange(V) // dims[0]) % dims[1]
                         + (np.arange(V) // (dims[0] * dims[1])) % dims[2]
                         + np.arange(V) // (dims[0] * dims[1] * dims[2])) % 2 == 0)[0]
        bfull = np.zeros((V, 3), dtype=np.complex128)
        bfull[ev] = inputs.gaussian_spinor(ev.size, inputs.RHS_SEED).numpy()
        per = oracle_per_iter(fat_h, lng_h, bfull, dims, mass, 1, 3)
        tot = per * batched_cg["fp64_iters_mean"] * nrhs
        rows.append(dict(lattice=list(dims), links="near_unit", mass=mass, tol=tol, nrhs=nrhs,
                         gpu_fp64_seconds=batched_cg["fp64_seconds"], gpu_mixed="batched double-int20",
                         gpu_mixed_seconds=batched_cg["batched_seconds"], oracle_seconds=round(tot, 1),
                         oracle_seconds_per_iter=round(per, 4), oracle_iters=batched_cg["fp64_iters_mean"],
                         extrapolated=True, oracle_over_gpu_mixed=round(tot / batched_cg["batched_seconds"], 1)))
        log(f"[bench]   CG {dims} x{nrhs}: oracle {tot:.0f} s (extrapolated), GPU batched {batched_cg['batched_seconds']} s")
        del fat_h, lng_h, bfull
    return rows


def _pack_like(hisq, inputs, dims, gf, dev, kind):
    fat, lng = inputs.make_links(dims, kind, inputs.GAUGE_SEED + 90, device=dev)
    return hisq.pack_gauge(fat, lng, dims, gf, long_recon=12)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=str, default="48,48,48,96")
    ap.add_argument("--mass", type=float, default=0.005)
    ap.add_argument("--nshift", type=int, default=12)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--ms", type=str, default="int30")
    ap.add_argument("--ref", type=str, default="int20")
    ap.add_argument("--recon", type=int, default=12, choices=(12, 18),
                    help="long-link storage of the solver's operators (12: two rows)")
    ap.add_argument("--ms-recon", type=int, default=8, choices=(8, 12, 18),
                    help="long-link storage of the multi-shift operator (8: eight parameters)")
    ap.add_argument("--batch-refine", type=int, default=3, choices=(0, 1, 2, 3),
                    help="refine the shifted systems together (1), together while the base is refined "
                         "concurrently (2), together with the base in the same block (3), or one after another (0)")
    ap.add_argument("--shift-floor", type=float, default=0.0,
                    help="multi-shift: relative residual below which a shifted system stops (0: none with FP64 "
                         "arithmetic, the spinor format's epsilon with FP32 arithmetic)")
    ap.add_argument("--grad-buffer", type=int, default=16,
                    help="multi-shift solves: iterations per block of buffered updates (0: the library default, 8)")
    ap.add_argument("--ms-shape", type=str, default=None, metavar="STAGE,BLOCK,GRID,ORDER",
                    help="pin the launch shape of the multi-shift operator instead of autotuning it")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-stability", action="store_true",
                    help="skip the 16^4 CG-stability table (not part of the timed step)")
    ap.add_argument("--no-alt", action="store_true", help="skip the double-single-half mixed solve")
    ap.add_argument("--bicgstab", type=str, default=None, metavar="X,Y,Z,T",
                    help="also run the BiCGStab(4) precision comparison on this lattice (see --bicgstab-mass)")
    ap.add_argument("--bicgstab-mass", type=float, default=0.001)
    ap.add_argument("--bicgstab-links", type=str, default="near_unit", choices=("near_unit", "haar"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-cg", action="store_true",
                    help="also time a lone FP64 CG per shift (the plain FP64 baseline, about 15 s)")
    ap.add_argument("--formats", action="store_true",
                    help="per-triplet Dslash GB/s and mixed CG iterations/time on 32^4, m = 0.01")
    ap.add_argument("--dslash-reps", type=int, default=20)
    ap.add_argument("--kernels-only", action="store_true", help="only the per-triplet Dslash table")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the warm-up and timed steps of the multi-shift solve (for kernel traces)")
    ap.add_argument("--no-graph", action="store_true",
                    help="enqueue the solver's iterations directly instead of replaying them as hipGraphs")
    ap.add_argument("--kernel", type=str, default=None,
                    help="only these rows of the Dslash table (comma-separated keys, e.g. int30_r8)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--batched", action="store_true",
                    help="also time the 16-right-hand-side Dslash on 32^3x64 against 16 single applications")
    ap.add_argument("--batched-shapes", type=str, default=None, metavar="NR,RG,STAGE,ORDER[;...]",
                    help="with --batched-only: pin and time these launch shapes instead of the autotuned one")
    ap.add_argument("--batched-only", nargs="?", const="both", default=None, choices=("both", "32x64", "48x96"),
                    help="only the batched FIX16/INT20 Dslash with two-row long links: 16 right-hand sides on "
                         "32^3x64 and 11 (a block of 16) on 48^3x96, as the refinement runs it (for counters); "
                         "32x64 or 48x96 selects one of the two")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "domain decomposition over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2302_09224_amd import hisq, inputs

    hisq.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dims = tuple(int(v) for v in args.dims.split(","))
    V = dims[0] * dims[1] * dims[2] * dims[3]
    vh = V // 2
    shifts = [10.0 ** (-5 + 6 * i / (args.nshift - 1)) for i in range(args.nshift)] if args.nshift > 1 else [1e-5]
    tols = [args.tol] * len(shifts)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
        del src, dst

    if args.batched_only:
        cases = {"32x64": ((32, 32, 32, 64), 16), "48x96": ((48, 48, 48, 96), 11)}
        shapes = ([tuple(int(v) for v in sh.split(",")) for sh in args.batched_shapes.split(";") if sh.strip()]
                  if args.batched_shapes else None)
        res = [bench_batched(args, hisq, inputs, torch, dev, dims=d, nrhs=n, names=("int20",), recon=12,
                             shapes=shapes)
               for k, (d, n) in cases.items() if args.batched_only in ("both", k)]
        print(json.dumps(dict(batched=res, tuning=hisq.hisq_tune_report().strip().splitlines())))
        return

    t0 = time.time()
    log(f"[bench] generating near-unit links on {dims} (seed {inputs.GAUGE_SEED + 3})")
    fat, lng = inputs.make_links(dims, "near_unit", inputs.GAUGE_SEED + 3, device=dev)
    b = inputs.gaussian_spinor(vh, inputs.SOURCE_SEED + 3, device=dev)
    torch.cuda.synchronize()
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s")

    fms, fref = hisq.fmt(args.ms), hisq.fmt(args.ref)
    f64 = hisq.fmt("double")

    # ---------------- per-triplet Dslash (Fig. 3 analog) ----------------
    kernels = {}
    gauges = {}

    def gauge(gf, recon):
        if (gf, recon) not in gauges:
            gauges[(gf, recon)] = hisq.pack_gauge(fat, lng, dims, gf, long_recon=recon)
        return gauges[(gf, recon)]

    def link_bytes(gf, recon):
        return 8 * hisq.GAUGE_BYTES[gf] + 8 * long_link_bytes(hisq, gf, recon)

    stream = torch.cuda.current_stream()
    names = ("double", "single", "half", "int20", "int30", "int30_fp32", "int24", "sx24", "sx24_int30")
    table = [(n, 18) for n in names] + [(n, 12) for n in names] + [("double", 8), ("int30", 8)]
    if args.solve_only:
        table = []
    if args.kernel:
        want = set(args.kernel.split(","))
        table = [(n, r) for n, r in table if (n if r == 18 else f"{n}_r{r}") in want]
    for name, recon in table:
        key = name if recon == 18 else f"{name}_r{recon}"
        f = hisq.fmt(name)
        pg = gauge(f.gauge, recon)
        pin = hisq.pack_spinor(b, f.spinor)
        out = torch.empty_like(pin)
        for _ in range(3):
            hisq.hisq_dslash(out, pin, pg.desc, 1, f)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for r in range(args.dslash_reps):
            hisq.hisq_dslash(out, pin, pg.desc, 1, f)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.dslash_reps
        nbytes = vh * (link_bytes(f.gauge, recon) + 2 * hisq.SPINOR_BYTES[f.spinor])
        kernels[key] = dict(triplet=repr(f), long_recon=recon, us=round(ms * 1e3, 2), alg_bytes=nbytes,
                            gbs=round(nbytes / ms / 1e6, 1), gflops=round(FLOP_PER_SITE * vh / ms / 1e6, 1),
                            frac_hbm=round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4))
        log(f"[bench] dslash {key:15s} {kernels[key]['us']:9.1f} us  {kernels[key]['gbs']:7.1f} GB/s "
            f"{kernels[key]['gflops']:7.1f} GFLOP/s  ({100 * kernels[key]['frac_hbm']:.1f}% HBM)")
        del pin, out
    batched = None
    if args.batched:
        batched = bench_batched(args, hisq, inputs, torch, dev)
    multi = None if args.solve_only else bench_multi(hisq, inputs, torch, dev)
    batched_cg = None if (args.kernels_only or args.solve_only) else bench_batched_cg(hisq, inputs, torch, dev)
    stability = None if (args.kernels_only or args.no_stability or args.solve_only) else bench_cg_stability(
        hisq, inputs, torch, dev)
    bicg = None
    if args.bicgstab:
        bicg = bench_bicgstab(hisq, inputs, torch, dev, tuple(int(v) for v in args.bicgstab.split(",")),
                              args.bicgstab_mass, args.bicgstab_links)
    formats = bench_formats(hisq, inputs, torch, dev, args.dslash_reps) if args.formats else None
    if args.kernels_only:
        tuning = hisq.hisq_tune_report().strip().splitlines()
        print(json.dumps(dict(kernels=kernels, batched=batched, multi_lattice=multi, tuning=tuning, formats=formats,
                              config={"lattice": list(dims)})))
        return
    gauges.clear()
    torch.cuda.empty_cache()

    # ---------------- the timed step ----------------
    ms_recon = args.ms_recon if hisq.fmt(args.ms).compute == 64 else args.recon   # eight parameters: FP64 only
    if args.ms_shape:
        stage, block, grid, order = (int(v) for v in args.ms_shape.split(","))
        hisq.hisq_tune_set(args.ms, dims, 1, 1, 1, stage, block, grid, sweep=order, long_recon=ms_recon)
        log(f"[bench] multi-shift operator pinned: stage {stage} block {block} grid {grid} order {order}")

    def solve_once(ms, ref, ms_long=None, **kw):
        """pack the links the solve needs (FP64 + its two triplets) and run it;
        ms_long: long-link storage of the multi-shift operator (default --recon)"""
        f_ms, f_ref = hisq.fmt(ms), hisq.fmt(ref)
        # the FP64 operator of the reliable updates and true residuals: FP64 links, the
        # long ones as two rows when --recon 12 (rebuilt to within FP64 rounding)
        g64 = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64, long_recon=args.recon)
        rms = ms_long or args.recon
        gms = hisq.pack_gauge(fat, lng, dims, f_ms.gauge, long_recon=rms)
        gref = gms if (f_ref.gauge == f_ms.gauge and rms == args.recon) else hisq.pack_gauge(
            fat, lng, dims, f_ref.gauge, long_recon=args.recon)
        if args.no_graph:
            kw["use_graph"] = 0
        if args.grad_buffer:
            kw["grad_buffer"] = args.grad_buffer
        return hisq.multishift_cg_solve(b, shifts, tols, g64, gms, gref, args.mass, ms_fmt=ms, ref_fmt=ref, **kw)

    def step():
        return solve_once(args.ms, args.ref, ms_long=ms_recon, batch_refine=args.batch_refine,
                          shift_floor=args.shift_floor)

    def timed_once(ms, ref, **kw):
        """one warm-up solve (launch shapes of new keys are tuned there), then one timed"""
        xw, _ = solve_once(ms, ref, **kw)
        del xw
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xw, sw = solve_once(ms, ref, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        del xw
        torch.cuda.empty_cache()
        return dt, sw

    for w in range(args.warmup):
        log(f"[bench] warmup {w + 1}/{args.warmup}")
        xs, st = step()
        log(f"[bench]   {st['seconds']:.2f}s, ms iters {st['iters']}, refine {st['refine_iters']}, "
            f"resid max {max(st['shift_resid']):.2e}")
        del xs
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        xs, st = step()
        stats.append(st)
        log(f"[bench] step {k + 1}/{args.steps}: {st['seconds']:.2f}s (multi-shift {st['phase_seconds'][0]:.2f}, "
            f"base refinement {st['phase_seconds'][1]:.2f}, shifted refinement {st['phase_seconds'][2]:.2f}), "
            f"ms iters {st['iters']}, refine {st['refine_iters']}, resid max {max(st['shift_resid']):.2e}")
        if k + 1 < args.steps:
            del xs
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed / args.steps * 1e3
    if args.solve_only:
        print(json.dumps(dict(ms_per_step=round(ms_per_step, 2), steps=[
            dict(seconds=round(st_["seconds"], 4), phase_seconds=[round(v, 4) for v in st_["phase_seconds"]],
                 ms_iters=st_["iters"], refine_iters=st_["refine_iters"], reliable_updates=st_["reliable_updates"],
                 dslash_sloppy=st_["dslash_sloppy"], dslash_f64=st_["dslash_f64"]) for st_ in stats],
            config={"workload": f"multishift_cg_{'x'.join(map(str, dims))}", "ms_triplet": repr(fms),
                    "refine_triplet": repr(fref), "ms_long_recon": ms_recon, "long_recon": args.recon,
                    "batch_refine": args.batch_refine, "graphs": not args.no_graph,
                    "shift_floor": args.shift_floor or "auto", "grad_buffer": args.grad_buffer or 8,
                    "ms_shape": args.ms_shape or "tuned"})))
        return
    # packing: every packed field reads its FP64 source once and writes its storage
    def pack_field_bytes(gf, recon):
        return 4 * V * (2 * 144 + hisq.GAUGE_BYTES[gf] + long_link_bytes(hisq, gf, recon))
    rms = ms_recon
    pack_bytes = pack_field_bytes(hisq.GAUGE_F64, args.recon) + pack_field_bytes(fms.gauge, rms)
    if fref.gauge != fms.gauge or rms != args.recon:
        pack_bytes += pack_field_bytes(fref.gauge, args.recon)
    step_bytes = float(np.mean([s["alg_bytes"] for s in stats])) + pack_bytes
    value = step_bytes / (ms_per_step / 1e3) / 1e9
    last = stats[-1]
    resid_ok = all(r <= t * (1 + 1e-6) for r, t in zip(last["shift_resid"], tols))

    tuning = hisq.hisq_tune_report().strip().splitlines()
    for line in tuning:
        log(f"[bench] tuned: {line}")

    # ---------------- FP64 GPU multi-shift comparator ----------------
    fp64 = None
    if not args.no_fp64:
        log("[bench] FP64 multi-shift comparator (all-FP64 multi-shift CG, no reliable updates)")
        del xs
        torch.cuda.empty_cache()
        # its multi-shift operator stores the long links as the mixed solve's does
        t64, st64 = timed_once("double", "double", ms_long=ms_recon, delta=0.0)
        fp64 = dict(seconds=round(t64, 3), ms_long_recon=ms_recon, iters=st64["iters"],
                    refine_iters=st64["refine_iters"],
                    phase_seconds=[round(v, 3) for v in st64["phase_seconds"]],
                    resid_max=max(st64["shift_resid"]), speedup_mixed=round(t64 / (ms_per_step / 1e3), 3))
        log(f"[bench]   FP64: {t64:.2f}s, iters {st64['iters']}, refine {st64['refine_iters']}")
    fp64_cg = None
    if args.fp64_cg:
        log("[bench] FP64 CG per shift (one plain FP64 CG solve per shift, no reliable updates)")
        g64c = hisq.pack_gauge(fat, lng, dims, hisq.GAUGE_F64, long_recon=args.recon)
        hisq.cg_solve(b, g64c, g64c, args.mass, shift=shifts[-1], tol=args.tol, sloppy="double", delta=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, res = [], []
        for sv, tv in zip(shifts, tols):
            x1, s1 = hisq.cg_solve(b, g64c, g64c, args.mass, shift=sv, tol=tv, sloppy="double", delta=0.0)
            its.append(s1["iters"])
            res.append(float(f"{s1['true_resid']:.3g}"))
            del x1
        torch.cuda.synchronize()
        tcg = time.perf_counter() - t0
        fp64_cg = dict(seconds=round(tcg, 3), iters=its, resid=res,
                       speedup_mixed=round(tcg / (ms_per_step / 1e3), 3))
        log(f"[bench]   FP64 CG per shift: {tcg:.2f}s, iters {its}")
        del g64c
        torch.cuda.empty_cache()
    alt = None
    if not args.no_alt:
        log("[bench] mixed double-single-half multi-shift")
        ta, sa = timed_once("single", "half", batch_refine=args.batch_refine)
        alt = dict(ms_triplet="f32/f32/fp32", refine_triplet="fix16/half16/fp32", seconds=round(ta, 3),
                   phase_seconds=[round(v, 3) for v in sa["phase_seconds"]],
                   ms_iters=sa["iters"], refine_iters=sa["refine_iters"], resid_max=max(sa["shift_resid"]),
                   resid_after_ms=[float(f"{r:.3g}") for r in sa["shift_resid_ms"]])
        log(f"[bench]   double-single-half: {ta:.2f}s, ms iters {sa['iters']}, refine {sa['refine_iters']}")

    # ---------------- roofline of the dominant kernel ----------------
    dom = args.ms if rms == 18 else f"{args.ms}_r{rms}"
    kd = kernels[dom]
    traffic = counter_traffic(f"k_dslash<{kd['triplet']}>", dims, rms)
    roofline = dict(bound="hbm", achieved=kd["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(kd["gbs"] / HBM_PEAK_GBS, 4), traffic=traffic,
                    traffic_over_alg=round(traffic / kd["alg_bytes"], 3) if traffic else None,
                    kernel=f"k_dslash<{kd['triplet']}>", alg_bytes_per_launch=kd["alg_bytes"],
                    us_per_launch=kd["us"])

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(np, dims, fat, lng, b, shifts, tols, args.mass, kernels,
                           fp64["iters"] if fp64 else None, ms_per_step / 1e3)
        cpu["cg_time_to_solution"] = cg_time_to_solution(np, hisq, inputs, torch, dev, batched_cg)

    line = {
        "metric": "HISQ Dslash GB/s (% HBM peak); multi-shift CG s to 1e-10 vs FP64 CG",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic (seeded near-unit SU(3) links exp(0.3iH), Gaussian source)",
        "config": {"workload": f"multishift_cg_{'x'.join(map(str, dims))}", "lattice": list(dims),
                   "mass": args.mass, "shifts": [float(f"{s:.4g}") for s in shifts], "tol": args.tol,
                   "ms_triplet": repr(fms), "refine_triplet": repr(fref), "long_recon": args.recon,
                   "ms_long_recon": rms,
                   "batch_refine": args.batch_refine, "graphs": not args.no_graph,
                   "shift_floor": args.shift_floor or "auto", "grad_buffer": args.grad_buffer or 8,
                   "ms_shape": args.ms_shape or "tuned", "parallelism": "single GPU"},
        "multishift": {"mixed_seconds": round(ms_per_step / 1e3, 3), "ms_iters": last["iters"],
                       "phase_seconds": [round(v, 3) for v in last["phase_seconds"]],
                       "refine_iters": last["refine_iters"], "reliable_updates": last["reliable_updates"],
                       "resid_after_ms": [float(f"{r:.3g}") for r in last["shift_resid_ms"]],
                       "resid": [float(f"{r:.3g}") for r in last["shift_resid"]], "all_converged": resid_ok,
                       "step_alg_bytes": step_bytes, "fp64_gpu": fp64, "fp64_cg_per_shift": fp64_cg,
                       "double_single_half": alt},
        "kernels": kernels,
        "batched": batched,
        "multi_lattice": multi,
        "batched_cg": batched_cg,
        "cg_stability": stability,
        "bicgstab": bicg,
        "formats": formats,
        "tuning": tuning,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
