"""Write format_bounds.txt: the per-triplet error bounds of the GPU parity
tests, measured with the oracle alone.

The storage formats make the Dslash and the normal operator differ from the
unquantised FP64 operator by an amount the paper states only per format (the
epsilon of each spinor format, the fixed-point gauge of Sec. 2's footnote and
Sec. 4).  The bound of a triplet is 4 times the largest max-norm relative
error over five seeds at 16^4 (near-unit links), computed with the oracle's
format emulation (links and spinor after an encode/decode round trip in the
oracle codecs, the FP64 Dslash of those, the result stored in the spinor
format again; for the normal operator the intermediate odd-parity vector is
stored as well), plus the compute precision's own allowance eps_c per
operator application (1e-6 for FP32 arithmetic, 1e-13 for FP64: the
tolerances of the plain IEEE triplets).  The emulation leaves out only the
kernels' compute-precision rounding, which eps_c covers, and at most one
output quantum, which the stored result already carries.

    python tests/golden/make_format_bounds.py      # rewrites format_bounds.txt (about 2 minutes)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2302_09224_amd import inputs  # noqa: E402

# name: (gauge format, spinor format, compute bits)
TRIPLETS = {
    "double": ("f64", "f64", 64), "single": ("f32", "f32", 32), "int30": ("fix32", "int30", 64),
    "int30_fp32": ("fix32", "int30", 32), "int24": ("fix32", "int24", 32), "sx24": ("sx24", "int24", 32),
    "sx24_int30": ("sx24", "int30", 64), "int20": ("fix16", "int20", 32), "half": ("fix16", "half16", 32),
}
DIMS = (16, 16, 16, 16)
SEEDS = 5
MASS, SHIFT = 0.05, 0.01
FACTOR = 4.0


def rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def measure(seed):
    fat, lng = inputs.make_links(DIMS, "near_unit", seed=inputs.GAUGE_SEED + 500 + seed)
    fat, lng = fat.numpy(), lng.numpy()
    V = oracle.volume(DIMS)
    ev, od = oracle.parity_sites(DIMS, 0), oracle.parity_sites(DIMS, 1)
    psi = inputs.gaussian_spinor(V, inputs.SOURCE_SEED + 500 + seed).numpy()
    src = np.zeros_like(psi)
    src[od] = psi[od]
    ref = oracle.dslash(fat, lng, src, DIMS, 0)[ev]
    p = np.zeros_like(psi)
    p[ev] = psi[ev]
    ref_n = oracle.normal_op(fat, lng, p, DIMS, MASS, SHIFT)[ev]
    c = 4 * MASS * MASS + SHIFT
    out = {}
    for name, (gf, sf, cb) in TRIPLETS.items():
        fq = oracle.gauge_roundtrip(fat, gf, cb)
        errs = []
        for recon in (18, 12):
            lq = oracle.long_recon_roundtrip(lng, DIMS, gf, cb) if recon == 12 else oracle.gauge_roundtrip(lng, gf, cb)
            y = oracle.dslash(fq, lq, oracle.to_full(oracle.spinor_roundtrip(psi[od], sf), DIMS, 1), DIMS, 0)[ev]
            errs.append(rel_inf(oracle.spinor_roundtrip(y, sf), ref))
        lq = oracle.gauge_roundtrip(lng, gf, cb)
        pq = oracle.spinor_roundtrip(psi[ev], sf)
        t = oracle.dslash(fq, lq, oracle.to_full(pq, DIMS, 0), DIMS, 1)[od]
        t = oracle.spinor_roundtrip(t, sf)
        n = c * pq - oracle.dslash(fq, lq, oracle.to_full(t, DIMS, 1), DIMS, 0)[ev]
        out[name] = (max(errs), rel_inf(oracle.spinor_roundtrip(n, sf), ref_n))
    return out


def main():
    res = [measure(s) for s in range(SEEDS)]
    lines = [
        "# Per-triplet error bounds of the GPU parity tests (written by make_format_bounds.py; oracle only).",
        f"# Max-norm relative error against the unquantised FP64 operator, max over {SEEDS} seeds at 16^4",
        "# (near-unit links, gauge seeds 1500..1504, source seeds 2500..2504), times "
        f"{FACTOR:g}, plus eps_c (1e-6 FP32, 1e-13 FP64 compute) per operator application:",
        "# the Dslash (long links 18-real and two-row, the larger; one application) and the normal operator",
        f"# (4m^2 + s) p - D_eo D_oe p with m = {MASS}, s = {SHIFT} (two applications).",
        "# columns: triplet | dslash_max dslash_bound | normal_max normal_bound",
    ]
    for name, (_, _, cb) in TRIPLETS.items():
        eps_c = 1e-6 if cb == 32 else 1e-13
        d = max(r[name][0] for r in res)
        n = max(r[name][1] for r in res)
        lines.append(f"{name} | {d:.3e} {FACTOR * d + eps_c:.3e} | {n:.3e} {FACTOR * n + 2 * eps_c:.3e}")
    with open(os.path.join(HERE, "format_bounds.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
