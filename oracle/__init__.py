"""FP64 CPU oracle for the HISQ hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the HIP implementation; the only thing both sides take from a common
place is their seeded inputs.

The arithmetic lives in ``hisq_oracle.c`` (plain C, FP64); this module
compiles it with gcc on first use and wraps it with numpy arrays.  Fields use
the canonical layouts: links complex128 ``[4, V, 3, 3]``, full-lattice
spinors complex128 ``[V, 3]`` (see ``paper_2302_09224_amd.inputs``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hisq_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True, out: str | None = None, src: str | None = None) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over sites); returns the path."""
    out = out or _LIB_PATH
    src = src or _SRC
    # -ffp-contract=off: the oracle's arithmetic is exactly what its source writes
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", out + ".tmp", src,
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _declare(lib):
    vp = ctypes.c_void_p
    lib.hisq_oracle_dslash.argtypes = [vp, vp, vp, vp, _c_int_p, ctypes.c_int]
    lib.hisq_oracle_dslash_sites.argtypes = [vp, vp, vp, vp, _c_int_p, vp, ctypes.c_long]
    lib.hisq_oracle_normal.argtypes = [vp, vp, vp, vp, vp, _c_int_p, ctypes.c_int, ctypes.c_double]
    lib.hisq_oracle_true_residual.argtypes = [vp, vp, vp, vp, _c_int_p, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double]
    lib.hisq_oracle_true_residual.restype = ctypes.c_double
    lib.hisq_oracle_cg.argtypes = [vp, vp, vp, vp, _c_int_p, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, _c_int_p, _c_dbl_p]
    lib.hisq_oracle_cg.restype = ctypes.c_int
    lib.hisq_oracle_multishift_cg.argtypes = [vp, vp, vp, vp, _c_int_p, ctypes.c_int, ctypes.c_double,
                                              vp, ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.hisq_oracle_multishift_cg.restype = ctypes.c_int
    lib.hisq_oracle_threads.argtypes = []
    lib.hisq_oracle_threads.restype = ctypes.c_int
    lib.hisq_oracle_set_threads.argtypes = [ctypes.c_int]
    lib.hisq_oracle_set_threads.restype = None
    lib.hisq_oracle_phase_params.argtypes = [vp, vp, vp, ctypes.c_long]
    lib.hisq_oracle_phase_params.restype = None
    for name in ("half16_encode",):
        getattr(lib, "hisq_oracle_" + name).argtypes = [vp, vp, vp, ctypes.c_long]
    lib.hisq_oracle_half16_decode.argtypes = [vp, vp, vp, ctypes.c_long]
    for name in ("int20_encode", "int20_decode", "int30_encode", "int30_decode"):
        getattr(lib, "hisq_oracle_" + name).argtypes = [vp, vp, ctypes.c_long]
    for name in ("fix16_encode", "fix32_encode"):
        getattr(lib, "hisq_oracle_" + name).argtypes = [vp, vp, ctypes.c_long, ctypes.c_double]
    for name in ("fix16_decode", "fix32_decode"):
        getattr(lib, "hisq_oracle_" + name).argtypes = [vp, vp, ctypes.c_long, ctypes.c_double, ctypes.c_int]
    return lib


def load(path: str | None = None):
    """Load the compiled oracle (building it if it is missing or stale)."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if (not os.path.exists(_LIB_PATH)
                    or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
                build()
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dims(dims):
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    return d


def volume(dims):
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


def site_parities(dims):
    """parity (x+y+z+t)%2 of every lexicographic site"""
    X, Y, Z, T = dims
    i = np.arange(volume(dims))
    return ((i % X) + (i // X) % Y + (i // (X * Y)) % Z + i // (X * Y * Z)) % 2


def parity_sites(dims, parity):
    """lexicographic indices of one parity, in checkerboard order (i//2)"""
    return np.nonzero(site_parities(dims) == parity)[0]


def to_full(cb_field, dims, parity):
    """embed a checkerboard-ordered one-parity spinor in a full-lattice one"""
    full = np.zeros((volume(dims), 3), dtype=np.complex128)
    full[parity_sites(dims, parity)] = cb_field
    return full


def from_full(full, dims, parity):
    return np.ascontiguousarray(full[parity_sites(dims, parity)])


# ---------------------------------------------------------------------------
# operator and solvers
# ---------------------------------------------------------------------------

def threads(lib=None):
    """number of OpenMP threads the oracle's site loops use"""
    return (lib or load()).hisq_oracle_threads()


def set_threads(n, lib=None):
    """use n OpenMP threads in the oracle's site loops from now on"""
    (lib or load()).hisq_oracle_set_threads(int(n))


def dslash(fat, lng, psi, dims, parity=-1, out=None, lib=None):
    """(D psi) on the sites of `parity` (all sites for -1); other sites of
    `out` are left as they were (zeros for a fresh output)."""
    lib = lib or load()
    fat = _arr(fat, np.complex128)
    lng = _arr(lng, np.complex128)
    psi = _arr(psi, np.complex128)
    V = volume(dims)
    assert fat.size == 36 * V and lng.size == 36 * V and psi.size == 3 * V
    if out is None:
        out = np.zeros((V, 3), dtype=np.complex128)
    lib.hisq_oracle_dslash(_ptr(out), _ptr(fat), _ptr(lng), _ptr(psi), _dims(dims), int(parity))
    return out


def dslash_sites(fat, lng, psi, dims, sites, lib=None):
    """(D psi)(x) at the listed lexicographic sites, complex128 [n, 3]"""
    lib = lib or load()
    fat = _arr(fat, np.complex128)
    lng = _arr(lng, np.complex128)
    psi = _arr(psi, np.complex128)
    sites = _arr(sites, np.int64)
    out = np.zeros((sites.size, 3), dtype=np.complex128)
    lib.hisq_oracle_dslash_sites(_ptr(out), _ptr(fat), _ptr(lng), _ptr(psi), _dims(dims),
                                 _ptr(sites), sites.size)
    return out


def normal_op(fat, lng, v, dims, mass, shift=0.0, parity=0, lib=None):
    """(4m^2 + shift) v - D_pq D_qp v for a full-lattice v supported on parity p"""
    lib = lib or load()
    fat = _arr(fat, np.complex128)
    lng = _arr(lng, np.complex128)
    v = _arr(v, np.complex128)
    V = volume(dims)
    out = np.zeros((V, 3), dtype=np.complex128)
    tmp = np.zeros((V, 3), dtype=np.complex128)
    lib.hisq_oracle_normal(_ptr(out), _ptr(v), _ptr(tmp), _ptr(fat), _ptr(lng), _dims(dims),
                           int(parity), 4.0 * mass * mass + shift)
    return out


def true_residual(fat, lng, x, b, dims, mass, shift=0.0, parity=0, lib=None):
    lib = lib or load()
    fat = _arr(fat, np.complex128)
    lng = _arr(lng, np.complex128)
    x = _arr(x, np.complex128)
    b = _arr(b, np.complex128)
    return lib.hisq_oracle_true_residual(_ptr(x), _ptr(b), _ptr(fat), _ptr(lng), _dims(dims),
                                         int(parity), float(mass), float(shift))


def cg(fat, lng, b, dims, mass, shift=0.0, tol=1e-10, maxiter=100000, x0=None, parity=0, lib=None):
    """plain FP64 CG; returns (x, iterations, true relative residual, status)"""
    lib = lib or load()
    fat = _arr(fat, np.complex128)
    lng = _arr(lng, np.complex128)
    b = _arr(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else _arr(x0, np.complex128).copy()
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    st = lib.hisq_oracle_cg(_ptr(x), _ptr(b), _ptr(fat), _ptr(lng), _dims(dims), int(parity),
                            float(mass), float(shift), float(tol), int(maxiter),
                            ctypes.byref(it), ctypes.byref(res))
    return x, it.value, res.value, st


def multishift_cg(fat, lng, b, dims, mass, shifts, tol, maxiter=100000, parity=0, lib=None, residuals=True):
    """FP64 multi-shift CG; returns dict(x=[...], iters, resid, zeta, r, status)
    (residuals=False: the final true residuals are not computed, resid is zero)"""
    lib = lib or load()
    fat = _arr(fat, np.complex128)
    lng = _arr(lng, np.complex128)
    b = _arr(b, np.complex128)
    shifts = _arr(shifts, np.float64)
    n = shifts.size
    tol = _arr(np.broadcast_to(np.asarray(tol, dtype=np.float64), (n,)), np.float64)
    xs = [np.zeros_like(b) for _ in range(n)]
    xp = (ctypes.c_void_p * n)(*[x.ctypes.data for x in xs])
    iters = np.zeros(n, dtype=np.int32)
    resid = np.zeros(n, dtype=np.float64)
    zeta = np.zeros(n, dtype=np.float64)
    r = np.zeros_like(b)
    st = lib.hisq_oracle_multishift_cg(ctypes.cast(xp, ctypes.c_void_p), _ptr(b), _ptr(fat), _ptr(lng),
                                       _dims(dims), int(parity), float(mass), _ptr(shifts), n, _ptr(tol),
                                       int(maxiter), _ptr(iters), _ptr(resid) if residuals else None, _ptr(zeta),
                                       _ptr(r))
    return dict(x=xs, iters=iters, resid=resid, zeta=zeta, r=r, status=st)


def full_op(fat, lng, x, dims, mass, lib=None):
    """M x = 2m x + D x on the whole lattice (the unpreconditioned HISQ operator;
    its even-site Schur complement M^dag M |_even is 4m^2 - D_eo D_oe)"""
    return 2.0 * mass * _arr(x, np.complex128) + dslash(fat, lng, x, dims, -1, lib=lib)


def bicgstab_l(fat, lng, b, dims, mass, l=4, tol=1e-10, maxiter=100000, x0=None, lib=None, on_mr=None):
    """FP64 BiCGStab(l) (Sleijpen and Fokkema 1993, the method Sec. 6.1 runs in
    mixed precision) for M x = b on the whole lattice, M = 2m + D.
    Each cycle: l BiCG steps (building u_0..u_l and r_0..r_l with one shadow
    residual), then the minimal-residual step over r_1..r_l by modified
    Gram-Schmidt.  Inner products <a, b> = a^H b.  Returns (x, matvecs, true
    relative residual, status 0 converged / 1 iteration cap / 2 breakdown).
    on_mr(r0, rhat): test hook called after every minimal-residual step with the
    new r_0 and the orthogonalised r_1..r_l."""
    b = _arr(b, np.complex128)
    M = lambda v: full_op(fat, lng, v, dims, mass, lib)
    x = np.zeros_like(b) if x0 is None else _arr(x0, np.complex128).copy()
    r = [b - M(x)] + [np.zeros_like(b) for _ in range(l)]
    u = [np.zeros_like(b) for _ in range(l + 1)]
    rt = r[0].copy()
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0, 0
    k = 0
    status = 1
    while k < maxiter:
        if np.linalg.norm(r[0]) <= tol * bn:
            status = 0
            break
        rho0 = -omega * rho0
        # BiCG part
        for j in range(l):
            rho1 = np.vdot(rt, r[j])
            if rho0 == 0:
                return x, k, np.linalg.norm(b - M(x)) / bn, 2
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = M(u[j])
            gam = np.vdot(rt, u[j + 1])
            if gam == 0:
                return x, k, np.linalg.norm(b - M(x)) / bn, 2
            alpha = rho0 / gam
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = M(r[j])
            x = x + alpha * u[0]
            k += 2
        # minimal-residual part
        tau = np.zeros((l + 1, l + 1), dtype=np.complex128)
        sigma = np.zeros(l + 1)
        gp = np.zeros(l + 1, dtype=np.complex128)
        for j in range(1, l + 1):
            for i in range(1, j):
                tau[i, j] = np.vdot(r[i], r[j]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = np.vdot(r[j], r[j]).real
            if sigma[j] == 0.0:
                return x, k, np.linalg.norm(b - M(x)) / bn, 2
            gp[j] = np.vdot(r[j], r[0]) / sigma[j]
        g = np.zeros(l + 1, dtype=np.complex128)
        g[l] = gp[l]
        omega = g[l]
        for j in range(l - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, l + 1))
        gpp = np.zeros(l + 1, dtype=np.complex128)
        for j in range(1, l):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, l))
        x = x + g[1] * r[0]
        r[0] = r[0] - gp[l] * r[l]
        u[0] = u[0] - g[l] * u[l]
        for j in range(1, l):
            u[0] = u[0] - g[j] * u[j]
            x = x + gpp[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        if on_mr is not None:
            on_mr(r[0], r[1:])
    res = np.linalg.norm(b - M(x)) / bn
    return x, k, res, status


# ---------------------------------------------------------------------------
# storage codecs (per-site records)
# ---------------------------------------------------------------------------

def _reals6(v, dtype):
    """complex [n,3] or real [n,6] -> contiguous real [n,6] of dtype"""
    v = np.asarray(v)
    if np.iscomplexobj(v):
        v = np.stack([v.real, v.imag], axis=-1).reshape(v.shape[0], 6)
    return np.ascontiguousarray(v, dtype=dtype).reshape(-1, 6)


def _complex3(r):
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3, 2)
    return r[..., 0] + 1j * r[..., 1]


def half16_encode(v, lib=None):
    """QUDA half spinor: (q int16 [n,6], norm float32 [n]); input rounded to FP32"""
    lib = lib or load()
    a = _reals6(v, np.float32)
    n = a.shape[0]
    q = np.zeros((n, 6), dtype=np.int16)
    nm = np.zeros(n, dtype=np.float32)
    lib.hisq_oracle_half16_encode(_ptr(a), _ptr(q), _ptr(nm), n)
    return q, nm


def half16_decode(q, norm, lib=None):
    lib = lib or load()
    q = _arr(q, np.int16).reshape(-1, 6)
    nm = _arr(norm, np.float32)
    v = np.zeros((q.shape[0], 6), dtype=np.float32)
    lib.hisq_oracle_half16_decode(_ptr(q), _ptr(nm), _ptr(v), q.shape[0])
    return v


def int20_encode(v, lib=None):
    """20-bit shared-exponent spinor: uint32 [n,4]; input rounded to FP32"""
    lib = lib or load()
    a = _reals6(v, np.float32)
    w = np.zeros((a.shape[0], 4), dtype=np.uint32)
    lib.hisq_oracle_int20_encode(_ptr(a), _ptr(w), a.shape[0])
    return w


def int20_decode(w, lib=None):
    lib = lib or load()
    w = _arr(w, np.uint32).reshape(-1, 4)
    v = np.zeros((w.shape[0], 6), dtype=np.float32)
    lib.hisq_oracle_int20_decode(_ptr(w), _ptr(v), w.shape[0])
    return v


def int30_encode(v, lib=None):
    """30-bit shared-exponent spinor: uint32 [n,6]; FP64 input"""
    lib = lib or load()
    a = _reals6(v, np.float64)
    w = np.zeros((a.shape[0], 6), dtype=np.uint32)
    lib.hisq_oracle_int30_encode(_ptr(a), _ptr(w), a.shape[0])
    return w


def int30_decode(w, lib=None):
    lib = lib or load()
    w = _arr(w, np.uint32).reshape(-1, 6)
    v = np.zeros((w.shape[0], 6), dtype=np.float64)
    lib.hisq_oracle_int30_decode(_ptr(w), _ptr(v), w.shape[0])
    return v


# ---------------------------------------------------------------------------
# the shared-exponent family (Sec. 4): the 20- and 30-bit spinors are two
# members of one rule with component width B.  Written here once more in
# numpy, independently of the C codecs above, so that B = 20 and B = 30 can
# be checked against them (and through them against the worked examples of
# Appendix A and Listing 3); B = 24 (20 bytes per site) is the generated member.
# ---------------------------------------------------------------------------

def shared_exponent_words(bits):
    """32-bit words of one site record: six B-bit components and an 8-bit exponent"""
    return (6 * bits + 8 + 31) // 32


def _shared_exponent_fields(bits):
    """(word, bit offset, width) of re0, im0, re1, im1, re2, im2, E: the fields
    follow one another from the least significant bit of word 0 (Appendix A)"""
    return [((f * bits) // 32, (f * bits) % 32, bits if f < 6 else 8) for f in range(7)]


def shared_exponent_encode(v, bits):
    """records uint32 [n, words] of colour vectors v in the B-bit member.
    M = max |component| of the site; t = M / (2^(B-1) - 1); the stored exponent
    E is the biased exponent of t plus one (t rounded up to a power of two),
    clamped to [1, 254] (1 for t = 0); q = round-half-even(v * 2^(127-E)).  The
    arithmetic is FP32 for B <= 24 (the input is first rounded to FP32, as for
    the 20-bit format) and FP64 above (as for the 30-bit format).  A field that
    crosses a word boundary keeps its high bits at the top of the earlier word
    and its low bits at the bottom of the next one (Appendix A)."""
    ft = np.float32 if bits <= 24 else np.float64
    a = _reals6(v, ft)
    m = np.abs(a).max(axis=1)
    t = m / ft(2 ** (bits - 1) - 1)
    _, ex = np.frexp(t)                        # t = f 2^ex, f in [1/2, 1): unbiased exponent ex - 1
    e = np.where(t > 0, ex.astype(np.int64) + 127, 1).clip(1, 254)
    inv = np.ldexp(ft(1.0), (127 - e).astype(np.int32)).astype(ft)
    q = np.rint(a * inv[:, None]).astype(np.int64)
    vals = [q[:, k] & ((1 << bits) - 1) for k in range(6)] + [e]
    words = np.zeros((a.shape[0], shared_exponent_words(bits)), dtype=np.uint64)
    for val, (k, off, width) in zip(vals, _shared_exponent_fields(bits)):
        val = val.astype(np.uint64)
        spill = off + width - 32               # bits that go to the next word
        if spill <= 0:
            words[:, k] |= val << np.uint64(off)
        else:
            words[:, k] |= (val >> np.uint64(spill)) << np.uint64(off)
            words[:, k + 1] |= val & np.uint64((1 << spill) - 1)
    return (words & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def shared_exponent_decode(w, bits):
    """reals [n, 6] (FP32 for B <= 24, else FP64) of records of the B-bit member:
    v = q * 2^(E-127) with q the B-bit two's-complement components"""
    ft = np.float32 if bits <= 24 else np.float64
    w = np.asarray(w, dtype=np.uint32).reshape(-1, shared_exponent_words(bits)).astype(np.uint64)
    vals = []
    for k, off, width in _shared_exponent_fields(bits):
        spill = off + width - 32
        if spill <= 0:
            x = (w[:, k] >> np.uint64(off)) & np.uint64((1 << width) - 1)
        else:
            hi = (w[:, k] >> np.uint64(off)) & np.uint64((1 << (width - spill)) - 1)
            x = (hi << np.uint64(spill)) | (w[:, k + 1] & np.uint64((1 << spill) - 1))
        vals.append(x.astype(np.int64))
    q = np.stack(vals[:6], axis=1)
    q = np.where(q >= 2 ** (bits - 1), q - 2 ** bits, q)
    scale = np.ldexp(ft(1.0), (vals[6] - 127).astype(np.int32)).astype(ft)
    return q.astype(ft) * scale[:, None]


def int24_encode(v, lib=None):
    """24-bit shared-exponent spinor (generated member): uint32 [n,5]; FP32 input"""
    return shared_exponent_encode(v, 24)


def int24_decode(w, lib=None):
    return shared_exponent_decode(w, 24)


def field_absmax(u):
    """global max over the real and imaginary parts of a link field"""
    u = np.asarray(u)
    return float(max(np.abs(u.real).max(), np.abs(u.imag).max())) if u.size else 0.0


def fix_encode(u, bits, absmax=None, lib=None):
    """fixed-point gauge: complex links -> int16/int32 array of the real
    components (re, im interleaved), scaled by the global max"""
    lib = lib or load()
    absmax = field_absmax(u) if absmax is None else float(absmax)
    r = np.ascontiguousarray(np.asarray(u, dtype=np.complex128)).view(np.float64).ravel()
    if bits == 16:
        q = np.zeros(r.size, dtype=np.int16)
        lib.hisq_oracle_fix16_encode(_ptr(r), _ptr(q), r.size, absmax)
    elif bits == 32:
        q = np.zeros(r.size, dtype=np.int32)
        lib.hisq_oracle_fix32_encode(_ptr(r), _ptr(q), r.size, absmax)
    else:
        raise ValueError(bits)
    return q, absmax


def fix_decode(q, absmax, compute_bits, shape=None, lib=None):
    """fixed-point gauge -> complex128 (values exactly as the compute precision sees them)"""
    lib = lib or load()
    q = np.ascontiguousarray(q)
    u = np.zeros(q.size, dtype=np.float64)
    if q.dtype == np.int16:
        lib.hisq_oracle_fix16_decode(_ptr(q), _ptr(u), q.size, float(absmax), int(compute_bits))
    elif q.dtype == np.int32:
        lib.hisq_oracle_fix32_decode(_ptr(q), _ptr(u), q.size, float(absmax), int(compute_bits))
    else:
        raise ValueError(q.dtype)
    c = u.view(np.complex128)
    return c.reshape(shape) if shape is not None else c


# ---------------------------------------------------------------------------
# storage emulation: what a field looks like after a round trip through a format
# ---------------------------------------------------------------------------

SPINOR_FORMATS = ("f64", "f32", "half16", "int20", "int30", "int24")
GAUGE_FORMATS = ("f64", "f32", "fix16", "fix32", "sx24")


def spinor_roundtrip(v, fmt, lib=None):
    """complex [n,3] -> complex128 [n,3] after encode+decode in `fmt`"""
    v = np.asarray(v, dtype=np.complex128).reshape(-1, 3)
    if fmt == "f64":
        return v.copy()
    if fmt == "f32":
        return v.astype(np.complex64).astype(np.complex128)
    if fmt == "half16":
        q, nm = half16_encode(v, lib)
        return _complex3(half16_decode(q, nm, lib))
    if fmt == "int20":
        return _complex3(int20_decode(int20_encode(v, lib), lib))
    if fmt == "int30":
        return _complex3(int30_decode(int30_encode(v, lib), lib))
    if fmt == "int24":
        return _complex3(int24_decode(int24_encode(v)))
    raise ValueError(fmt)


def spinor_decode_records(rec, fmt, lib=None):
    """per-site records of a format -> complex128 [n,3].
    rec: f64 complex [n,3]; f32 complex64 [n,3]; half16 (q [n,6], norm [n]);
    int20 uint32 [n,4]; int30 uint32 [n,6]; int24 uint32 [n,5]"""
    if fmt in ("f64", "f32"):
        return np.asarray(rec).astype(np.complex128).reshape(-1, 3)
    if fmt == "half16":
        q, nm = rec
        return _complex3(half16_decode(q, nm, lib))
    if fmt == "int20":
        return _complex3(int20_decode(rec, lib))
    if fmt == "int30":
        return _complex3(int30_decode(rec, lib))
    if fmt == "int24":
        return _complex3(int24_decode(rec))
    raise ValueError(fmt)


def sx24_rows_encode(u):
    """link rows (complex [..., nrow, 3]) as 24-bit shared-exponent records,
    uint32 [..., nrow, 5]: each colour row is one record of the B = 24 member"""
    u = np.asarray(u, dtype=np.complex128)
    return shared_exponent_encode(u.reshape(-1, 3), 24).reshape(u.shape[:-1] + (5,))


def sx24_rows_roundtrip(u):
    u = np.asarray(u, dtype=np.complex128)
    return _complex3(shared_exponent_decode(sx24_rows_encode(u).reshape(-1, 5), 24)).reshape(u.shape)


def gauge_roundtrip(u, fmt, compute_bits, lib=None):
    """links after encode in `fmt` and decode in the compute precision"""
    u = np.asarray(u, dtype=np.complex128)
    if fmt == "sx24":
        return sx24_rows_roundtrip(u)
    if fmt == "f64":
        return u.astype(np.complex64).astype(np.complex128) if compute_bits == 32 else u.copy()
    if fmt == "f32":
        return u.astype(np.complex64).astype(np.complex128)
    bits = {"fix16": 16, "fix32": 32}[fmt]
    q, absmax = fix_encode(u, bits, lib=lib)
    return fix_decode(q, absmax, compute_bits, shape=u.shape, lib=lib)


def spinor_quantum(v, fmt):
    """per-site storage quantum (spacing of representable values) of `fmt` for
    the site values v (complex [n,3]); used for rounding-flip tolerances"""
    v = np.asarray(v, dtype=np.complex128).reshape(-1, 3)
    m = np.maximum(np.abs(v.real).max(axis=1), np.abs(v.imag).max(axis=1))
    if fmt == "f64":
        return m * 2.0 ** -52
    if fmt == "f32":
        return m * 2.0 ** -23
    if fmt == "half16":
        return m / 32767.0
    if fmt == "int20":
        return m * 2.0 ** -18
    if fmt == "int30":
        return m * 2.0 ** -28
    if fmt == "int24":
        return m * 2.0 ** -22
    raise ValueError(fmt)


# ---------------------------------------------------------------------------
# two-row storage of the long links (Sec. 1, compression of special unitary
# matrices): the third row of U in SU(3) is conj(row 1 x row 2), because the
# rows are orthonormal and det U = 1.
# ---------------------------------------------------------------------------

def long_phases(dims):
    """float64 [4, V]: eta_mu(x) (eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
    eta_3 = (-1)^(x+y+z)) times -1 on the three-hop temporal link for
    t >= T-3 (antiperiodic time), the sign the long links carry"""
    X, Y, Z, T = dims
    i = np.arange(volume(dims))
    x, y, z, t = i % X, (i // X) % Y, (i // (X * Y)) % Z, i // (X * Y * Z)
    e = np.stack([np.zeros_like(x), x, x + y, x + y + z])
    e[3] += (t >= T - 3)
    return np.where(e % 2 == 1, -1.0, 1.0)


def su3_third_row(rows):
    """rows [..., 2, 3] (first two rows of a special unitary matrix) -> the
    third row conj(r1 x r2), [..., 3]"""
    a, b = rows[..., 0, :], rows[..., 1, :]
    c = np.empty(a.shape, dtype=np.complex128)
    for k in range(3):
        i, j = (k + 1) % 3, (k + 2) % 3
        c[..., k] = np.conj(a[..., i] * b[..., j] - a[..., j] * b[..., i])
    return c


def long_link_split(lng, dims):
    """L_mu(x) = c * phase_mu(x) * U_mu(x), U in SU(3), c real: returns
    (c, U).  det L = c^3 phase (phase^3 = phase), so c is the real cube root
    of phase * Re det L at every site; the sites must agree (c is global).
    Raises ValueError when they do not or U is not special unitary."""
    lng = np.asarray(lng, dtype=np.complex128)
    ph = long_phases(dims)
    det = np.linalg.det(lng.reshape(-1, 3, 3)).reshape(ph.shape)
    cs = np.cbrt((ph * det).real)
    c = float(np.mean(cs))
    if c == 0.0 or np.abs(cs - c).max() > 1e-12 * abs(c) or np.abs(det.imag).max() > 1e-12 * abs(c) ** 3:
        raise ValueError("long links are not c * phase * SU(3) with one real c")
    u = lng / (c * ph)[..., None, None]
    uh = np.conj(np.swapaxes(u, -1, -2))
    if np.abs(uh @ u - np.eye(3)).max() > 1e-12:
        raise ValueError("long links are not c * phase * SU(3): U is not unitary")
    return c, u


def long_recon_roundtrip(lng, dims, fmt, compute_bits, lib=None):
    """long links as a Dslash sees them when only two rows of U are stored in
    `fmt` (fixed-point scale: max |real component| of the whole of U) and the
    third is rebuilt; the rebuild is exact here (FP64), the kernel's own
    rounding of it is covered by the compute-precision tolerance"""
    c, u = long_link_split(lng, dims)
    rows = np.ascontiguousarray(u[..., :2, :])
    if fmt in ("fix16", "fix32"):
        scale = max(np.abs(u.real).max(), np.abs(u.imag).max())
        q, _ = fix_encode(rows, 16 if fmt == "fix16" else 32, absmax=scale, lib=lib)
        rows = fix_decode(q, scale, compute_bits, shape=rows.shape, lib=lib)
    elif fmt == "sx24":
        rows = sx24_rows_roundtrip(rows)
    elif fmt == "f32" or compute_bits == 32:
        rows = rows.astype(np.complex64).astype(np.complex128)
    full = np.concatenate([rows, su3_third_row(rows)[..., None, :]], axis=-2)
    return c * long_phases(dims)[..., None, None] * full


def su3_eight_params(u):
    """special unitary u [..., 3, 3] -> its eight stored reals [..., 8]:
    Re/Im of u[0,1], u[0,2] and u[1,0], then tan(arg(u[0,0])/4) and
    tan(arg(u[2,0])/4) (each in [-1, 1] for an argument in [-pi, pi])"""
    u = np.asarray(u, dtype=np.complex128)
    p = np.empty(u.shape[:-2] + (8,))
    for k, z in enumerate((u[..., 0, 1], u[..., 0, 2], u[..., 1, 0])):
        p[..., 2 * k], p[..., 2 * k + 1] = z.real, z.imag
    p[..., 6] = np.tan(np.angle(u[..., 0, 0]) / 4)
    p[..., 7] = np.tan(np.angle(u[..., 2, 0]) / 4)
    return p


def su3_from_eight(p):
    """the special unitary matrix with the given eight parameters (Sec. 1,
    "Compression": 8 of the 18 reals fix a special unitary matrix).  Row 1
    has unit norm, which fixes |u00|; column 1 has unit norm, which fixes
    |u20|; their phases are e^{i theta} with tan(theta/4) = v.  The rest of
    row 2 follows from two linear conditions, orthogonality to row 1 and
    u20 = conj(u01 u12 - u02 u11) (row 3 = conj(row 1 x row 2)), solved as a
    2x2 linear system; row 3 is then that cross product."""
    p = np.asarray(p, dtype=np.float64)
    shape = p.shape[:-1]
    p = p.reshape(-1, 8)
    a2, a3, b1 = p[:, 0] + 1j * p[:, 1], p[:, 2] + 1j * p[:, 3], p[:, 4] + 1j * p[:, 5]

    def unit(v):                       # e^{i theta}, v = tan(theta/4): e^{i theta/2} = (1 + iv)^2 / (1 + v^2)
        h = (1 + 1j * v) ** 2 / (1 + v * v)
        return h * h
    a1 = np.sqrt(np.maximum(1 - np.abs(a2) ** 2 - np.abs(a3) ** 2, 0.0)) * unit(p[:, 6])
    c1 = np.sqrt(np.maximum(1 - np.abs(a1) ** 2 - np.abs(b1) ** 2, 0.0)) * unit(p[:, 7])
    # [conj(a2) conj(a3); -a3 a2] (b2, b3) = (-conj(a1) b1, conj(c1))
    m = np.empty((p.shape[0], 2, 2), dtype=np.complex128)
    m[:, 0, 0], m[:, 0, 1], m[:, 1, 0], m[:, 1, 1] = np.conj(a2), np.conj(a3), -a3, a2
    rhs = np.stack([-np.conj(a1) * b1, np.conj(c1)], axis=-1)
    b23 = np.linalg.solve(m, rhs[..., None])[..., 0]
    row1 = np.stack([a1, a2, a3], axis=-1)
    row2 = np.stack([b1, b23[:, 0], b23[:, 1]], axis=-1)
    row3 = np.conj(np.cross(row1, row2))
    return np.stack([row1, row2, row3], axis=-2).reshape(shape + (3, 3))


def phase_param(z, lib=None):
    """tan(arg(z)/4) (0 for z = 0) by the fixed operation sequence of
    hisq_oracle_phase_params (the half-angle identities with r = |z| =
    sqrt(fma(x, x, y*y)); each branch free of cancellation), complex -> float64"""
    lib = lib or load()
    z = np.asarray(z, dtype=np.complex128)
    x = np.ascontiguousarray(z.real, dtype=np.float64)
    y = np.ascontiguousarray(z.imag, dtype=np.float64)
    v = np.zeros(x.shape, dtype=np.float64)
    lib.hisq_oracle_phase_params(_ptr(x), _ptr(y), _ptr(v), x.size)
    return v


LONG8_FORMATS = ("f64", "fix32")


def _long8_records(lng, ph, c, m, fmt, lib=None):
    """the eight-parameter records of long links lng [..., 3, 3] with phases ph
    [...], the global real c of L = c * phase * U and the long field's max
    |real component| m (the fixed-point scale of the entries)"""
    lng = np.asarray(lng, dtype=np.complex128)
    w = lng * (ph * np.sign(c))[..., None, None]
    z = np.stack([w[..., 0, 1], w[..., 0, 2], w[..., 1, 0],
                  phase_param(w[..., 0, 0], lib) + 1j * phase_param(w[..., 2, 0], lib)], axis=-1)
    if fmt == "f64":
        return np.ascontiguousarray(z).view(np.float64)
    q, _ = fix_encode(z[..., :3], 32, absmax=m, lib=lib)
    qv, _ = fix_encode(z[..., 3], 32, absmax=1.0, lib=lib)
    out = np.empty(z.shape[:-1] + (8,), dtype=np.int32)
    out[..., :6] = q.reshape(z.shape[:-1] + (6,))
    out[..., 6:] = qv.reshape(z.shape[:-1] + (2,))
    return out


def _long8_rebuild(rec, ph, c, m, fmt, lib=None):
    """links from their eight-parameter records (the inverse storage step of
    _long8_records, then su3_from_eight in FP64)"""
    if fmt == "f64":
        p = rec.astype(np.float64).copy()
    else:
        p = np.empty(rec.shape, dtype=np.float64)
        p[..., :6] = fix_decode(np.ascontiguousarray(rec[..., :6]), m, 64, lib=lib).view(np.float64).reshape(
            rec.shape[:-1] + (6,))
        p[..., 6:] = fix_decode(np.ascontiguousarray(rec[..., 6:]), 1.0, 64, lib=lib).view(np.float64).reshape(
            rec.shape[:-1] + (2,))
    p[..., :6] /= abs(c)
    return c * ph[..., None, None] * su3_from_eight(p)


def long_recon8_encode(lng, dims, fmt, lib=None):
    """long links L = c * phase * U (U special unitary) stored as eight
    parameters per link, [4, V, 8]: Re/Im of the entries (0,1), (0,2) and
    (1,0) of W = L * phase * sign(c) = |c| U (exact: sign flips only), then
    phase_param of W[0,0] and of W[2,0].  f64: the values; fix32: int32,
    q = rint(x * (2^31 - 1) / m) with m the long field's max |real
    component| for the entries and m = 1 for the two phase parameters.
    Only FP64-compute triplets use this storage (F64 or FIX32 links)."""
    if fmt not in LONG8_FORMATS:
        raise ValueError(f"eight-parameter long links in {fmt}")
    c, _ = long_link_split(lng, dims)
    return _long8_records(lng, long_phases(dims), c, field_absmax(lng), fmt, lib)


def long_recon8_roundtrip(lng, dims, fmt, compute_bits=64, lib=None):
    """long links as a Dslash sees them when stored by long_recon8_encode and
    rebuilt (su3_from_eight in FP64: the kernel's own FP64 rounding of the
    rebuild is covered by the tests' compute-precision allowance, amplified
    by the rebuild's conditioning)"""
    c, _ = long_link_split(lng, dims)
    m = field_absmax(lng)
    ph = long_phases(dims)
    return _long8_rebuild(_long8_records(lng, ph, c, m, fmt, lib), ph, c, m, fmt, lib)


def long8_links_roundtrip(lng, ph, c, m, fmt, lib=None):
    """long_recon8_roundtrip for a subset of the links of a field: lng
    [..., 3, 3], their phases ph [...] (from long_phases), the field's c and
    max |real component| m given"""
    if fmt not in LONG8_FORMATS:
        raise ValueError(f"eight-parameter long links in {fmt}")
    return _long8_rebuild(_long8_records(lng, ph, c, m, fmt, lib), ph, c, m, fmt, lib)


def emulated_dslash(fat, lng, psi, dims, parity, gauge_fmt, spinor_fmt, compute_bits, lib=None, long_recon=18):
    """FP64 Dslash of the inputs as the storage formats hold them (links and
    spinor after a round trip), before the output is stored.  long_recon=12:
    the long links kept as two rows (long_recon_roundtrip); 8: as eight
    parameters (long_recon8_roundtrip)."""
    f = gauge_roundtrip(fat, gauge_fmt, compute_bits, lib)
    if long_recon == 12:
        l = long_recon_roundtrip(lng, dims, gauge_fmt, compute_bits, lib)
    elif long_recon == 8:
        l = long_recon8_roundtrip(lng, dims, gauge_fmt, compute_bits, lib)
    else:
        l = gauge_roundtrip(lng, gauge_fmt, compute_bits, lib)
    p = spinor_roundtrip(psi, spinor_fmt, lib)
    return dslash(f, l, p, dims, parity, lib=lib)
