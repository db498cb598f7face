"""Python binding of libhisq (ctypes).

The functions named ``hisq_*`` are one-to-one wrappers of the C ABI declared
in ``include/hisq.h``: they only marshal arguments (torch tensors become
device pointers, the current torch stream becomes the hipStream_t) and turn a
non-OK status into :class:`HisqError`.  The few helpers below them
(``pack_gauge``, ``pack_spinor``, ``cg_solve`` ...) allocate the output
tensors with torch and then call exactly one of those wrappers.  Every step
of the computation runs in the HIP kernels of libhisq; there is no CPU or
PyTorch fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhisq.so")

# storage formats (include/hisq.h)
SPINOR_F64, SPINOR_F32, SPINOR_HALF16, SPINOR_INT20, SPINOR_INT30, SPINOR_INT24 = range(6)
GAUGE_F64, GAUGE_F32, GAUGE_FIX16, GAUGE_FIX32, GAUGE_SX24 = range(5)
SPINOR_BYTES = {SPINOR_F64: 48, SPINOR_F32: 24, SPINOR_HALF16: 16, SPINOR_INT20: 16, SPINOR_INT30: 24,
                SPINOR_INT24: 20}
GAUGE_BYTES = {GAUGE_F64: 144, GAUGE_F32: 72, GAUGE_FIX16: 36, GAUGE_FIX32: 72, GAUGE_SX24: 60}
SPINOR_NAMES = {SPINOR_F64: "f64", SPINOR_F32: "f32", SPINOR_HALF16: "half16", SPINOR_INT20: "int20",
                SPINOR_INT30: "int30", SPINOR_INT24: "int24"}
GAUGE_NAMES = {GAUGE_F64: "f64", GAUGE_F32: "f32", GAUGE_FIX16: "fix16", GAUGE_FIX32: "fix32", GAUGE_SX24: "sx24"}

HISQ_MAX_SHIFTS = 32
HISQ_MAX_GRAD_BUFFER = 16

STATUS = {0: "HISQ_OK", -1: "HISQ_EINVAL", -2: "HISQ_EALIGN", -3: "HISQ_EHIP", -4: "HISQ_ENOCONV",
          -5: "HISQ_EBREAKDOWN", -6: "HISQ_EWORKSPACE", -7: "HISQ_ERANGE", -8: "HISQ_EIO"}


class hisq_fmt(ctypes.Structure):
    _fields_ = [("gauge", ctypes.c_int), ("spinor", ctypes.c_int), ("compute", ctypes.c_int)]

    def __repr__(self):
        return f"{GAUGE_NAMES[self.gauge]}/{SPINOR_NAMES[self.spinor]}/fp{self.compute}"


class hisq_gauge(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("fmt", ctypes.c_int), ("fat", ctypes.c_void_p),
                ("lng", ctypes.c_void_p), ("fat_max", ctypes.c_double), ("long_max", ctypes.c_double),
                ("long_recon", ctypes.c_int), ("long_coeff", ctypes.c_double)]


RECON_18, RECON_12, RECON_8 = 18, 12, 8
FIELD_SPINOR, FIELD_GAUGE = 1, 2


class hisq_field_header(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("fmt", ctypes.c_int), ("dims", ctypes.c_int * 4), ("nsites", ctypes.c_long),
                ("long_recon", ctypes.c_int), ("bytes0", ctypes.c_size_t), ("bytes1", ctypes.c_size_t)]


class hisq_solver_params(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("maxiter", ctypes.c_int), ("grad_buffer", ctypes.c_int),
                ("pr_beta", ctypes.c_int), ("reproject", ctypes.c_int), ("poll_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("shift_floor", ctypes.c_double), ("batch_refine", ctypes.c_int),
                ("ru_estimate", ctypes.c_int)]


class hisq_solver_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("dslash_sloppy", ctypes.c_int), ("dslash_f64", ctypes.c_int), ("true_resid", ctypes.c_double),
                ("seconds", ctypes.c_double), ("alg_bytes", ctypes.c_double), ("nshift", ctypes.c_int),
                ("shift_iters", ctypes.c_int * HISQ_MAX_SHIFTS),
                ("shift_resid_ms", ctypes.c_double * HISQ_MAX_SHIFTS),
                ("refine_iters", ctypes.c_int * HISQ_MAX_SHIFTS),
                ("shift_resid", ctypes.c_double * HISQ_MAX_SHIFTS),
                ("phase_seconds", ctypes.c_double * 3)]

    def as_dict(self):
        n = max(1, self.nshift)
        return dict(status=STATUS.get(self.status, self.status), iters=self.iters,
                    reliable_updates=self.reliable_updates, dslash_sloppy=self.dslash_sloppy,
                    dslash_f64=self.dslash_f64, true_resid=self.true_resid, seconds=self.seconds,
                    alg_bytes=self.alg_bytes, nshift=self.nshift,
                    shift_iters=list(self.shift_iters[:n]), shift_resid_ms=list(self.shift_resid_ms[:n]),
                    refine_iters=list(self.refine_iters[:n]), shift_resid=list(self.shift_resid[:n]),
                    phase_seconds=list(self.phase_seconds))


# named precision triplets gauge/fermion/compute (Sec. 4)
TRIPLETS = {
    "double": (GAUGE_F64, SPINOR_F64, 64),
    "single": (GAUGE_F32, SPINOR_F32, 32),
    "half": (GAUGE_FIX16, SPINOR_HALF16, 32),
    "int20": (GAUGE_FIX16, SPINOR_INT20, 32),
    "int30": (GAUGE_FIX32, SPINOR_INT30, 64),
    "int30_fp32": (GAUGE_FIX32, SPINOR_INT30, 32),
    "int24": (GAUGE_FIX32, SPINOR_INT24, 32),      # generated shared-exponent member
    "sx24": (GAUGE_SX24, SPINOR_INT24, 32),        # links and spinors both 24-bit shared-exponent records
    "sx24_int30": (GAUGE_SX24, SPINOR_INT30, 64),  # 24-bit shared-exponent links, 30-bit spinors, FP64
}


def fmt(name_or_tuple) -> hisq_fmt:
    t = TRIPLETS[name_or_tuple] if isinstance(name_or_tuple, str) else tuple(name_or_tuple)
    return hisq_fmt(*t)


class HisqError(RuntimeError):
    def __init__(self, status, where, msg):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


_lib = None


def load():
    """Load libhisq.so (built in-tree by ``paper_2302_09224_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_09224_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    ip = ctypes.POINTER(ctypes.c_int)
    G = ctypes.POINTER(hisq_gauge)
    P = ctypes.POINTER(hisq_solver_params)
    S = ctypes.POINTER(hisq_solver_stats)
    sig = {
        "hisq_gauge_bytes": (sz, [ip, i]),
        "hisq_spinor_bytes": (sz, [ctypes.c_long, i]),
        "hisq_gauge_pack": (i, [G, vp, vp, vp, vp, ip, i, vp]),
        "hisq_gauge_pack_recon": (i, [G, vp, vp, vp, vp, ip, i, i, vp]),
        "hisq_gauge_long_bytes": (sz, [ip, i, i]),
        "hisq_spinor_pack": (i, [vp, vp, ctypes.c_long, i, vp]),
        "hisq_spinor_unpack": (i, [vp, vp, ctypes.c_long, i, vp]),
        "hisq_dslash": (i, [vp, vp, G, i, hisq_fmt, vp]),
        "hisq_dslash_xpay": (i, [vp, vp, G, i, hisq_fmt, d, vp, d, vp]),
        "hisq_normal_op": (i, [vp, vp, vp, G, d, d, hisq_fmt, vp]),
        "hisq_normal_op_noalloc": (i, [vp, vp, G, d, d, hisq_fmt, vp]),
        "hisq_dslash_batched": (i, [vp, vp, G, i, hisq_fmt, i, vp]),
        "hisq_dslash_multi": (i, [i, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(G), i, hisq_fmt, vp]),
        "hisq_solver_params_default": (None, [P]),
        "hisq_cg_workspace_bytes": (sz, [ip, hisq_fmt, P]),
        "hisq_cg_solve": (i, [vp, vp, G, G, d, d, d, hisq_fmt, P, vp, sz, S, vp]),
        "hisq_multishift_workspace_bytes": (sz, [ip, i, hisq_fmt, hisq_fmt, P]),
        "hisq_multishift_cg_solve": (i, [ctypes.POINTER(vp), vp, ctypes.POINTER(d), i, ctypes.POINTER(d), G, G, G,
                                         d, hisq_fmt, hisq_fmt, P, vp, sz, S, vp]),
        "hisq_cg_batched_workspace_bytes": (sz, [ip, i, hisq_fmt, P]),
        "hisq_bicgstab_workspace_bytes": (sz, [ip, i, hisq_fmt]),
        "hisq_bicgstab_solve": (i, [vp, vp, G, G, d, d, i, hisq_fmt, P, vp, sz, S, vp]),
        "hisq_cg_solve_batched": (i, [vp, vp, i, G, G, d, d, d, hisq_fmt, P, vp, sz, S, vp]),
        "hisq_last_error": (ctypes.c_char_p, []),
        "hisq_version": (ctypes.c_char_p, []),
        "hisq_tune_report": (sz, [ctypes.c_char_p, sz]),
        "hisq_tune_set": (i, [hisq_fmt, ip, i, i, i, i, i, i, i, i]),
        "hisq_tune_set_fused": (i, [hisq_fmt, ip, i, i, i, i, i, i, i, i]),
        "hisq_tune_clear": (None, []),
        "hisq_tune_save": (i, [ctypes.c_char_p]),
        "hisq_tune_load": (i, [ctypes.c_char_p, ip]),
        "hisq_field_info": (i, [ctypes.c_char_p, ctypes.POINTER(hisq_field_header)]),
        "hisq_spinor_save": (i, [ctypes.c_char_p, vp, ctypes.c_long, i, vp]),
        "hisq_spinor_load": (i, [ctypes.c_char_p, vp, ctypes.c_long, i, vp]),
        "hisq_gauge_save": (i, [ctypes.c_char_p, G, vp]),
        "hisq_gauge_load": (i, [ctypes.c_char_p, G, vp, sz, vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status, where):
    if status != 0:
        raise HisqError(status, where, load().hisq_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("libhisq takes device tensors")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream=None):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(v) for v in dims])


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C ABI
# ---------------------------------------------------------------------------

def hisq_gauge_bytes(dims, gauge_fmt):
    return load().hisq_gauge_bytes(_dims(dims), int(gauge_fmt))


def hisq_gauge_long_bytes(dims, gauge_fmt, long_recon):
    return load().hisq_gauge_long_bytes(_dims(dims), int(gauge_fmt), int(long_recon))


def hisq_gauge_pack_recon(fat_dst, long_dst, fat_src, long_src, dims, gauge_fmt, long_recon, stream=None):
    g = hisq_gauge()
    _check(load().hisq_gauge_pack_recon(ctypes.byref(g), _ptr(fat_dst), _ptr(long_dst), _ptr(fat_src),
                                        _ptr(long_src), _dims(dims), int(gauge_fmt), int(long_recon),
                                        _stream(stream)), "hisq_gauge_pack_recon")
    return g


def hisq_spinor_bytes(nsites, spinor_fmt):
    return load().hisq_spinor_bytes(int(nsites), int(spinor_fmt))


def hisq_gauge_pack(fat_dst, long_dst, fat_src, long_src, dims, gauge_fmt, stream=None):
    g = hisq_gauge()
    _check(load().hisq_gauge_pack(ctypes.byref(g), _ptr(fat_dst), _ptr(long_dst), _ptr(fat_src), _ptr(long_src),
                                  _dims(dims), int(gauge_fmt), _stream(stream)), "hisq_gauge_pack")
    return g


def hisq_spinor_pack(dst, src, nsites, spinor_fmt, stream=None):
    _check(load().hisq_spinor_pack(_ptr(dst), _ptr(src), int(nsites), int(spinor_fmt), _stream(stream)),
           "hisq_spinor_pack")


def hisq_spinor_unpack(dst, src, nsites, spinor_fmt, stream=None):
    _check(load().hisq_spinor_unpack(_ptr(dst), _ptr(src), int(nsites), int(spinor_fmt), _stream(stream)),
           "hisq_spinor_unpack")


def hisq_dslash(out, inp, gauge, parity, f, stream=None):
    _check(load().hisq_dslash(_ptr(out), _ptr(inp), ctypes.byref(gauge), int(parity), f, _stream(stream)),
           "hisq_dslash")


def hisq_dslash_xpay(out, inp, gauge, parity, f, a, x, b, stream=None):
    _check(load().hisq_dslash_xpay(_ptr(out), _ptr(inp), ctypes.byref(gauge), int(parity), f, float(a), _ptr(x),
                                   float(b), _stream(stream)), "hisq_dslash_xpay")


def hisq_normal_op(out, inp, tmp, gauge, mass, shift, f, stream=None):
    _check(load().hisq_normal_op(_ptr(out), _ptr(inp), _ptr(tmp), ctypes.byref(gauge), float(mass), float(shift), f,
                                 _stream(stream)), "hisq_normal_op")


def hisq_normal_op_noalloc(out, inp, gauge, mass, shift, f, stream=None):
    _check(load().hisq_normal_op_noalloc(_ptr(out), _ptr(inp), ctypes.byref(gauge), float(mass), float(shift), f,
                                         _stream(stream)), "hisq_normal_op_noalloc")


def hisq_dslash_multi(outs, ins, gauges, parity, f, stream=None):
    """one launch over several lattices: outs[i] = D ins[i] with gauges[i] (hisq_gauge descriptors)"""
    n = len(outs)
    o = (ctypes.c_void_p * n)(*[_ptr(t) for t in outs])
    a = (ctypes.c_void_p * n)(*[_ptr(t) for t in ins])
    gp = (ctypes.POINTER(hisq_gauge) * n)(*[ctypes.pointer(g) for g in gauges])
    _check(load().hisq_dslash_multi(n, o, a, gp, int(parity), f, _stream(stream)), "hisq_dslash_multi")


def hisq_dslash_batched(out, inp, gauge, parity, f, nrhs, stream=None):
    _check(load().hisq_dslash_batched(_ptr(out), _ptr(inp), ctypes.byref(gauge), int(parity), f, int(nrhs),
                                      _stream(stream)), "hisq_dslash_batched")


def hisq_solver_params_default():
    p = hisq_solver_params()
    load().hisq_solver_params_default(ctypes.byref(p))
    return p


def hisq_cg_workspace_bytes(dims, sloppy, params=None):
    return load().hisq_cg_workspace_bytes(_dims(dims), sloppy, ctypes.byref(params) if params else None)


def hisq_cg_solve(x, b, g64, gs, mass, shift, tol, sloppy, params, ws, ws_bytes, stream=None):
    st = hisq_solver_stats()
    status = load().hisq_cg_solve(_ptr(x), _ptr(b), ctypes.byref(g64), ctypes.byref(gs), float(mass), float(shift),
                                  float(tol), sloppy, ctypes.byref(params) if params else None, _ptr(ws),
                                  int(ws_bytes), ctypes.byref(st), _stream(stream))
    return status, st


def hisq_multishift_workspace_bytes(dims, nshift, ms_fmt, ref_fmt, params=None):
    return load().hisq_multishift_workspace_bytes(_dims(dims), int(nshift), ms_fmt, ref_fmt,
                                                  ctypes.byref(params) if params else None)


def hisq_multishift_cg_solve(xs, b, shifts, tol, g64, g_ms, g_ref, mass, ms_fmt, ref_fmt, params, ws, ws_bytes,
                             stream=None):
    n = len(shifts)
    xp = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
    sh = (ctypes.c_double * n)(*[float(s) for s in shifts])
    tl = (ctypes.c_double * n)(*[float(t) for t in tol])
    st = hisq_solver_stats()
    status = load().hisq_multishift_cg_solve(xp, _ptr(b), sh, n, tl, ctypes.byref(g64), ctypes.byref(g_ms),
                                             ctypes.byref(g_ref), float(mass), ms_fmt, ref_fmt,
                                             ctypes.byref(params) if params else None, _ptr(ws), int(ws_bytes),
                                             ctypes.byref(st), _stream(stream))
    return status, st


def hisq_cg_batched_workspace_bytes(dims, nrhs, sloppy, params=None):
    return load().hisq_cg_batched_workspace_bytes(_dims(dims), int(nrhs), sloppy,
                                                  ctypes.byref(params) if params else None)


def hisq_cg_solve_batched(x, b, nrhs, g64, gs, mass, shift, tol, sloppy, params, ws, ws_bytes, stream=None):
    st = hisq_solver_stats()
    status = load().hisq_cg_solve_batched(_ptr(x), _ptr(b), int(nrhs), ctypes.byref(g64), ctypes.byref(gs),
                                          float(mass), float(shift), float(tol), sloppy,
                                          ctypes.byref(params) if params else None, _ptr(ws), int(ws_bytes),
                                          ctypes.byref(st), _stream(stream))
    return status, st


def hisq_last_error():
    return load().hisq_last_error().decode()


def hisq_tune_set(f, dims, rhs_block, nr, rg, stage, block, grid, sweep=0, long_recon=RECON_18):
    f = fmt(f) if isinstance(f, (str, tuple)) else f
    _check(load().hisq_tune_set(f, _dims(dims), int(long_recon), int(rhs_block), int(nr), int(rg), int(stage),
                                int(block), int(grid), int(sweep)), "hisq_tune_set")


def hisq_tune_set_fused(f, dims, rhs_block, nr, rg, stage, block, grid, sweep=0, long_recon=RECON_18):
    f = fmt(f) if isinstance(f, (str, tuple)) else f
    _check(load().hisq_tune_set_fused(f, _dims(dims), int(long_recon), int(rhs_block), int(nr), int(rg),
                                      int(stage), int(block), int(grid), int(sweep)), "hisq_tune_set_fused")


def hisq_tune_clear():
    load().hisq_tune_clear()


def hisq_tune_save(path):
    _check(load().hisq_tune_save(os.fsencode(path)), "hisq_tune_save")


def hisq_tune_load(path):
    """enter the launch shapes of a tune cache file; returns how many"""
    n = ctypes.c_int(0)
    _check(load().hisq_tune_load(os.fsencode(path), ctypes.byref(n)), "hisq_tune_load")
    return n.value


def hisq_tune_report():
    lib = load()
    n = lib.hisq_tune_report(None, 0)
    buf = ctypes.create_string_buffer(int(n))
    lib.hisq_tune_report(buf, n)
    return buf.value.decode()


def hisq_version():
    return load().hisq_version().decode()


# ---------------------------------------------------------------------------
# torch conveniences: allocate outputs, then call one wrapper above
# ---------------------------------------------------------------------------

def _empty_bytes(n, device):
    # 256-byte aligned by the caching allocator; +16 keeps zero-size fields valid
    return torch.empty(max(16, int(n)), dtype=torch.uint8, device=device)


class PackedGauge:
    """Packed fat + long link fields and their hisq_gauge descriptor."""

    def __init__(self, fat, lng, desc, dims, gauge_fmt):
        self.fat, self.lng, self.desc, self.dims, self.fmt = fat, lng, desc, tuple(dims), gauge_fmt


def pack_gauge(fat, lng, dims, gauge_fmt, long_recon=RECON_18, stream=None):
    """canonical complex128 links [4,V,3,3] (device) -> PackedGauge; long_recon=12
    stores the long links as two rows (they must be lambda * phase * SU(3))"""
    fat = torch.view_as_real(fat.contiguous()) if fat.is_complex() else fat.contiguous()
    lng = torch.view_as_real(lng.contiguous()) if lng.is_complex() else lng.contiguous()
    fd = _empty_bytes(hisq_gauge_bytes(dims, gauge_fmt), fat.device)
    ld = _empty_bytes(hisq_gauge_long_bytes(dims, gauge_fmt, long_recon), fat.device)
    g = hisq_gauge_pack_recon(fd, ld, fat, lng, dims, gauge_fmt, long_recon, stream)
    return PackedGauge(fd, ld, g, dims, gauge_fmt)


def pack_spinor(v, spinor_fmt, stream=None):
    """complex128 [n,3] (device) -> packed uint8 field"""
    v = torch.view_as_real(v.contiguous()) if v.is_complex() else v.contiguous()
    n = v.numel() // 6
    out = _empty_bytes(hisq_spinor_bytes(n, spinor_fmt), v.device)
    hisq_spinor_pack(out, v, n, spinor_fmt, stream)
    return out


def unpack_spinor(packed, nsites, spinor_fmt, stream=None):
    """packed field -> complex128 [n,3] (device)"""
    out = torch.empty((int(nsites), 3), dtype=torch.complex128, device=packed.device)
    hisq_spinor_unpack(torch.view_as_real(out), packed, nsites, spinor_fmt, stream)
    return out


def field_info(path):
    """header of a packed-field file as a dict (no device access)"""
    info = hisq_field_header()
    _check(load().hisq_field_info(os.fsencode(path), ctypes.byref(info)), "hisq_field_info")
    return dict(kind=info.kind, fmt=info.fmt, dims=tuple(info.dims), nsites=info.nsites, long_recon=info.long_recon,
                bytes0=info.bytes0, bytes1=info.bytes1)


def save_spinor(path, packed, nsites, spinor_fmt, stream=None):
    _check(load().hisq_spinor_save(os.fsencode(path), _ptr(packed), int(nsites), int(spinor_fmt), _stream(stream)),
           "hisq_spinor_save")


def load_spinor(path, device="cuda", stream=None):
    """-> (packed uint8 field on device, nsites, spinor format)"""
    info = field_info(path)
    if info["kind"] != FIELD_SPINOR:
        raise HisqError(-1, "load_spinor", f"{path} holds a gauge field")
    out = _empty_bytes(info["bytes0"], device)
    _check(load().hisq_spinor_load(os.fsencode(path), _ptr(out), info["nsites"], info["fmt"], _stream(stream)),
           "hisq_spinor_load")
    return out, info["nsites"], info["fmt"]


def save_gauge(path, gauge: PackedGauge, stream=None):
    _check(load().hisq_gauge_save(os.fsencode(path), ctypes.byref(gauge.desc), _stream(stream)), "hisq_gauge_save")


def load_gauge(path, device="cuda", stream=None):
    """-> PackedGauge read from a file written by save_gauge"""
    info = field_info(path)
    if info["kind"] != FIELD_GAUGE:
        raise HisqError(-1, "load_gauge", f"{path} holds a spinor field")
    fd = _empty_bytes(info["bytes0"], device)
    ld = _empty_bytes(info["bytes1"], device)
    g = hisq_gauge()
    _check(load().hisq_gauge_load(os.fsencode(path), ctypes.byref(g), _ptr(fd), fd.numel(), _ptr(ld), ld.numel(),
                                  _stream(stream)), "hisq_gauge_load")
    return PackedGauge(fd, ld, g, tuple(g.dims), g.fmt)


def dslash(packed_in, gauge: PackedGauge, parity, f, stream=None):
    vh = (gauge.dims[0] * gauge.dims[1] * gauge.dims[2] * gauge.dims[3]) // 2
    out = _empty_bytes(hisq_spinor_bytes(vh, f.spinor), packed_in.device)
    hisq_dslash(out, packed_in, gauge.desc, parity, f, stream)
    return out


def _solver_params(**kw):
    p = hisq_solver_params_default()
    names = {f[0] for f in hisq_solver_params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver parameter {k!r}")
        setattr(p, k, v)
    return p


def cg_solve(b, g64: PackedGauge, gs: PackedGauge, mass, shift=0.0, tol=1e-10, sloppy="single", x0=None, **params):
    """mixed-precision CG; b complex128 [Vh,3] on even sites; returns (x, stats dict)"""
    f = fmt(sloppy)
    p = _solver_params(**params)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    nbytes = hisq_cg_workspace_bytes(g64.dims, f, p)
    ws = _empty_bytes(nbytes, b.device)
    status, st = hisq_cg_solve(torch.view_as_real(x), torch.view_as_real(b.contiguous()), g64.desc, gs.desc, mass,
                               shift, tol, f, p, ws, nbytes)
    if status not in (0, -4):
        _check(status, "hisq_cg_solve")
    return x, st.as_dict()


def multishift_cg_solve(b, shifts, tol, g64, g_ms, g_ref, mass, ms_fmt="single", ref_fmt="half", **params):
    """mixed-precision multi-shift CG + refinement; returns ([x_i], stats dict)"""
    fm, fr = fmt(ms_fmt), fmt(ref_fmt)
    p = _solver_params(**params)
    n = len(shifts)
    tol = list(tol) if hasattr(tol, "__len__") else [float(tol)] * n
    xs = [torch.empty_like(b) for _ in range(n)]
    nbytes = hisq_multishift_workspace_bytes(g64.dims, n, fm, fr, p)
    ws = _empty_bytes(nbytes, b.device)
    status, st = hisq_multishift_cg_solve([torch.view_as_real(x) for x in xs], torch.view_as_real(b.contiguous()),
                                          shifts, tol, g64.desc, g_ms.desc, g_ref.desc, mass, fm, fr, p, ws, nbytes)
    if status not in (0, -4):
        _check(status, "hisq_multishift_cg_solve")
    return xs, st.as_dict()


def hisq_bicgstab_workspace_bytes(dims, l, sloppy):
    return load().hisq_bicgstab_workspace_bytes(_dims(dims), int(l), sloppy)


def bicgstab_solve(b, g64, gs, mass, tol=1e-10, l=4, sloppy="single", x0=None, **params):
    """mixed-precision BiCGStab(l) for (2m + D) x = b on the whole lattice;
    b complex128 [V,3] (all sites, lexicographic); returns (x, stats dict)"""
    f = fmt(sloppy)
    p = _solver_params(**params)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    nbytes = hisq_bicgstab_workspace_bytes(g64.dims, l, f)
    if nbytes == 0:
        raise HisqError(-1, "hisq_bicgstab_workspace_bytes", "unsupported arguments")
    ws = _empty_bytes(nbytes, b.device)
    st = hisq_solver_stats()
    status = load().hisq_bicgstab_solve(_ptr(torch.view_as_real(x)), _ptr(torch.view_as_real(b.contiguous())),
                                        ctypes.byref(g64.desc), ctypes.byref(gs.desc), float(mass), float(tol),
                                        int(l), f, ctypes.byref(p), _ptr(ws), nbytes, ctypes.byref(st),
                                        _stream(None))
    if status not in (0, -4):
        _check(status, "hisq_bicgstab_solve")
    return x, st.as_dict()


def cg_solve_batched(b, g64, gs, mass, shift=0.0, tol=1e-10, sloppy="half", x0=None, **params):
    """nrhs independent CG solves sharing each Dslash; b complex128 [nrhs,Vh,3]"""
    f = fmt(sloppy)
    p = _solver_params(**params)
    nrhs = b.shape[0]
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    nbytes = hisq_cg_batched_workspace_bytes(g64.dims, nrhs, f, p)
    ws = _empty_bytes(nbytes, b.device)
    status, st = hisq_cg_solve_batched(torch.view_as_real(x), torch.view_as_real(b.contiguous()), nrhs, g64.desc,
                                       gs.desc, mass, shift, tol, f, p, ws, nbytes)
    if status not in (0, -4):
        _check(status, "hisq_cg_solve_batched")
    return x, st.as_dict()
