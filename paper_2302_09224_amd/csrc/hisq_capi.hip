// hisq_capi.hip -- C-ABI entry points of libhisq that are not solvers:
// sizes, packing, the Dslash calls, error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "hisq_internal.h"

namespace hisq {

namespace {
thread_local char g_err[1024] = "";
}

hisq_status set_error(hisq_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

bool dims_ok(const int dims[4]) {
    long v = 1;
    for (int k = 0; k < 4; k++) {
        if (dims[k] < 4 || (dims[k] & 1)) return false;
        v *= dims[k];
    }
    return v / 2 < (1L << 30);  // checkerboard indices and their byte offsets per plane fit the kernels' ints
}

Geom make_geom(const int dims[4]) {
    Geom g;
    g.X = dims[0];
    g.Y = dims[1];
    g.Z = dims[2];
    g.T = dims[3];
    g.X2 = g.X / 2;
    g.vh = g.X2 * g.Y * g.Z * g.T;
    g.sy = g.X2;
    g.sz = g.X2 * g.Y;
    g.st = g.X2 * g.Y * g.Z;
    g.dX2 = make_fastdiv((unsigned)g.X2);
    g.dY = make_fastdiv((unsigned)g.Y);
    g.dZ = make_fastdiv((unsigned)g.Z);
    return g;
}

size_t spinor_field_bytes(size_t nsites, int sf) { return nsites * (size_t)spinor_site_bytes(sf); }

size_t gauge_field_bytes(const int dims[4], int gf) {
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    return 4 * V * (size_t)gauge_matrix_bytes(gf);
}

bool triplet_ok(const hisq_fmt &f) {
    const int k = f.gauge * 100 + f.spinor * 10 + (f.compute == 64 ? 1 : 0);
    if (f.compute != 32 && f.compute != 64) return false;
    switch (k) {
    case GF_F64 * 100 + SF_F64 * 10 + 1:
    case GF_F32 * 100 + SF_F32 * 10 + 0:
    case GF_FIX16 * 100 + SF_HALF16 * 10 + 0:
    case GF_FIX16 * 100 + SF_INT20 * 10 + 0:
    case GF_FIX32 * 100 + SF_INT30 * 10 + 1:
    case GF_FIX32 * 100 + SF_INT30 * 10 + 0:
    case GF_FIX32 * 100 + SF_INT24 * 10 + 0:
    case GF_SX24 * 100 + SF_INT24 * 10 + 0:
    case GF_SX24 * 100 + SF_INT30 * 10 + 1: return true;
    default: return false;
    }
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

void gauge_args(DslashArgs &a, const hisq_gauge *g) {
    a.fat = (const char *)g->fat;
    a.lng = (const char *)g->lng;
    // fixed point: element = q * max / Q; shared-exponent rows carry their own scale
    const double q = g->fmt == HISQ_GAUGE_FIX16 ? 32767.0 : g->fmt == HISQ_GAUGE_FIX32 ? 2147483647.0 : 0.0;
    const bool fixed = q > 0.0;
    a.gfat = fixed ? g->fat_max / q : 1.0;
    a.glong = fixed ? g->long_max / q : 1.0;
    a.long_recon = g->long_recon == HISQ_RECON_12 ? 12 : g->long_recon == HISQ_RECON_8 ? 8 : 18;
    a.lcoef = g->long_coeff;
    // eight-parameter storage holds |c| U: its entries times glong / |c| are those of U
    if (a.long_recon == 8 && g->long_coeff != 0.0) a.glong /= fabs(g->long_coeff);
}

namespace {
std::mutex g_scratch_mu;
LibScratch g_scratch[64];
constexpr size_t SCRATCH_DOUBLES = 16384;
}  // namespace

hisq_status lib_scratch(LibScratch **out) {
    int d = 0;
    HISQ_TRY_HIP(hipGetDevice(&d));
    if (d < 0 || d >= 64) return set_error(HISQ_EINVAL, "device index %d out of range", d);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    LibScratch &s = g_scratch[d];
    if (!s.dev) {
        HISQ_TRY_HIP(hipMalloc((void **)&s.dev, SCRATCH_DOUBLES * sizeof(double)));
        HISQ_TRY_HIP(hipHostMalloc((void **)&s.host, 64 * sizeof(double), hipHostMallocDefault));
        s.ndev = SCRATCH_DOUBLES;
    }
    *out = &s;
    return HISQ_OK;
}

}  // namespace hisq

using namespace hisq;

namespace {

hisq_status check_gauge_arg(const hisq_gauge *g, int want_fmt) {
    if (!g || !g->fat || !g->lng) return set_error(HISQ_EINVAL, "null gauge field");
    if (!dims_ok(g->dims)) return set_error(HISQ_EINVAL, "gauge dims invalid (each even and >= 4)");
    if (g->fmt != want_fmt) return set_error(HISQ_EINVAL, "gauge format %d does not match the triplet (%d)", g->fmt, want_fmt);
    if (!aligned16(g->fat) || !aligned16(g->lng)) return set_error(HISQ_EALIGN, "gauge fields must be 16-byte aligned");
    return HISQ_OK;
}

DslashArgs base_args(const hisq_gauge *g, void *out, const void *in, int parity) {
    DslashArgs a;
    memset(&a, 0, sizeof(a));
    a.out = (char *)out;
    a.in = (const char *)in;
    a.b = 1.0;
    a.g = make_geom(g->dims);
    a.parity = parity;
    a.red = RED_NONE;
    a.nrhs = 1;
    gauge_args(a, g);
    return a;
}

hisq_status dslash_common(void *out, const void *in, const hisq_gauge *g, int parity, hisq_fmt fmt, const char *what) {
    if (!triplet_ok(fmt)) return set_error(HISQ_EINVAL, "%s: unsupported triplet %d/%d/%d", what, fmt.gauge, fmt.spinor, fmt.compute);
    HISQ_TRY(check_gauge_arg(g, fmt.gauge));
    if (!out || !in) return set_error(HISQ_EINVAL, "%s: null spinor", what);
    if (!aligned16(out) || !aligned16(in)) return set_error(HISQ_EALIGN, "%s: spinors must be 16-byte aligned", what);
    if (parity != 0 && parity != 1) return set_error(HISQ_EINVAL, "%s: parity must be 0 or 1", what);
    if (out == in) return set_error(HISQ_EINVAL, "%s: out and in must not alias", what);
    if (!recon_ok(fmt, g->long_recon, false))
        return set_error(HISQ_EINVAL, "%s: eight-parameter long links need FP64 arithmetic on F64 or FIX32 links", what);
    return HISQ_OK;
}

}  // namespace

extern "C" const char *hisq_last_error(void) { return hisq::g_err; }

extern "C" const char *hisq_version(void) { return "libhisq 0.1 (gfx950)"; }

extern "C" size_t hisq_gauge_bytes(const int dims[4], int gauge_fmt) {
    if (!dims || !dims_ok(dims) || gauge_fmt < 0 || gauge_fmt > HISQ_GAUGE_SX24) return 0;
    return gauge_field_bytes(dims, gauge_fmt);
}

extern "C" size_t hisq_spinor_bytes(long nsites, int spinor_fmt) {
    if (nsites < 0 || spinor_fmt < 0 || spinor_fmt > 5) return 0;
    return spinor_field_bytes((size_t)nsites, spinor_fmt);
}

extern "C" size_t hisq_gauge_long_bytes(const int dims[4], int gauge_fmt, int long_recon) {
    if (!dims || !dims_ok(dims) || gauge_fmt < 0 || gauge_fmt > HISQ_GAUGE_SX24) return 0;
    if (long_recon == HISQ_RECON_18) return gauge_field_bytes(dims, gauge_fmt);
    if (long_recon == HISQ_RECON_8) {
        if (gauge_fmt != HISQ_GAUGE_F64 && gauge_fmt != HISQ_GAUGE_FIX32) return 0;
        return (size_t)4 * dims[0] * dims[1] * dims[2] * dims[3] * gauge_matrix_bytes8(gauge_fmt);
    }
    if (long_recon != HISQ_RECON_12) return 0;
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    return 4 * V * (size_t)gauge_matrix_bytes12(gauge_fmt);
}

extern "C" hisq_status hisq_gauge_pack(hisq_gauge *g, void *fat_dst, void *long_dst, const double *fat_src,
                                       const double *long_src, const int dims[4], int gauge_fmt, void *stream) {
    return hisq_gauge_pack_recon(g, fat_dst, long_dst, fat_src, long_src, dims, gauge_fmt, HISQ_RECON_18, stream);
}

extern "C" hisq_status hisq_gauge_pack_recon(hisq_gauge *g, void *fat_dst, void *long_dst, const double *fat_src,
                                             const double *long_src, const int dims[4], int gauge_fmt, int long_recon,
                                             void *stream) {
    if (!g || !fat_dst || !long_dst || !fat_src || !long_src || !dims)
        return set_error(HISQ_EINVAL, "hisq_gauge_pack: null argument");
    if (long_recon != HISQ_RECON_18 && long_recon != HISQ_RECON_12 && long_recon != HISQ_RECON_8)
        return set_error(HISQ_EINVAL, "hisq_gauge_pack: long_recon must be 18, 12 or 8");
    if (long_recon == HISQ_RECON_8 && gauge_fmt != HISQ_GAUGE_F64 && gauge_fmt != HISQ_GAUGE_FIX32)
        return set_error(HISQ_EINVAL, "hisq_gauge_pack: eight-parameter long links are stored in F64 or FIX32 only");
    if (!dims_ok(dims)) return set_error(HISQ_EINVAL, "hisq_gauge_pack: dims must be even and >= 4");
    if (gauge_fmt < 0 || gauge_fmt > HISQ_GAUGE_SX24) return set_error(HISQ_EINVAL, "hisq_gauge_pack: bad gauge format %d", gauge_fmt);
    if (!aligned16(fat_dst) || !aligned16(long_dst) || !aligned16(fat_src) || !aligned16(long_src))
        return set_error(HISQ_EALIGN, "hisq_gauge_pack: pointers must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    LibScratch *ls = nullptr;
    HISQ_TRY(lib_scratch(&ls));
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    const Geom geo = make_geom(dims);
    const size_t nreal = (size_t)4 * 2 * geo.vh * 18;
    double *part = ls->dev;                       // partial maxima
    double *mx = ls->dev + ls->ndev - 2;          // the two global maxima
    int nb = 0;
    HISQ_TRY_HIP(launch_absmax(fat_src, nreal, part, &nb, st));
    HISQ_TRY_HIP(launch_reduce_max(part, nb, mx, st));
    HISQ_TRY_HIP(launch_absmax(long_src, nreal, part, &nb, st));
    HISQ_TRY_HIP(launch_reduce_max(part, nb, mx + 1, st));
    HISQ_TRY_HIP(hipMemcpyAsync(ls->host, mx, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HISQ_TRY_HIP(hipStreamSynchronize(st));
    const double fmax_ = ls->host[0], lmax_ = ls->host[1];
    if (!std::isfinite(fmax_) || !std::isfinite(lmax_))
        return set_error(HISQ_ERANGE, "hisq_gauge_pack: non-finite link element");
    HISQ_TRY_HIP(launch_gauge_pack((char *)fat_dst, fat_src, geo, gauge_fmt, mx, st));
    double long_scale = lmax_, coeff = 1.0;
    if (long_recon == HISQ_RECON_18) {
        HISQ_TRY_HIP(launch_gauge_pack((char *)long_dst, long_src, geo, gauge_fmt, mx + 1, st));
    } else {
        // verify L = lambda * sigma * phase * SU(3) and find lambda, sigma and max |U|
        int nbc = 0;
        HISQ_TRY_HIP(launch_long_check(long_src, geo, part, &nbc, st));
        std::vector<double> ck((size_t)7 * nbc);
        HISQ_TRY_HIP(hipMemcpyAsync(ck.data(), part, ck.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HISQ_TRY_HIP(hipStreamSynchronize(st));
        double mn = 1e300, mxl = 0.0, np = 0.0, nn = 0.0, defect = 0.0, imr = 0.0, umax = 0.0;
        for (int b = 0; b < nbc; b++) {
            const double *c = &ck[(size_t)7 * b];
            mn = std::min(mn, c[0]);
            mxl = std::max(mxl, c[1]);
            np += c[2];
            nn += c[3];
            defect = std::max(defect, c[4]);
            imr = std::max(imr, c[5]);
            umax = std::max(umax, c[6]);
        }
        const double tol = gauge_fmt == HISQ_GAUGE_F64 ? 1e-13
                           : (gauge_fmt == HISQ_GAUGE_F32 || gauge_fmt == HISQ_GAUGE_SX24) ? 1e-7
                           : gauge_fmt == HISQ_GAUGE_FIX16 ? 1e-5 : 1e-9;
        const double lam = 0.5 * (mn + mxl);
        if (!(lam > 0.0) || (mxl - mn) > tol * lam || defect > tol || imr > tol || (np > 0 && nn > 0))
            return set_error(HISQ_EINVAL,
                             "hisq_gauge_pack_recon: long links are not lambda*phase*SU(3) within %g "
                             "(lambda in [%g,%g], unitarity defect %g, |Im det|/|det| %g, sign counts %g/%g)",
                             tol, mn, mxl, defect, imr, np, nn);
        coeff = np > 0 ? lam : -lam;
        if (long_recon == HISQ_RECON_8) {
            HISQ_TRY_HIP(launch_gauge_pack8((char *)long_dst, long_src, geo, gauge_fmt, np > 0 ? 1.0 : -1.0, lmax_, st));
        } else {
            long_scale = umax;
            HISQ_TRY_HIP(launch_gauge_pack12((char *)long_dst, long_src, geo, gauge_fmt, coeff, umax, st));
        }
    }
    HISQ_TRY_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < 4; k++) g->dims[k] = dims[k];
    g->fmt = gauge_fmt;
    g->fat = fat_dst;
    g->lng = long_dst;
    g->fat_max = fmax_;
    g->long_max = long_scale;
    g->long_recon = long_recon;
    g->long_coeff = coeff;
    return HISQ_OK;
}

extern "C" hisq_status hisq_spinor_pack(void *dst, const double *src, long nsites, int spinor_fmt, void *stream) {
    if (!dst || !src) return set_error(HISQ_EINVAL, "hisq_spinor_pack: null pointer");
    if (nsites < 0 || spinor_fmt < 0 || spinor_fmt > 5) return set_error(HISQ_EINVAL, "hisq_spinor_pack: bad size or format");
    if (!aligned16(dst) || !aligned16(src)) return set_error(HISQ_EALIGN, "hisq_spinor_pack: unaligned pointer");
    HISQ_TRY_HIP(launch_spinor_pack((char *)dst, src, (size_t)nsites, spinor_fmt, (hipStream_t)stream));
    return HISQ_OK;
}

extern "C" hisq_status hisq_spinor_unpack(double *dst, const void *src, long nsites, int spinor_fmt, void *stream) {
    if (!dst || !src) return set_error(HISQ_EINVAL, "hisq_spinor_unpack: null pointer");
    if (nsites < 0 || spinor_fmt < 0 || spinor_fmt > 5) return set_error(HISQ_EINVAL, "hisq_spinor_unpack: bad size or format");
    if (!aligned16(dst) || !aligned16(src)) return set_error(HISQ_EALIGN, "hisq_spinor_unpack: unaligned pointer");
    HISQ_TRY_HIP(launch_spinor_unpack(dst, (const char *)src, (size_t)nsites, spinor_fmt, (hipStream_t)stream));
    return HISQ_OK;
}

extern "C" hisq_status hisq_dslash(void *out, const void *in, const hisq_gauge *g, int parity, hisq_fmt fmt,
                                   void *stream) {
    HISQ_TRY(dslash_common(out, in, g, parity, fmt, "hisq_dslash"));
    DslashArgs a = base_args(g, out, in, parity);
    const DslashPlan plan = dslash_plan(fmt, a.g, 1, &a, (hipStream_t)stream);
    HISQ_TRY_HIP(launch_dslash(a, fmt, plan, (hipStream_t)stream, nullptr));
    return HISQ_OK;
}

extern "C" hisq_status hisq_dslash_multi(int n, void *const *out, const void *const *in, const hisq_gauge *const *g,
                                         int parity, hisq_fmt fmt, void *stream) {
    if (n < 1 || n > HISQ_MAX_LATTICES) return set_error(HISQ_EINVAL, "hisq_dslash_multi: n must be in [1,%d]", HISQ_MAX_LATTICES);
    if (!out || !in || !g) return set_error(HISQ_EINVAL, "hisq_dslash_multi: null argument");
    MultiArgs m;
    memset(&m, 0, sizeof(m));
    m.n = n;
    int lr = -1;
    long long blocks = 0;
    for (int i = 0; i < n; i++) {
        if (!g[i]) return set_error(HISQ_EINVAL, "hisq_dslash_multi: null gauge %d", i);
        HISQ_TRY(dslash_common(out[i], in[i], g[i], parity, fmt, "hisq_dslash_multi"));
        if (g[i]->long_recon == HISQ_RECON_8)
            return set_error(HISQ_EINVAL, "hisq_dslash_multi: eight-parameter long links have no multi-lattice form");
        const int r = g[i]->long_recon == HISQ_RECON_12 ? 12 : 18;
        if (lr >= 0 && r != lr) return set_error(HISQ_EINVAL, "hisq_dslash_multi: lattices differ in long-link storage");
        lr = r;
        for (int k = 0; k < i; k++)
            if (out[i] == out[k] || out[i] == in[k] || in[i] == out[k])
                return set_error(HISQ_EINVAL, "hisq_dslash_multi: lattice %d aliases lattice %d", i, k);
        m.a[i] = base_args(g[i], out[i], in[i], parity);
        m.boff[i] = (int)blocks;
        blocks += (m.a[i].g.vh + MULTI_BLOCK - 1) / MULTI_BLOCK;
        if (blocks > 0x7fffffff) return set_error(HISQ_EINVAL, "hisq_dslash_multi: too many sites");
    }
    m.boff[n] = (int)blocks;
    HISQ_TRY_HIP(launch_dslash_multi(m, fmt, lr, (hipStream_t)stream));
    return HISQ_OK;
}

extern "C" hisq_status hisq_dslash_xpay(void *out, const void *in, const hisq_gauge *g, int parity, hisq_fmt fmt,
                                        double a, const void *x, double b, void *stream) {
    HISQ_TRY(dslash_common(out, in, g, parity, fmt, "hisq_dslash_xpay"));
    if (x && !aligned16(x)) return set_error(HISQ_EALIGN, "hisq_dslash_xpay: x unaligned");
    if (x == in) return set_error(HISQ_EINVAL, "hisq_dslash_xpay: x has the other parity's sites and cannot be `in`");
    DslashArgs d = base_args(g, out, in, parity);
    d.b = b;
    d.x = (const char *)x;
    d.a = a;
    const DslashPlan plan = dslash_plan(fmt, d.g, 1, &d, (hipStream_t)stream);
    HISQ_TRY_HIP(launch_dslash(d, fmt, plan, (hipStream_t)stream, nullptr));
    return HISQ_OK;
}

extern "C" hisq_status hisq_normal_op(void *out, const void *in, void *tmp, const hisq_gauge *g, double mass,
                                      double shift, hisq_fmt fmt, void *stream) {
    HISQ_TRY(dslash_common(tmp, in, g, 1, fmt, "hisq_normal_op"));
    if (!out || !aligned16(out)) return set_error(HISQ_EALIGN, "hisq_normal_op: out null or unaligned");
    if (out == in || out == tmp) return set_error(HISQ_EINVAL, "hisq_normal_op: out must not alias in or tmp");
    DslashArgs d1 = base_args(g, tmp, in, 1);
    const DslashPlan plan = dslash_plan(fmt, d1.g, 1, &d1, (hipStream_t)stream);
    HISQ_TRY_HIP(launch_dslash(d1, fmt, plan, (hipStream_t)stream, nullptr));
    DslashArgs d2 = base_args(g, out, tmp, 0);
    d2.b = -1.0;
    d2.x = (const char *)in;
    d2.a = 4.0 * mass * mass + shift;
    HISQ_TRY_HIP(launch_dslash(d2, fmt, plan, (hipStream_t)stream, nullptr));
    return HISQ_OK;
}

extern "C" hisq_status hisq_dslash_batched(void *out, const void *in, const hisq_gauge *g, int parity, hisq_fmt fmt,
                                           int nrhs, void *stream) {
    HISQ_TRY(dslash_common(out, in, g, parity, fmt, "hisq_dslash_batched"));
    if (nrhs < 1 || nrhs > 16) return set_error(HISQ_EINVAL, "hisq_dslash_batched: nrhs must be in [1,16]");
    if (!has_batched_form(fmt))
        return set_error(HISQ_EINVAL, "hisq_dslash_batched: triplet FIX32/INT30/32 has no batched kernel");
    if (!recon_ok(fmt, g->long_recon, true))
        return set_error(HISQ_EINVAL, "hisq_dslash_batched: eight-parameter long links have no batched form");
    DslashArgs a = base_args(g, out, in, parity);
    a.nrhs = nrhs;
    a.field_stride = spinor_field_bytes((size_t)a.g.vh, fmt.spinor);
    const DslashPlan plan = dslash_plan(fmt, a.g, nrhs, &a, (hipStream_t)stream);
    HISQ_TRY_HIP(launch_dslash(a, fmt, plan, (hipStream_t)stream, nullptr));
    return HISQ_OK;
}

// ---------------------------------------------------------------------------
// The normal operator without allocation.  Its odd-parity intermediate lives
// in `scratch`, a file-scope device array that every device holds from the
// loading of this code object until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: its device address on the current
// device is looked up once per device and kept in g_scratch_dev.
// ---------------------------------------------------------------------------

static __device__ __align__(256) char scratch[HISQ_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_dev_mu;
void *g_scratch_dev[64];   // address of `scratch` on device d, nullptr until looked up

hisq_status noalloc_scratch(void **ptr) {
    int d = 0;
    HISQ_TRY_HIP(hipGetDevice(&d));
    if (d < 0 || d >= 64) return set_error(HISQ_EINVAL, "device index %d out of range", d);
    std::lock_guard<std::mutex> lk(g_scratch_dev_mu);
    if (!g_scratch_dev[d]) {
        void *p = nullptr;
        HISQ_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(HISQ_EHIP, "hisq_normal_op_noalloc: no device address for the scratch array");
        g_scratch_dev[d] = p;
    }
    *ptr = g_scratch_dev[d];
    return HISQ_OK;
}

}  // namespace

extern "C" hisq_status hisq_normal_op_noalloc(void *out, const void *in, const hisq_gauge *g, double mass,
                                              double shift, hisq_fmt fmt, void *stream) {
    HISQ_TRY(dslash_common(out, in, g, 0, fmt, "hisq_normal_op_noalloc"));
    const Geom geo = make_geom(g->dims);
    const size_t need = spinor_field_bytes((size_t)geo.vh, fmt.spinor);
    if (need > HISQ_NOALLOC_SCRATCH_BYTES)
        return set_error(HISQ_EINVAL,
                         "hisq_normal_op_noalloc: the odd-parity intermediate needs %zu bytes, more than the "
                         "%zu-byte scratch array (use hisq_normal_op with a tmp field)",
                         need, (size_t)HISQ_NOALLOC_SCRATCH_BYTES);
    void *tmp = nullptr;
    HISQ_TRY(noalloc_scratch(&tmp));
    DslashArgs d1 = base_args(g, tmp, in, 1);
    const DslashPlan plan = dslash_plan_lookup(fmt, geo, 1, d1.long_recon);
    HISQ_TRY_HIP(launch_dslash(d1, fmt, plan, (hipStream_t)stream, nullptr));
    DslashArgs d2 = base_args(g, out, tmp, 0);
    d2.b = -1.0;
    d2.x = (const char *)in;
    d2.a = 4.0 * mass * mass + shift;
    HISQ_TRY_HIP(launch_dslash(d2, fmt, plan, (hipStream_t)stream, nullptr));
    return HISQ_OK;
}
