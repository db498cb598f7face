// hisq_bicgstab.hip -- mixed-precision BiCGStab(l) (Sec. 6.1; the method of
// Sleijpen and Fokkema) for the whole-lattice HISQ operator M = 2m + D.
//
// The Krylov vectors r_0..r_l, u_0..u_l and the shadow residual live in the
// sloppy triplet's storage format; the solution is accumulated in FP64 at
// every update (Sec. 3.1 item 1).  Reliable updates (Sec. 3, delta): when the
// iterated |r_0| drops by delta below its maximum since the last update (or
// meets the target), r = b - M x is computed with the FP64 operator and
// replaces r_0.  Every scalar (rho, alpha, beta, tau, sigma, gamma, omega) is
// formed on the device by one-thread kernels from fixed-order reductions, and
// every vector kernel reads its coefficients from device memory, so a whole
// cycle (l BiCG steps and the minimal-residual step) is enqueued without the
// host, replayed as a captured hipGraph, and followed by one synchronisation,
// where the host reads |r_0|^2 and decides on a reliable update.
//
// A whole-lattice field is two single-parity fields back to back: the even
// sites, then the odd sites, each in the usual packed layout of Vh sites.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "hisq_internal.h"

namespace hisq {

namespace {

constexpr int BL_MAXK = 8;    // vectors combined or dotted in one pass
constexpr int BL_BLOCK = 256;

constexpr int BL_MAXL = HISQ_MAX_BICGSTAB_L;

struct VecList {
    const char *p[BL_MAXK];
};

// device scalars of one solve (complex values as re, im)
struct BlCtl {
    int stop;     // guard of every kernel of a cycle: 0 while running, -1 after a breakdown
    int broke;    // 1: a BiCG or minimal-residual denominator vanished, 2: non-finite residual
    double one[2];
    double rho0[2], alpha[2], omega[2];
    double beta_neg[2], alpha_neg[2], tau_neg[2];
    double tau[BL_MAXL + 1][BL_MAXL + 1][2];
    double sigma[BL_MAXL + 1];
    double gp[BL_MAXL + 1][2], gm[BL_MAXL + 1][2];
    double cx[BL_MAXK][2], cu[BL_MAXK][2], cr[BL_MAXK][2];   // coefficients of the closing updates
    double rs2;
};
// what the host reads after a cycle
struct BlSummary {
    int stop, broke;
    double rs2;
};

__device__ __forceinline__ size_t bl_tid() { return (size_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ size_t bl_stride() { return (size_t)gridDim.x * blockDim.x; }

// y = a*y + sum_k c_k x_k on the 2*vh sites of whole-lattice fields (half h at
// byte offset h*fb); a and c (K complex values) in device memory;
// partial[block] = |y_new|^2 (stored values) if partial
template <int SF, class R>
__global__ void k_bl_combine(char *y, const double *a, int read_y, VecList xs, const double *c, int K, size_t vh,
                             size_t fb, double *partial, const int *stop) {
    __shared__ double lds[8];
    if (*stop < 0) return;
    const double are = a[0], aim = a[1];
    double acc[1] = {0.0};
    for (size_t i = bl_tid(); i < 2 * vh; i += bl_stride()) {
        const size_t h = i >= vh ? 1 : 0, s = i - h * vh;
        CVec<R> o;
        if (read_y) {
            const CVec<R> v = SpinorIO<SF, R>::load(y + h * fb, vh, s);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                o.re[q] = (R)are * v.re[q] - (R)aim * v.im[q];
                o.im[q] = (R)are * v.im[q] + (R)aim * v.re[q];
            }
        } else {
            cvec_zero(o);
        }
        for (int k = 0; k < K; k++) {
            const CVec<R> v = SpinorIO<SF, R>::load(xs.p[k] + h * fb, vh, s);
            const R cr = (R)c[2 * k], ci = (R)c[2 * k + 1];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                o.re[q] = fma(cr, v.re[q], fma(-ci, v.im[q], o.re[q]));
                o.im[q] = fma(cr, v.im[q], fma(ci, v.re[q], o.im[q]));
            }
        }
        const CVec<R> st = SpinorIO<SF, R>::store(y + h * fb, vh, s, o);
        if (partial) {
#pragma unroll
            for (int q = 0; q < 3; q++) acc[0] += (double)st.re[q] * st.re[q] + (double)st.im[q] * st.im[q];
        }
    }
    if (partial) {
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
    }
}

// <x_k, y> for k < K (re, im) and |y|^2: partial[(block)*(2K+1) + v]
template <int SF, class R>
__global__ void k_bl_dots(VecList xs, int K, const char *y, size_t vh, size_t fb, double *partial, const int *stop) {
    __shared__ double lds[4 * (2 * BL_MAXK + 1)];
    if (*stop < 0) return;
    double acc[2 * BL_MAXK + 1];
#pragma unroll
    for (int v = 0; v < 2 * BL_MAXK + 1; v++) acc[v] = 0.0;
    for (size_t i = bl_tid(); i < 2 * vh; i += bl_stride()) {
        const size_t h = i >= vh ? 1 : 0, s = i - h * vh;
        const CVec<R> w = SpinorIO<SF, R>::load(y + h * fb, vh, s);
#pragma unroll
        for (int q = 0; q < 3; q++) acc[2 * BL_MAXK] += (double)w.re[q] * w.re[q] + (double)w.im[q] * w.im[q];
#pragma unroll
        for (int k = 0; k < BL_MAXK; k++) {
            if (k >= K) break;
            const CVec<R> v = SpinorIO<SF, R>::load(xs.p[k] + h * fb, vh, s);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                acc[2 * k] += (double)v.re[q] * w.re[q] + (double)v.im[q] * w.im[q];
                acc[2 * k + 1] += (double)v.re[q] * w.im[q] - (double)v.im[q] * w.re[q];
            }
        }
    }
    block_sum<2 * BL_MAXK + 1>(acc, lds);
    if (threadIdx.x == 0) {
        for (int k = 0; k < K; k++) {
            partial[(size_t)blockIdx.x * (2 * K + 1) + 2 * k] = acc[2 * k];
            partial[(size_t)blockIdx.x * (2 * K + 1) + 2 * k + 1] = acc[2 * k + 1];
        }
        partial[(size_t)blockIdx.x * (2 * K + 1) + 2 * K] = acc[2 * BL_MAXK];
    }
}

// out[v] = sum over nb blocks of partial[b*nv + v], v < nv (one block, fixed order)
__global__ void k_bl_fin(const double *partial, int nb, int nv, double *out) {
    __shared__ double lds[4];
    for (int v = 0; v < nv; v++) {
        double acc[1] = {0.0};
        for (int b = threadIdx.x; b < nb; b += blockDim.x) acc[0] += partial[(size_t)b * nv + v];
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) out[v] = acc[0];
        __syncthreads();
    }
}

// x64 += sum_k c_k v_k (FP64 solution, sloppy vectors; c in device memory)
template <int SF, class R>
__global__ void k_bl_xupdate(char *x64, VecList vs, const double *c, int K, size_t vh, size_t fb, size_t fb64,
                             const int *stop) {
    if (*stop < 0) return;
    for (size_t i = bl_tid(); i < 2 * vh; i += bl_stride()) {
        const size_t h = i >= vh ? 1 : 0, s = i - h * vh;
        CVec<double> x = SpinorIO<SF_F64, double>::load(x64 + h * fb64, vh, s);
        for (int k = 0; k < K; k++) {
            const CVec<R> v = SpinorIO<SF, R>::load(vs.p[k] + h * fb, vh, s);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                x.re[q] += c[2 * k] * (double)v.re[q] - c[2 * k + 1] * (double)v.im[q];
                x.im[q] += c[2 * k] * (double)v.im[q] + c[2 * k + 1] * (double)v.re[q];
            }
        }
        SpinorIO<SF_F64, double>::store(x64 + h * fb64, vh, s, x);
    }
}

// ---- the scalars of the method, one thread ----
enum BlOp { BL_START, BL_RHO, BL_GAM, BL_TAU, BL_SIGMA, BL_MR, BL_RS2 };

__device__ __forceinline__ void bl_mul(const double *a, const double *b, double *o) {
    const double re = a[0] * b[0] - a[1] * b[1], im = a[0] * b[1] + a[1] * b[0];
    o[0] = re;
    o[1] = im;
}
// a / b with Smith's scaling (no overflow of |b|^2)
__device__ __forceinline__ void bl_div(const double *a, const double *b, double *o) {
    double re, im;
    if (fabs(b[0]) >= fabs(b[1])) {
        const double r = b[1] / b[0], d = b[0] + b[1] * r;
        re = (a[0] + a[1] * r) / d;
        im = (a[1] - a[0] * r) / d;
    } else {
        const double r = b[0] / b[1], d = b[0] * r + b[1];
        re = (a[0] * r + a[1]) / d;
        im = (a[1] * r - a[0]) / d;
    }
    o[0] = re;
    o[1] = im;
}
__device__ __forceinline__ bool bl_zero(const double *a) { return a[0] == 0.0 && a[1] == 0.0; }
__device__ __forceinline__ bool bl_finite(const double *a) { return __builtin_isfinite(a[0]) && __builtin_isfinite(a[1]); }

// res: the finished reduction of the step's dot products (<x, y> as re, im, then |y|^2)
__global__ void k_bl_step(BlCtl *c, const double *res, int op, int i, int j, int l) {
    if (threadIdx.x || c->stop < 0) return;
    auto fail = [&](int code) {
        c->broke = code;
        c->stop = -1;
    };
    switch (op) {
    case BL_START: {   // rho0 = -omega rho0
        double t[2];
        bl_mul(c->omega, c->rho0, t);
        c->rho0[0] = -t[0];
        c->rho0[1] = -t[1];
        break;
    }
    case BL_RHO: {     // rho1 = <r~, r_j>; beta = alpha rho1 / rho0; rho0 = rho1
        const double rho1[2] = {res[0], res[1]};
        if (bl_zero(c->rho0) || !bl_finite(rho1)) {
            fail(1);
            break;
        }
        double t[2], beta[2];
        bl_mul(c->alpha, rho1, t);
        bl_div(t, c->rho0, beta);
        c->rho0[0] = rho1[0];
        c->rho0[1] = rho1[1];
        c->beta_neg[0] = -beta[0];
        c->beta_neg[1] = -beta[1];
        break;
    }
    case BL_GAM: {     // gamma = <r~, u_{j+1}>; alpha = rho0 / gamma
        const double gam[2] = {res[0], res[1]};
        if (bl_zero(gam) || !bl_finite(gam)) {
            fail(1);
            break;
        }
        bl_div(c->rho0, gam, c->alpha);
        c->alpha_neg[0] = -c->alpha[0];
        c->alpha_neg[1] = -c->alpha[1];
        break;
    }
    case BL_TAU: {     // tau_ij = <r_i, r_j> / sigma_i
        c->tau[i][j][0] = res[0] / c->sigma[i];
        c->tau[i][j][1] = res[1] / c->sigma[i];
        c->tau_neg[0] = -c->tau[i][j][0];
        c->tau_neg[1] = -c->tau[i][j][1];
        break;
    }
    case BL_SIGMA: {   // sigma_j = |r_j|^2; gamma'_j = <r_j, r_0> / sigma_j
        const double s2 = res[2];
        c->sigma[j] = s2;
        if (!(s2 > 0.0) || !__builtin_isfinite(s2)) {
            fail(1);
            break;
        }
        c->gp[j][0] = res[0] / s2;
        c->gp[j][1] = -res[1] / s2;
        break;
    }
    case BL_MR: {      // gamma_l, gamma_j (back substitution), gamma''_j; the closing coefficients
        double gpp[BL_MAXL + 1][2];
        c->gm[l][0] = c->gp[l][0];
        c->gm[l][1] = c->gp[l][1];
        c->omega[0] = c->gm[l][0];
        c->omega[1] = c->gm[l][1];
        for (int jj = l - 1; jj >= 1; jj--) {
            double sr = c->gp[jj][0], si = c->gp[jj][1];
            for (int ii = jj + 1; ii <= l; ii++) {
                double t[2];
                bl_mul(c->tau[jj][ii], c->gm[ii], t);
                sr -= t[0];
                si -= t[1];
            }
            c->gm[jj][0] = sr;
            c->gm[jj][1] = si;
        }
        for (int jj = 1; jj < l; jj++) {
            double sr = c->gm[jj + 1][0], si = c->gm[jj + 1][1];
            for (int ii = jj + 1; ii < l; ii++) {
                double t[2];
                bl_mul(c->tau[jj][ii], c->gm[ii + 1], t);
                sr += t[0];
                si += t[1];
            }
            gpp[jj][0] = sr;
            gpp[jj][1] = si;
        }
        // x += gamma_1 r_0 + sum_{j<l} gamma''_j r_j; u_0 -= sum gamma_j u_j; r_0 -= sum gamma'_j r_j
        c->cx[0][0] = c->gm[1][0];
        c->cx[0][1] = c->gm[1][1];
        for (int jj = 1; jj < l; jj++) {
            c->cx[jj][0] = gpp[jj][0];
            c->cx[jj][1] = gpp[jj][1];
        }
        for (int jj = 1; jj <= l; jj++) {
            c->cu[jj - 1][0] = -c->gm[jj][0];
            c->cu[jj - 1][1] = -c->gm[jj][1];
            c->cr[jj - 1][0] = -c->gp[jj][0];
            c->cr[jj - 1][1] = -c->gp[jj][1];
        }
        break;
    }
    case BL_RS2:       // |r_0|^2 after the cycle
        c->rs2 = res[0];
        if (!__builtin_isfinite(res[0])) fail(2);
        break;
    default: break;
    }
}

__global__ void k_bl_summary(const BlCtl *c, BlSummary *o) {
    if (threadIdx.x) return;
    o->stop = c->stop;
    o->broke = c->broke;
    o->rs2 = c->rs2;
}

// canonical lexicographic [V][3] <-> (even field, odd field) in F64 layout
__global__ void k_bl_split(char *dst, const double *src, Geom g, size_t fb64) {
    const size_t V = 2 * (size_t)g.vh;
    for (size_t i = bl_tid(); i < V; i += bl_stride()) {
        size_t r = i;
        const int x = (int)(r % g.X); r /= g.X;
        const int y = (int)(r % g.Y); r /= g.Y;
        const int z = (int)(r % g.Z);
        const int t = (int)(r / g.Z);
        const int par = (x + y + z + t) & 1;
        CVec<double> v;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            v.re[q] = src[6 * i + 2 * q];
            v.im[q] = src[6 * i + 2 * q + 1];
        }
        SpinorIO<SF_F64, double>::store(dst + par * fb64, g.vh, i >> 1, v);
    }
}

__global__ void k_bl_merge(double *dst, const char *src, Geom g, size_t fb64) {
    const size_t V = 2 * (size_t)g.vh;
    for (size_t i = bl_tid(); i < V; i += bl_stride()) {
        size_t r = i;
        const int x = (int)(r % g.X); r /= g.X;
        const int y = (int)(r % g.Y); r /= g.Y;
        const int z = (int)(r % g.Z);
        const int t = (int)(r / g.Z);
        const int par = (x + y + z + t) & 1;
        const CVec<double> v = SpinorIO<SF_F64, double>::load(src + par * fb64, g.vh, i >> 1);
#pragma unroll
        for (int q = 0; q < 3; q++) {
            dst[6 * i + 2 * q] = v.re[q];
            dst[6 * i + 2 * q + 1] = v.im[q];
        }
    }
}

#define HISQ_BL_DISPATCH(sf, compute, CALL)                                                          \
    do {                                                                                             \
        switch ((sf) * 2 + ((compute) == 64)) {                                                      \
        case SF_F64 * 2 + 1: { constexpr int SFc = SF_F64; typedef double Rc; CALL; } break;         \
        case SF_F32 * 2 + 0: { constexpr int SFc = SF_F32; typedef float Rc; CALL; } break;          \
        case SF_HALF16 * 2 + 0: { constexpr int SFc = SF_HALF16; typedef float Rc; CALL; } break;    \
        case SF_INT20 * 2 + 0: { constexpr int SFc = SF_INT20; typedef float Rc; CALL; } break;      \
        case SF_INT30 * 2 + 1: { constexpr int SFc = SF_INT30; typedef double Rc; CALL; } break;     \
        case SF_INT30 * 2 + 0: { constexpr int SFc = SF_INT30; typedef float Rc; CALL; } break;      \
        case SF_INT24 * 2 + 0: { constexpr int SFc = SF_INT24; typedef float Rc; CALL; } break;      \
        default: return set_error(HISQ_EINVAL, "bicgstab: unsupported sloppy triplet");             \
        }                                                                                            \
    } while (0)

struct Bl {
    Geom g;
    size_t vh, fb, fb64;          // bytes of one parity field: sloppy, FP64
    hisq_fmt f;
    const hisq_gauge *g64, *gs;
    double mass;
    hipStream_t st;
    int nbl;                      // grid of the vector kernels
    double *partial;              // >= nbl * (2*BL_MAXK+1) and >= 2 * dslash partials
    double *dres;                 // device results of a reduction (<= 2*BL_MAXK+1)
    double *hres;                 // pinned host copy
    DslashPlan plan_s{}, plan_64{};
    int nb64 = 0;
    long matvecs = 0, f64apps = 0;
    double alg = 0.0;

    BlCtl *ctl = nullptr;         // device scalars
    const int *stopp = nullptr;   // &ctl->stop

    // y = a*y + sum c_k x_k (a, c: device addresses of complex values); with
    // norm, |y|^2 is reduced into dres[0]
    hisq_status combine(char *y, const double *a, bool read_y, const std::vector<const char *> &x, const double *c,
                        bool norm) {
        VecList xl;
        memset(&xl, 0, sizeof(xl));
        const int K = (int)x.size();
        if (K > BL_MAXK) return set_error(HISQ_EINVAL, "bicgstab: too many vectors in one update");
        for (int k = 0; k < K; k++) xl.p[k] = x[k];
        double *pp = norm ? partial : nullptr;
        HISQ_BL_DISPATCH(f.spinor, f.compute,
                         hipLaunchKernelGGL((k_bl_combine<SFc, Rc>), dim3(nbl), dim3(BL_BLOCK), 0, st, y, a,
                                            read_y ? 1 : 0, xl, c, K, vh, fb, pp, stopp));
        HISQ_TRY_HIP(hipGetLastError());
        alg += 2.0 * vh * spinor_site_bytes(f.spinor) * (K + (read_y ? 2 : 1));
        if (norm) {
            hipLaunchKernelGGL(k_bl_fin, dim3(1), dim3(BL_BLOCK), 0, st, partial, nbl, 1, dres);
            HISQ_TRY_HIP(hipGetLastError());
        }
        return HISQ_OK;
    }

    // dres = (<x, y> re, im, |y|^2)
    hisq_status dot(const char *x, const char *y) {
        VecList xl;
        memset(&xl, 0, sizeof(xl));
        xl.p[0] = x;
        HISQ_BL_DISPATCH(f.spinor, f.compute,
                         hipLaunchKernelGGL((k_bl_dots<SFc, Rc>), dim3(nbl), dim3(BL_BLOCK), 0, st, xl, 1, y, vh, fb,
                                            partial, stopp));
        HISQ_TRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_bl_fin, dim3(1), dim3(BL_BLOCK), 0, st, partial, nbl, 3, dres);
        HISQ_TRY_HIP(hipGetLastError());
        alg += 2.0 * vh * spinor_site_bytes(f.spinor) * 2;
        return HISQ_OK;
    }

    hisq_status step(int op, int i = 0, int j = 0, int l = 0) {
        hipLaunchKernelGGL(k_bl_step, dim3(1), dim3(64), 0, st, ctl, dres, op, i, j, l);
        HISQ_TRY_HIP(hipGetLastError());
        return HISQ_OK;
    }

    hisq_status xupdate(char *x64, const std::vector<const char *> &v, const double *c) {
        VecList vl;
        memset(&vl, 0, sizeof(vl));
        const int K = (int)v.size();
        for (int k = 0; k < K; k++) vl.p[k] = v[k];
        HISQ_BL_DISPATCH(f.spinor, f.compute,
                         hipLaunchKernelGGL((k_bl_xupdate<SFc, Rc>), dim3(nbl), dim3(BL_BLOCK), 0, st, x64, vl, c, K,
                                            vh, fb, fb64, stopp));
        HISQ_TRY_HIP(hipGetLastError());
        alg += 2.0 * vh * (96.0 + K * spinor_site_bytes(f.spinor));
        return HISQ_OK;
    }

    DslashArgs dargs(const hisq_gauge *gg, int sf) const {
        DslashArgs a;
        memset(&a, 0, sizeof(a));
        a.b = 1.0;
        a.g = g;
        a.red = RED_NONE;
        a.nrhs = 1;
        a.field_stride = spinor_field_bytes(vh, sf);
        gauge_args(a, gg);
        return a;
    }

    // out = M in = 2m in + D in (sloppy): per output parity p, out_p = D in_q + 2m in_p
    // (skipped after a breakdown in the cycle)
    hisq_status matvec(char *out, const char *in) {
        for (int p = 0; p < 2; p++) {
            DslashArgs a = dargs(gs, f.spinor);
            a.out = out + p * fb;
            a.in = in + (1 - p) * fb;
            a.x = in + p * fb;
            a.a = 2.0 * mass;
            a.parity = p;
            a.guard = Guard{stopp, 0, 0};
            HISQ_TRY_HIP(launch_dslash(a, f, plan_s, st, nullptr));
        }
        matvecs++;
        alg += 2.0 * vh * (dslash_link_bytes(gs) + 3.0 * spinor_site_bytes(f.spinor));
        return HISQ_OK;
    }

    // r64 = b64 - M x64 with the FP64 operator; returns |r64|^2
    hisq_status residual64(char *r64, const char *x64, const char *b64, double *r2) {
        const hisq_fmt f64 = {HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64};
        for (int p = 0; p < 2; p++) {
            DslashArgs a = dargs(g64, SF_F64);
            a.out = r64 + p * fb64;
            a.in = x64 + (1 - p) * fb64;
            a.x = x64 + p * fb64;
            a.y = b64 + p * fb64;
            a.b = -1.0;
            a.a = -2.0 * mass;
            a.c = 1.0;
            a.parity = p;
            a.red = RED_NORM;
            a.partial = partial + (size_t)p * nb64;
            a.pstride = 0;
            HISQ_TRY_HIP(launch_dslash(a, f64, plan_64, st, nullptr));
        }
        f64apps++;
        alg += 2.0 * vh * (dslash_link_bytes(g64) + 4.0 * 48);
        hipLaunchKernelGGL(k_bl_fin, dim3(1), dim3(BL_BLOCK), 0, st, partial, 2 * nb64, 1, dres);
        HISQ_TRY_HIP(hipGetLastError());
        HISQ_TRY_HIP(hipMemcpyAsync(hres, dres, sizeof(double), hipMemcpyDeviceToHost, st));
        HISQ_TRY_HIP(hipStreamSynchronize(st));
        *r2 = hres[0];
        return HISQ_OK;
    }

    hisq_status to_sloppy(char *dst, const char *src64) {
        for (int p = 0; p < 2; p++)
            HISQ_TRY_HIP(launch_spinor_convert(dst + p * fb, f.spinor, src64 + p * fb64, SF_F64, vh, st));
        alg += 2.0 * vh * (48.0 + spinor_site_bytes(f.spinor));
        return HISQ_OK;
    }
};

inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// library-owned stream per device (default priority), ordered after the caller's
// stream with an event; a cycle is captured from it (the caller's stream may be
// the null stream, which cannot be captured)
struct BlDev {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::mutex mu;
};
BlDev g_bldev[64];

struct BlLayout {
    size_t fb, fb64, part_doubles, total;
    size_t off_part, off_dres, off_ctl, off_x64, off_b64, off_r64, off_vec;
    int nvec;
};

BlLayout bl_layout(const Geom &g, int l, const hisq_fmt &f) {
    BlLayout L;
    L.fb = al256(spinor_field_bytes(g.vh, f.spinor));
    L.fb64 = al256(spinor_field_bytes(g.vh, SF_F64));
    const size_t nbl = (size_t)blas_blocks(2 * (size_t)g.vh);
    L.part_doubles = std::max(nbl * (2 * BL_MAXK + 1), 2 * dslash_max_blocks(g));
    L.nvec = 2 * (l + 1) + 1;   // r_0..r_l, u_0..u_l, shadow
    size_t off = 0;
    L.off_part = off;
    off += al256(L.part_doubles * sizeof(double));
    L.off_dres = off;
    off += al256(64 * sizeof(double));
    L.off_ctl = off;
    off += al256(sizeof(BlCtl));
    L.off_x64 = off;
    off += 2 * L.fb64;
    L.off_b64 = off;
    off += 2 * L.fb64;
    L.off_r64 = off;
    off += 2 * L.fb64;
    L.off_vec = off;
    off += (size_t)L.nvec * 2 * L.fb;
    L.total = off;
    return L;
}

}  // namespace

}  // namespace hisq

using namespace hisq;

extern "C" size_t hisq_bicgstab_workspace_bytes(const int dims[4], int l, hisq_fmt sloppy) {
    if (!dims || !dims_ok(dims) || !triplet_ok(sloppy) || l < 1 || l > HISQ_MAX_BICGSTAB_L) return 0;
    return bl_layout(make_geom(dims), l, sloppy).total;
}

extern "C" hisq_status hisq_bicgstab_solve(double *x, const double *b, const hisq_gauge *g64, const hisq_gauge *gs,
                                           double mass, double tol, int l, hisq_fmt sloppy,
                                           const hisq_solver_params *p, void *ws, size_t ws_bytes,
                                           hisq_solver_stats *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    hisq_solver_stats tmp;
    hisq_solver_stats *sto = stats ? stats : &tmp;
    memset(sto, 0, sizeof(*sto));
    sto->status = HISQ_EINVAL;
    if (!x || !b || !g64 || !gs || !ws) return set_error(HISQ_EINVAL, "hisq_bicgstab_solve: null argument");
    if (l < 1 || l > HISQ_MAX_BICGSTAB_L) return set_error(HISQ_EINVAL, "l must be in [1,%d]", HISQ_MAX_BICGSTAB_L);
    if (!(tol > 0.0) || !(mass > 0.0)) return set_error(HISQ_EINVAL, "tol and mass must be > 0");
    if (!triplet_ok(sloppy)) return set_error(HISQ_EINVAL, "unsupported sloppy triplet");
    if (!aligned16(x) || !aligned16(b) || !aligned16(ws)) return set_error(HISQ_EALIGN, "unaligned pointer");
    const int *dims = g64->dims;
    if (!dims_ok(dims)) return set_error(HISQ_EINVAL, "bad lattice dims");
    if (g64->fmt != HISQ_GAUGE_F64 || !g64->fat || !g64->lng) return set_error(HISQ_EINVAL, "g64 must hold FP64 links");
    if (gs->fmt != sloppy.gauge || !gs->fat || !gs->lng) return set_error(HISQ_EINVAL, "gs does not match the sloppy triplet");
    if (!recon_ok(sloppy, gs->long_recon, false) ||
        !recon_ok(hisq_fmt{HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64}, g64->long_recon, false))
        return set_error(HISQ_EINVAL, "eight-parameter long links need FP64 arithmetic on F64 or FIX32 links");
    for (int k = 0; k < 4; k++)
        if (gs->dims[k] != dims[k]) return set_error(HISQ_EINVAL, "gauge dims differ");
    hisq_solver_params q;
    hisq_solver_params_default(&q);
    if (p) q = *p;
    if (q.maxiter <= 0) q.maxiter = 100000;
    const Geom g = make_geom(dims);
    const BlLayout L = bl_layout(g, l, sloppy);
    if (ws_bytes < L.total) return set_error(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.total);

    char *w = (char *)ws;
    Bl B;
    B.g = g;
    B.vh = g.vh;
    B.fb = L.fb;
    B.fb64 = L.fb64;
    B.f = sloppy;
    B.g64 = g64;
    B.gs = gs;
    B.mass = mass;
    int dev = 0;
    HISQ_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(HISQ_EINVAL, "device index %d out of range", dev);
    BlDev &dv = g_bldev[dev];
    std::unique_lock<std::mutex> lk(dv.mu);
    if (!dv.stream) {
        HISQ_TRY_HIP(hipStreamCreateWithFlags(&dv.stream, hipStreamNonBlocking));
        HISQ_TRY_HIP(hipEventCreateWithFlags(&dv.ev, hipEventDisableTiming));
    }
    HISQ_TRY_HIP(hipEventRecord(dv.ev, (hipStream_t)stream));
    HISQ_TRY_HIP(hipStreamWaitEvent(dv.stream, dv.ev, 0));
    B.st = dv.stream;
    B.nbl = blas_blocks(2 * (size_t)g.vh);
    B.partial = (double *)(w + L.off_part);
    B.dres = (double *)(w + L.off_dres);
    B.ctl = (BlCtl *)(w + L.off_ctl);
    B.stopp = &B.ctl->stop;
    HISQ_TRY_HIP(hipHostMalloc((void **)&B.hres, 64 * sizeof(double), hipHostMallocDefault));
    struct Free {
        double *p;
        ~Free() { (void)hipHostFree(p); }
    } free_hres{B.hres};
    char *x64 = w + L.off_x64, *b64 = w + L.off_b64, *r64 = w + L.off_r64;
    std::vector<char *> r(l + 1), u(l + 1);
    for (int i = 0; i <= l; i++) {
        r[i] = w + L.off_vec + (size_t)i * 2 * L.fb;
        u[i] = w + L.off_vec + (size_t)(l + 1 + i) * 2 * L.fb;
    }
    char *rt = w + L.off_vec + (size_t)(2 * l + 2) * 2 * L.fb;

    // launch shapes (autotuned on first use)
    {
        DslashArgs ps = B.dargs(gs, sloppy.spinor);
        ps.out = r[1];
        ps.in = r[0] + L.fb;
        B.plan_s = dslash_plan(sloppy, g, 1, &ps, B.st);
        const hisq_fmt f64 = {HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64};
        DslashArgs p64 = B.dargs(g64, SF_F64);
        p64.out = r64;
        p64.in = x64 + L.fb64;
        B.plan_64 = dslash_plan(f64, g, 1, &p64, B.st);
        B.nb64 = dslash_tile_blocks(g, B.plan_64.tile[0]);
    }

    hipLaunchKernelGGL(k_bl_split, dim3(B.nbl), dim3(BL_BLOCK), 0, B.st, x64, x, g, L.fb64);
    hipLaunchKernelGGL(k_bl_split, dim3(B.nbl), dim3(BL_BLOCK), 0, B.st, b64, b, g, L.fb64);
    HISQ_TRY_HIP(hipGetLastError());
    // |b|^2 in FP64 (both halves' block partials, then one fixed-order sum)
    double b2 = 0.0;
    {
        int nbe = 0, nbo = 0;
        HISQ_TRY_HIP(launch_norm2_f64(b64, g.vh, B.partial, &nbe, B.st));
        HISQ_TRY_HIP(launch_norm2_f64(b64 + L.fb64, g.vh, B.partial + nbe, &nbo, B.st));
        hipLaunchKernelGGL(k_bl_fin, dim3(1), dim3(BL_BLOCK), 0, B.st, B.partial, nbe + nbo, 1, B.dres);
        HISQ_TRY_HIP(hipGetLastError());
        HISQ_TRY_HIP(hipMemcpyAsync(B.hres, B.dres, sizeof(double), hipMemcpyDeviceToHost, B.st));
        HISQ_TRY_HIP(hipStreamSynchronize(B.st));
        b2 = B.hres[0];
    }
    double r2 = 0.0;
    HISQ_TRY(B.residual64(r64, x64, b64, &r2));
    hisq_status status = HISQ_OK;
    long rus = 0;
    const double tol2 = tol * tol * b2;
    const double delta2 = q.delta > 0 ? q.delta * q.delta : 0.0;
    if (b2 == 0.0) {   // x = 0
        HISQ_TRY_HIP(hipMemsetAsync(x, 0, 2 * (size_t)g.vh * 6 * sizeof(double), B.st));
        HISQ_TRY_HIP(hipStreamSynchronize(B.st));
        sto->status = HISQ_OK;
        return HISQ_OK;
    }
    if (r2 > tol2) {
        HISQ_TRY(B.to_sloppy(r[0], r64));
        HISQ_TRY(B.to_sloppy(rt, r64));
        HISQ_TRY_HIP(hipMemsetAsync(u[0], 0, 2 * L.fb, B.st));
        {   // rho0 = 1, alpha = 0, omega = 1
            BlCtl c0;
            memset(&c0, 0, sizeof(c0));
            c0.one[0] = c0.rho0[0] = c0.omega[0] = 1.0;
            HISQ_TRY_HIP(hipMemcpyAsync(B.ctl, &c0, sizeof(c0), hipMemcpyHostToDevice, B.st));
            HISQ_TRY_HIP(hipStreamSynchronize(B.st));
        }
        BlCtl *c = B.ctl;
        // one cycle: l BiCG steps, then the minimal-residual step by modified Gram-Schmidt
        auto enq_cycle = [&]() -> hisq_status {
            HISQ_TRY(B.step(BL_START));
            for (int j = 0; j < l; j++) {
                HISQ_TRY(B.dot(rt, r[j]));
                HISQ_TRY(B.step(BL_RHO));
                for (int i = 0; i <= j; i++) HISQ_TRY(B.combine(u[i], c->beta_neg, true, {r[i]}, c->one, false));
                HISQ_TRY(B.matvec(u[j + 1], u[j]));
                HISQ_TRY(B.dot(rt, u[j + 1]));
                HISQ_TRY(B.step(BL_GAM));
                for (int i = 0; i <= j; i++) HISQ_TRY(B.combine(r[i], c->one, true, {u[i + 1]}, c->alpha_neg, false));
                HISQ_TRY(B.matvec(r[j + 1], r[j]));
                HISQ_TRY(B.xupdate(x64, {u[0]}, c->alpha));
            }
            for (int j = 1; j <= l; j++) {
                for (int i = 1; i < j; i++) {
                    HISQ_TRY(B.dot(r[i], r[j]));
                    HISQ_TRY(B.step(BL_TAU, i, j));
                    HISQ_TRY(B.combine(r[j], c->one, true, {r[i]}, c->tau_neg, false));
                }
                HISQ_TRY(B.dot(r[0], r[j]));                  // <r_0, r_j> and |r_j|^2
                HISQ_TRY(B.step(BL_SIGMA, 0, j));
            }
            HISQ_TRY(B.step(BL_MR, 0, 0, l));
            std::vector<const char *> vx{r[0]}, vr, vu;
            for (int j = 1; j < l; j++) vx.push_back(r[j]);
            for (int j = 1; j <= l; j++) {
                vr.push_back(r[j]);
                vu.push_back(u[j]);
            }
            HISQ_TRY(B.xupdate(x64, vx, &c->cx[0][0]));
            HISQ_TRY(B.combine(u[0], c->one, true, vu, &c->cu[0][0], false));
            HISQ_TRY(B.combine(r[0], c->one, true, vr, &c->cr[0][0], true));
            HISQ_TRY(B.step(BL_RS2));
            hipLaunchKernelGGL(k_bl_summary, dim3(1), dim3(64), 0, B.st, c, (BlSummary *)B.dres);
            HISQ_TRY_HIP(hipGetLastError());
            return HISQ_OK;
        };
        hipGraphExec_t exec = nullptr;
        struct ExecFree {
            hipGraphExec_t *e;
            ~ExecFree() {
                if (*e) (void)hipGraphExecDestroy(*e);
            }
        } exec_free{&exec};
        double cyc_alg = 0.0;
        double rmax2 = r2;
        while (status == HISQ_OK) {
            if (B.matvecs >= q.maxiter) {
                status = set_error(HISQ_ENOCONV, "bicgstab: no convergence in %ld operator applications", B.matvecs);
                break;
            }
            if (q.use_graph) {
                if (!exec) {
                    const double a0 = B.alg;
                    hipGraph_t gr = nullptr;
                    HISQ_TRY_HIP(hipStreamBeginCapture(B.st, hipStreamCaptureModeThreadLocal));
                    hisq_status cs = enq_cycle();
                    hipError_t e = hipStreamEndCapture(B.st, &gr);
                    if (cs != HISQ_OK) {
                        if (gr) (void)hipGraphDestroy(gr);
                        return cs;
                    }
                    HISQ_TRY_HIP(e);
                    e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    HISQ_TRY_HIP(e);
                    cyc_alg = B.alg - a0;
                    B.alg = a0;
                    B.matvecs -= 2 * l;
                }
                HISQ_TRY_HIP(hipGraphLaunch(exec, B.st));
                B.alg += cyc_alg;
                B.matvecs += 2 * l;
            } else {
                HISQ_TRY(enq_cycle());
            }
            HISQ_TRY_HIP(hipMemcpyAsync(B.hres, B.dres, sizeof(BlSummary), hipMemcpyDeviceToHost, B.st));
            HISQ_TRY_HIP(hipStreamSynchronize(B.st));
            BlSummary sum;
            memcpy(&sum, B.hres, sizeof(sum));
            if (sum.broke == 2) {
                status = set_error(HISQ_EBREAKDOWN, "bicgstab: non-finite residual");
                break;
            }
            if (sum.broke) {
                status = set_error(HISQ_EBREAKDOWN, "bicgstab: breakdown after %ld operator applications", B.matvecs);
                break;
            }
            const double rs2 = sum.rs2;
            rmax2 = std::max(rmax2, rs2);
            // ---- reliable update ----
            if (rs2 < delta2 * rmax2 || rs2 <= tol2) {
                HISQ_TRY(B.residual64(r64, x64, b64, &r2));
                rus++;
                if (r2 <= tol2) break;
                HISQ_TRY(B.to_sloppy(r[0], r64));
                rmax2 = r2;
            }
        }
    }
    if (status == HISQ_ENOCONV || status == HISQ_EBREAKDOWN) {
        double rf = 0.0;   // report the true residual of the iterate handed back
        if (B.residual64(r64, x64, b64, &rf) == HISQ_OK) r2 = rf;
    }
    hipLaunchKernelGGL(k_bl_merge, dim3(B.nbl), dim3(BL_BLOCK), 0, B.st, x, x64, g, L.fb64);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(B.st);
    if (e != hipSuccess && status == HISQ_OK) status = set_error(HISQ_EHIP, "bicgstab: %s", hipGetErrorString(e));
    sto->status = status;
    sto->iters = (int)B.matvecs;
    sto->reliable_updates = (int)rus;
    sto->dslash_sloppy = (int)(2 * B.matvecs);
    sto->dslash_f64 = (int)(2 * B.f64apps);
    sto->true_resid = std::sqrt(r2 / b2);
    sto->alg_bytes = B.alg;
    sto->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}
