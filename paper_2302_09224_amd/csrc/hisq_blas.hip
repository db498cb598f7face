// hisq_blas.hip -- streaming kernels of libhisq: storage packing/unpacking,
// gauge-field packing, and the fused vector updates of the solvers.
//
// All of these are HBM-bound sweeps over one or a few fields; each is written
// as a grid-stride loop with a capped grid so that its reductions produce a
// fixed, small number of per-block partials (summed later in a fixed order:
// the reductions are bitwise reproducible).  Reductions accumulate in FP64
// and are taken on the values as stored (after packing), which is what the
// next iteration will read.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "hisq_internal.h"

namespace hisq {

int blas_blocks(size_t n) {
    size_t nb = (n + BLAS_BLOCK - 1) / BLAS_BLOCK;
    if (nb > BLAS_MAX_BLOCKS) nb = BLAS_MAX_BLOCKS;
    if (nb < 1) nb = 1;
    return (int)nb;
}

namespace {

// natural arithmetic precision of a spinor format
template <int SF> struct Natural { typedef float T; };
template <> struct Natural<SF_F64> { typedef double T; };
template <> struct Natural<SF_INT30> { typedef double T; };

__device__ __forceinline__ size_t gtid() { return (size_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ size_t gstride() { return (size_t)gridDim.x * blockDim.x; }

// canonical complex128 [n][3] (device) <-> register vector
template <class R> __device__ __forceinline__ CVec<R> load_canon(const double *src, size_t s) {
    const f64x2 *p = reinterpret_cast<const f64x2 *>(src + 6 * s);
    CVec<R> v;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        f64x2 w = p[c];
        v.re[c] = (R)w.x;
        v.im[c] = (R)w.y;
    }
    return v;
}

template <class R> __device__ __forceinline__ void store_canon(double *dst, size_t s, const CVec<R> &v) {
    f64x2 *p = reinterpret_cast<f64x2 *>(dst + 6 * s);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        f64x2 w;
        w.x = (double)v.re[c];
        w.y = (double)v.im[c];
        p[c] = w;
    }
}

template <int SF> __global__ void k_spinor_pack(char *dst, const double *src, size_t n) {
    typedef typename Natural<SF>::T T;
    for (size_t s = gtid(); s < n; s += gstride()) SpinorIO<SF, T>::store(dst, n, s, load_canon<T>(src, s));
}

template <int SF> __global__ void k_spinor_unpack(double *dst, const char *src, size_t n) {
    typedef typename Natural<SF>::T T;
    for (size_t s = gtid(); s < n; s += gstride()) store_canon<T>(dst, s, SpinorIO<SF, T>::load(src, n, s));
}

template <int SFD, int SFS> __global__ void k_spinor_convert(char *dst, const char *src, size_t n) {
    for (size_t s = gtid(); s < n; s += gstride())
        SpinorIO<SFD, double>::store(dst, n, s, SpinorIO<SFS, double>::load(src, n, s));
}

__global__ void k_absmax(const double *src, size_t n, double *partial) {
    __shared__ double lds[16];
    double m = 0.0;
    int bad = 0;
    for (size_t i = gtid(); i < n; i += gstride()) {
        double v = src[i];
        bad |= !__builtin_isfinite(v);
        m = fmax(m, fabs(v));
    }
    if (bad) m = __builtin_inf();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = fmax(m, lds[w]);
        partial[blockIdx.x] = m;
    }
}

__global__ void k_reduce_max(const double *partial, int n, double *out) {
    __shared__ double lds[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, partial[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = fmax(m, lds[w]);
        *out = m;
    }
}

// row r of a link as a 24-bit shared-exponent record: words 0-3 in 16-byte
// plane r, word 4 in 4-byte plane r after the nrow 16-byte planes
__device__ __forceinline__ void sx24_store_row(char *base, size_t vh, size_t s, int r, int nrow, const double *v) {
    CVec<double> c;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        c.re[k] = v[2 * k];
        c.im[k] = v[2 * k + 1];
    }
    unsigned w[SxFmt<24>::W];
    SxCodec<24, double>::encode(c, w);
    u32x4 a;
    a.x = w[0]; a.y = w[1]; a.z = w[2]; a.w = w[3];
    st<u32x4>(base + r * 16 * vh + 16 * s, a);
    st<unsigned>(base + nrow * 16 * vh + r * 4 * vh + 4 * s, w[4]);
}

// canonical FP64 links [4][V][3][3] -> packed sub-fields (mu, parity)
template <int GF> __global__ void k_gauge_pack(char *dst, const double *src, Geom g, const double *absmax) {
    const size_t V = 2 * (size_t)g.vh;
    const size_t vh = g.vh;
    const size_t sub = (size_t)gauge_matrix_bytes(GF) * vh;
    const double m = *absmax;
    const double c = GF == GF_FIX16 ? (m > 0.0 ? 32767.0 / m : 0.0) : (m > 0.0 ? 2147483647.0 / m : 0.0);
    for (size_t idx = gtid(); idx < 4 * V; idx += gstride()) {
        const int mu = (int)(idx / V);
        const size_t site = idx - (size_t)mu * V;
        size_t r = site;
        const int x = (int)(r % g.X); r /= g.X;
        const int y = (int)(r % g.Y); r /= g.Y;
        const int z = (int)(r % g.Z);
        const int t = (int)(r / g.Z);
        const int par = (x + y + z + t) & 1;
        const size_t s = site >> 1;
        char *base = dst + (size_t)(2 * mu + par) * sub;
        const double *u = src + idx * 18;
        if (GF == GF_F64) {
#pragma unroll
            for (int k = 0; k < 9; k++) {
                f64x2 w;
                w.x = u[2 * k];
                w.y = u[2 * k + 1];
                st<f64x2>(base + k * 16 * vh + 16 * s, w);
            }
        } else if (GF == GF_F32) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                f32x4 w;
                w.x = (float)u[4 * k]; w.y = (float)u[4 * k + 1]; w.z = (float)u[4 * k + 2]; w.w = (float)u[4 * k + 3];
                st<f32x4>(base + k * 16 * vh + 16 * s, w);
            }
            f32x2 t2;
            t2.x = (float)u[16];
            t2.y = (float)u[17];
            st<f32x2>(base + 64 * vh + 8 * s, t2);
        } else if (GF == GF_FIX16) {
            unsigned q[18];
#pragma unroll
            for (int k = 0; k < 18; k++) q[k] = (unsigned)(int)__builtin_rint(u[k] * c) & 0xffffu;
#pragma unroll
            for (int k = 0; k < 2; k++) {
                u32x4 w;
                w.x = q[8 * k + 0] | (q[8 * k + 1] << 16);
                w.y = q[8 * k + 2] | (q[8 * k + 3] << 16);
                w.z = q[8 * k + 4] | (q[8 * k + 5] << 16);
                w.w = q[8 * k + 6] | (q[8 * k + 7] << 16);
                st<u32x4>(base + k * 16 * vh + 16 * s, w);
            }
            st<unsigned>(base + 32 * vh + 4 * s, q[16] | (q[17] << 16));
        } else if (GF == GF_SX24) {
#pragma unroll
            for (int r = 0; r < 3; r++) sx24_store_row(base, vh, s, r, 3, u + 6 * r);
        } else {  // GF_FIX32
            unsigned q[18];
#pragma unroll
            for (int k = 0; k < 18; k++) q[k] = (unsigned)(int)__builtin_rint(u[k] * c);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                u32x4 w;
                w.x = q[4 * k]; w.y = q[4 * k + 1]; w.z = q[4 * k + 2]; w.w = q[4 * k + 3];
                st<u32x4>(base + k * 16 * vh + 16 * s, w);
            }
            u32x2 t2;
            t2.x = q[16];
            t2.y = q[17];
            st<u32x2>(base + 64 * vh + 8 * s, t2);
        }
    }
}

// staggered phase of a three-hop link starting at (x,y,z,t) along mu: eta_mu(x)
// times -1 when the hop crosses the time boundary (the convention of the inputs)
__device__ __forceinline__ double link_phase3(int mu, int x, int y, int z, int t, int T) {
    const int e = mu == 0 ? 0 : mu == 1 ? x : mu == 2 ? x + y : x + y + z;
    const int b = (mu == 3 && t >= T - 3) ? 1 : 0;
    return ((e + b) & 1) ? -1.0 : 1.0;
}

// Long links for two-row storage: every L_mu(x) must be lambda * sigma * phase * U
// with U in SU(3), lambda > 0 and sigma = +-1 global.  Per block:
// [min lambda_x, max lambda_x, #sigma_x>0, #sigma_x<0, max unitarity defect,
//  max |Im det| / |det|, max |component| / lambda_x], lambda_x = |det L|^(1/3).
__global__ void k_long_check(const double *src, Geom g, double *partial) {
    __shared__ double lds[7][8];
    const size_t V = 2 * (size_t)g.vh;
    double mn = 1e300, mx = 0.0, np = 0.0, nn = 0.0, defect = 0.0, imr = 0.0, cmax = 0.0;
    for (size_t idx = gtid(); idx < 4 * V; idx += gstride()) {
        const int mu = (int)(idx / V);
        size_t r = idx - (size_t)mu * V;
        const int x = (int)(r % g.X); r /= g.X;
        const int y = (int)(r % g.Y); r /= g.Y;
        const int z = (int)(r % g.Z);
        const int t = (int)(r / g.Z);
        const double *u = src + idx * 18;
        double ar[9], ai[9];
        for (int k = 0; k < 9; k++) {
            ar[k] = u[2 * k];
            ai[k] = u[2 * k + 1];
        }
        // det by cofactors along row 0
        double dr = 0.0, di = 0.0;
        for (int k = 0; k < 3; k++) {
            const int i = (k + 1) % 3, j = (k + 2) % 3;
            const double cr = ar[3 + i] * ar[6 + j] - ai[3 + i] * ai[6 + j] - (ar[3 + j] * ar[6 + i] - ai[3 + j] * ai[6 + i]);
            const double ci = ar[3 + i] * ai[6 + j] + ai[3 + i] * ar[6 + j] - (ar[3 + j] * ai[6 + i] + ai[3 + j] * ar[6 + i]);
            dr += ar[k] * cr - ai[k] * ci;
            di += ar[k] * ci + ai[k] * cr;
        }
        const double ad = sqrt(dr * dr + di * di);
        const double lam = cbrt(ad);
        mn = fmin(mn, lam);
        mx = fmax(mx, lam);
        imr = fmax(imr, ad > 0 ? fabs(di) / ad : 1.0);
        const double sg = (dr >= 0 ? 1.0 : -1.0) * link_phase3(mu, x, y, z, t, g.T);
        if (sg > 0) np += 1.0; else nn += 1.0;
        const double inv = lam > 0 ? 1.0 / lam : 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double sr = 0.0, si = 0.0;  // (U^dag U)_ab
                for (int k = 0; k < 3; k++) {
                    sr += ar[3 * k + a] * ar[3 * k + b] + ai[3 * k + a] * ai[3 * k + b];
                    si += ar[3 * k + a] * ai[3 * k + b] - ai[3 * k + a] * ar[3 * k + b];
                }
                sr = sr * inv * inv - (a == b ? 1.0 : 0.0);
                si = si * inv * inv;
                defect = fmax(defect, fmax(fabs(sr), fabs(si)));
            }
        for (int k = 0; k < 9; k++) cmax = fmax(cmax, fmax(fabs(ar[k]), fabs(ai[k])) * inv);
    }
    double v[7] = {mn, mx, np, nn, defect, imr, cmax};
    for (int k = 0; k < 7; k++) {
        double w = v[k];
        for (int o = 32; o > 0; o >>= 1) {
            const double q = __shfl_xor(w, o, 64);
            w = (k == 0) ? fmin(w, q) : (k == 2 || k == 3) ? w + q : fmax(w, q);
        }
        if ((threadIdx.x & 63) == 0) lds[k][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 7; k++) {
            double w = lds[k][0];
            for (int j = 1; j < (int)(blockDim.x >> 6); j++)
                w = (k == 0) ? fmin(w, lds[k][j]) : (k == 2 || k == 3) ? w + lds[k][j] : fmax(w, lds[k][j]);
            partial[7 * blockIdx.x + k] = w;
        }
    }
}

// two rows of U = L / (lambda * sigma * phase) into the 12-real sub-fields;
// fixed-point formats scale by umax (the global max |component| of U)
template <int GF> __global__ void k_gauge_pack12(char *dst, const double *src, Geom g, double coef, double umax) {
    const size_t V = 2 * (size_t)g.vh;
    const size_t vh = g.vh;
    const size_t sub = (size_t)gauge_matrix_bytes12(GF) * vh;
    const double qs = GF == GF_FIX16 ? 32767.0 / umax : GF == GF_FIX32 ? 2147483647.0 / umax : 1.0;
    for (size_t idx = gtid(); idx < 4 * V; idx += gstride()) {
        const int mu = (int)(idx / V);
        const size_t site = idx - (size_t)mu * V;
        size_t r = site;
        const int x = (int)(r % g.X); r /= g.X;
        const int y = (int)(r % g.Y); r /= g.Y;
        const int z = (int)(r % g.Z);
        const int t = (int)(r / g.Z);
        const int par = (x + y + z + t) & 1;
        const size_t s = site >> 1;
        char *base = dst + (size_t)(2 * mu + par) * sub;
        const double *u = src + idx * 18;
        const double inv = 1.0 / (coef * link_phase3(mu, x, y, z, t, g.T));
        double w[12];
        for (int k = 0; k < 12; k++) w[k] = u[k] * inv;
        if (GF == GF_F64) {
            for (int k = 0; k < 6; k++) {
                f64x2 v;
                v.x = w[2 * k];
                v.y = w[2 * k + 1];
                st<f64x2>(base + k * 16 * vh + 16 * s, v);
            }
        } else if (GF == GF_F32) {
            for (int k = 0; k < 3; k++) {
                f32x4 v;
                v.x = (float)w[4 * k]; v.y = (float)w[4 * k + 1]; v.z = (float)w[4 * k + 2]; v.w = (float)w[4 * k + 3];
                st<f32x4>(base + k * 16 * vh + 16 * s, v);
            }
        } else if (GF == GF_FIX16) {
            unsigned q[12];
            for (int k = 0; k < 12; k++) q[k] = (unsigned)(int)__builtin_rint(w[k] * qs) & 0xffffu;
            u32x4 a;
            a.x = q[0] | (q[1] << 16); a.y = q[2] | (q[3] << 16); a.z = q[4] | (q[5] << 16); a.w = q[6] | (q[7] << 16);
            u32x2 b;
            b.x = q[8] | (q[9] << 16);
            b.y = q[10] | (q[11] << 16);
            st<u32x4>(base + 16 * s, a);
            st<u32x2>(base + 16 * vh + 8 * s, b);
        } else if (GF == GF_SX24) {
            for (int r = 0; r < 2; r++) sx24_store_row(base, vh, s, r, 2, w + 6 * r);
        } else {
            unsigned q[12];
            for (int k = 0; k < 12; k++) q[k] = (unsigned)(int)__builtin_rint(w[k] * qs);
            for (int k = 0; k < 3; k++) {
                u32x4 a;
                a.x = q[4 * k]; a.y = q[4 * k + 1]; a.z = q[4 * k + 2]; a.w = q[4 * k + 3];
                st<u32x4>(base + k * 16 * vh + 16 * s, a);
            }
        }
    }
}

// tan(arg(x + iy)/4), 0 at the origin, by the operation sequence the
// eight-parameter storage specifies (every operation correctly rounded; the
// one product-sum is an explicit fma, the rest leaves the compiler nothing to
// contract), so that the stored bits do not depend on the compiler
__device__ __noinline__ double phase_param(double x, double y) {
    const double r = sqrt(fma(x, x, y * y));
    if (r == 0.0) return 0.0;
    const double c = x / r, sn = y / r;
    double ch, sh;
    if (c >= 0.0) {
        ch = sqrt((1.0 + c) * 0.5);
        sh = sn / (2.0 * ch);
    } else {
        const double sa = sqrt((1.0 - c) * 0.5);
        sh = copysign(sa, sn);
        ch = fabs(sn) / (2.0 * sa);
    }
    return sh / (1.0 + ch);
}

// eight parameters of W = L * phase * sign (= |lambda| U): Re/Im of W01, W02,
// W10, then phase_param of W00 and of W20.  F64: four 16-byte planes; FIX32:
// two planes, the entries scaled by lmax, the phase parameters by 1.
template <int GF> __global__ void k_gauge_pack8(char *dst, const double *src, Geom g, double sign, double lmax) {
    const size_t V = 2 * (size_t)g.vh;
    const size_t vh = g.vh;
    const size_t sub = (size_t)gauge_matrix_bytes8(GF) * vh;
    const double qs = 2147483647.0 / lmax;
    for (size_t idx = gtid(); idx < 4 * V; idx += gstride()) {
        const int mu = (int)(idx / V);
        const size_t site = idx - (size_t)mu * V;
        size_t r = site;
        const int x = (int)(r % g.X); r /= g.X;
        const int y = (int)(r % g.Y); r /= g.Y;
        const int z = (int)(r % g.Z);
        const int t = (int)(r / g.Z);
        const int par = (x + y + z + t) & 1;
        const size_t s = site >> 1;
        char *base = dst + (size_t)(2 * mu + par) * sub;
        const double *u = src + idx * 18;
        const double ph = link_phase3(mu, x, y, z, t, g.T) * sign;    // +-1: the products are exact
        double p[8];
        for (int k = 0; k < 6; k++) p[k] = u[2 + k] * ph;             // W01, W02, W10 (reals 2..7)
        p[6] = phase_param(u[0] * ph, u[1] * ph);                     // W00
        p[7] = phase_param(u[12] * ph, u[13] * ph);                   // W20
        if (GF == GF_F64) {
            for (int k = 0; k < 4; k++) {
                f64x2 v;
                v.x = p[2 * k];
                v.y = p[2 * k + 1];
                st<f64x2>(base + k * 16 * vh + 16 * s, v);
            }
        } else {
            unsigned q[8];
            for (int k = 0; k < 8; k++) q[k] = (unsigned)(int)__builtin_rint(p[k] * (k < 6 ? qs : 2147483647.0));
            for (int k = 0; k < 2; k++) {
                u32x4 a;
                a.x = q[4 * k]; a.y = q[4 * k + 1]; a.z = q[4 * k + 2]; a.w = q[4 * k + 3];
                st<u32x4>(base + k * 16 * vh + 16 * s, a);
            }
        }
    }
}

__global__ void k_norm2_f64(const char *v, size_t n, double *partial) {
    __shared__ double lds[16];
    double acc = 0.0;
    for (size_t s = gtid(); s < n; s += gstride()) {
        CVec<double> a = SpinorIO<SF_F64, double>::load(v, n, s);
#pragma unroll
        for (int c = 0; c < 3; c++) acc += a.re[c] * a.re[c] + a.im[c] * a.im[c];
    }
    double w[1] = {acc};
    block_sum<1>(w, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = w[0];
}

// ---------------------------------------------------------------------------
// CG vector updates
// ---------------------------------------------------------------------------

template <int SF, class R>
__global__ void k_cg_axpy(char *r, const char *ap, const double *alpha, size_t n, double *partial, Guard gd,
                          char *r_copy) {
    __shared__ double lds[32];
    if (!gd.pass()) return;
    const R a = (R)(*alpha);
    double acc[2] = {0.0, 0.0};
    for (size_t s = gtid(); s < n; s += gstride()) {
        CVec<R> ro = SpinorIO<SF, R>::load(r, n, s);
        CVec<R> av = SpinorIO<SF, R>::load(ap, n, s);
        CVec<R> rn;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            rn.re[c] = fma(-a, av.re[c], ro.re[c]);
            rn.im[c] = fma(-a, av.im[c], ro.im[c]);
        }
        CVec<R> o = SpinorIO<SF, R>::store(r, n, s, rn);
        if (r_copy) (void)SpinorIO<SF, R>::store(r_copy, n, s, rn);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc[0] += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
            acc[1] += (double)o.re[c] * (double)ro.re[c] + (double)o.im[c] * (double)ro.im[c];
        }
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = acc[0];
        partial[2 * blockIdx.x + 1] = acc[1];
    }
}

template <int SF, class R>
__global__ void k_cg_pupdate(char *pd, const char *r, const char *ps, const SolverCtrl *ctrl, size_t n, double *ppart,
                             Guard gd) {
    __shared__ double lds[8];
    if (!gd.pass()) return;
    const R ar = (R)ctrl->pa_re, ai = (R)ctrl->pa_im, b = (R)ctrl->pb;
    double acc[1] = {0.0};
    for (size_t s = gtid(); s < n; s += gstride()) {
        CVec<R> rv = SpinorIO<SF, R>::load(r, n, s);
        CVec<R> pv = SpinorIO<SF, R>::load(ps, n, s);
        CVec<R> o;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            o.re[c] = fma(ar, rv.re[c], fma(-ai, rv.im[c], b * pv.re[c]));
            o.im[c] = fma(ar, rv.im[c], fma(ai, rv.re[c], b * pv.im[c]));
        }
        const CVec<R> st = SpinorIO<SF, R>::store(pd, n, s, o);
        if (ppart) {
#pragma unroll
            for (int c = 0; c < 3; c++) acc[0] += (double)st.re[c] * st.re[c] + (double)st.im[c] * st.im[c];
        }
    }
    if (ppart) {
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) ppart[blockIdx.x] = acc[0];
    }
}

// Buffered-vector loops load a group of vectors before using the first, so that
// a lane keeps that many loads in flight instead of one.  A short last group
// repeats its last vector (the same addresses, a cache hit) with coefficient 0,
// so that every load is used unconditionally and none is deferred to its use;
// the sums keep their order (fma(0, v, x) = x), so results do not depend on
// the grouping.
// Four vectors per group; two for FP64 vectors (twice the registers each).
template <int SF> constexpr int load_group() { return SF == SF_F64 ? 2 : 4; }

template <int SF, class R>
__global__ void k_flush_x(char *x64, SpinorList p, int count, const double *alpha_buf, size_t n, Guard gd) {
    if (!gd.pass()) return;
    constexpr int LOAD_GROUP = load_group<SF>();
    for (size_t s = gtid(); s < n; s += gstride()) {
        CVec<double> x = SpinorIO<SF_F64, double>::load(x64, n, s);
        for (int i0 = 0; i0 < count; i0 += LOAD_GROUP) {
            CVec<R> pv[LOAD_GROUP];
            double a[LOAD_GROUP];
#pragma unroll
            for (int k = 0; k < LOAD_GROUP; k++) {
                const int i = min(i0 + k, count - 1);
                pv[k] = SpinorIO<SF, R>::load(p.p[i], n, s);
                a[k] = i0 + k < count ? alpha_buf[i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < LOAD_GROUP; k++) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    x.re[c] = fma(a[k], (double)pv[k].re[c], x.re[c]);
                    x.im[c] = fma(a[k], (double)pv[k].im[c], x.im[c]);
                }
            }
        }
        SpinorIO<SF_F64, double>::store(x64, n, s, x);
    }
}

template <int SF, class R>
__global__ void k_ru_convert(char *rs, const char *r64, const char *p, const char *ap, const double *alpha, size_t n,
                             double *partial, Guard gd) {
    __shared__ double lds[64];
    if (!gd.pass()) return;
    const R a = alpha ? (R)(*alpha) : R(0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t s = gtid(); s < n; s += gstride()) {
        CVec<double> rt = SpinorIO<SF_F64, double>::load(r64, n, s);
        CVec<R> rold;
        if (ap) rold = SpinorIO<SF, R>::load(rs, n, s);
        CVec<R> rn;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            rn.re[c] = (R)rt.re[c];
            rn.im[c] = (R)rt.im[c];
        }
        CVec<R> o = SpinorIO<SF, R>::store(rs, n, s, rn);
#pragma unroll
        for (int c = 0; c < 3; c++) acc[0] += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
        if (p) {
            CVec<R> pv = SpinorIO<SF, R>::load(p, n, s);
            // <r, p> = sum conj(r) p
#pragma unroll
            for (int c = 0; c < 3; c++) {
                acc[1] += (double)o.re[c] * (double)pv.re[c] + (double)o.im[c] * (double)pv.im[c];
                acc[2] += (double)o.re[c] * (double)pv.im[c] - (double)o.im[c] * (double)pv.re[c];
            }
        }
        if (ap) {
            // the previous iterated residual r_k = r_{k+1}^iter + alpha A p_k
            CVec<R> av = SpinorIO<SF, R>::load(ap, n, s);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double pr = (double)rold.re[c] + (double)a * (double)av.re[c];
                const double pi = (double)rold.im[c] + (double)a * (double)av.im[c];
                acc[3] += (double)o.re[c] * pr + (double)o.im[c] * pi;
            }
        }
    }
    block_sum<4>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) partial[4 * blockIdx.x + k] = acc[k];
    }
}

// The shifted systems of the multi-shift CG (Sec. 3.2) over a block of
// `count` iterations, every shift in one launch.  The shifted gradient
// vectors obey p_i <- zeta_i r + beta_i p_i with the base residual r of the
// same iteration, and the shifted solutions x_i += alpha_i p_i; the solutions
// are updated once per block (buffered, Sec. 3.1 item 1).  So a shift's
// gradient vector is stored only at the block's start: the block's base
// residuals r_{k+1} are kept in a ring (rr.p[q], q < count), the finalize
// kernel records the shifts' scalars of every iteration (slot q), and this
// kernel replays the block's updates in registers, loading each residual once
// per group of G shifts.  A shift that stops in slot q takes its x update of
// that slot and no more; the shifts still active store their gradient vector
// again for the next block.
constexpr int RING_LOADS = 4;
template <int SF, class R, int G>
__global__ void __launch_bounds__(BLAS_BLOCK) k_shift_replay(SpinorList x64, SpinorList p, SpinorList rr,
                                                             const SolverCtrl *ctrl, int nshift, size_t n, int count,
                                                             Guard gd) {
    // the block's scalars staged in LDS: their reads then wait on the LDS
    // counter, not behind the residual loads in flight
    __shared__ double s_a[HISQ_MAX_GRAD_BUFFER][HISQ_MAX_SHIFTS], s_z[HISQ_MAX_GRAD_BUFFER][HISQ_MAX_SHIFTS],
        s_b[HISQ_MAX_GRAD_BUFFER][HISQ_MAX_SHIFTS];
    __shared__ unsigned s_e[HISQ_MAX_GRAD_BUFFER], s_r[HISQ_MAX_GRAD_BUFFER];
    if (!gd.pass()) return;
    for (int t = threadIdx.x; t < count * HISQ_MAX_SHIFTS; t += blockDim.x) {
        const int q = t / HISQ_MAX_SHIFTS, i = t % HISQ_MAX_SHIFTS;
        s_a[q][i] = ctrl->ai_buf[q][i];
        s_z[q][i] = ctrl->zb_buf[q][i];
        s_b[q][i] = ctrl->bb_buf[q][i];
    }
    for (int t = threadIdx.x; t < count; t += blockDim.x) {
        s_e[t] = (unsigned)ctrl->eb_buf[t];
        s_r[t] = (unsigned)ctrl->rmb_buf[t];
    }
    __syncthreads();
    const unsigned all = nshift >= 32 ? ~0u : (1u << nshift) - 1u;
    const unsigned upd = s_e[0] & ~1u & all;   // shifts can only leave during a block
    const unsigned keep = s_e[count - 1] & ~s_r[count - 1];
    for (size_t s = gtid(); s < n; s += gstride()) {
        for (unsigned m = upd; m;) {
            int ids[G];
#pragma unroll
            for (int k = 0; k < G; k++) {
                ids[k] = m ? __builtin_ctz(m) : -1;
                m &= m - 1u;
            }
            CVec<R> pv[G];
            CVec<double> xv[G];
#pragma unroll
            for (int k = 0; k < G; k++) {
                const int i = ids[k] >= 0 ? ids[k] : ids[0];   // a short group repeats its first shift, unused
                pv[k] = SpinorIO<SF, R>::load(p.p[i], n, s);
                xv[k] = SpinorIO<SF_F64, double>::load(x64.p[i], n, s);
            }
            // iteration q of the block, in order
            auto step = [&](int q, const CVec<R> &rv) {
                const unsigned eq = s_e[q], sq = s_r[q];
#pragma unroll
                for (int k = 0; k < G; k++) {
                    const int i = ids[k];
                    if (i < 0 || !((eq >> i) & 1u)) continue;
                    const double a = s_a[q][i];
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        xv[k].re[c] = fma(a, (double)pv[k].re[c], xv[k].re[c]);
                        xv[k].im[c] = fma(a, (double)pv[k].im[c], xv[k].im[c]);
                    }
                    if ((sq >> i) & 1u) continue;
                    const R zi = (R)s_z[q][i], bi = (R)s_b[q][i];
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        pv[k].re[c] = fma(zi, rv.re[c], bi * pv[k].re[c]);
                        pv[k].im[c] = fma(zi, rv.im[c], bi * pv[k].im[c]);
                    }
                }
            };
            // the residuals are loaded RING_LOADS slots at a time, all in flight
            // before the first of them is used; the updates keep slot order
            int q = 0;
            for (; q + RING_LOADS <= count; q += RING_LOADS) {
                CVec<R> rv[RING_LOADS];
#pragma unroll
                for (int u = 0; u < RING_LOADS; u++) rv[u] = SpinorIO<SF, R>::load(rr.p[q + u], n, s);
#pragma unroll
                for (int u = 0; u < RING_LOADS; u++) step(q + u, rv[u]);
            }
            for (; q < count; q++) step(q, SpinorIO<SF, R>::load(rr.p[q], n, s));
#pragma unroll
            for (int k = 0; k < G; k++) {
                const int i = ids[k];
                if (i < 0) continue;
                SpinorIO<SF_F64, double>::store(x64.p[i], n, s, xv[k]);
                if ((keep >> i) & 1u) (void)SpinorIO<SF, R>::store(p.p[i], n, s, pv[k]);
            }
        }
    }
}
// shifts per group: the gradient vectors and FP64 solutions of four shifts in registers
constexpr int REPLAY_GROUP = 4;

// ---------------------------------------------------------------------------
// batched (nrhs independent systems) vector updates
// ---------------------------------------------------------------------------

template <int SF, class R>
__global__ void k_bcg_axpy(char *r, const char *ap, const SolverCtrl *ctrl, size_t n, size_t fs, int nrhs,
                           double *partial, Guard gd) {
    __shared__ double lds[32];
    if (!gd.pass()) return;
    for (int j = 0; j < nrhs; j++) {
        double acc[2] = {0.0, 0.0};
        if (ctrl->bactive[j]) {
            const R a = (R)ctrl->balpha[j];
            char *rj = r + j * fs;
            const char *aj = ap + j * fs;
            for (size_t s = gtid(); s < n; s += gstride()) {
                CVec<R> ro = SpinorIO<SF, R>::load(rj, n, s);
                CVec<R> av = SpinorIO<SF, R>::load(aj, n, s);
                CVec<R> rn;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    rn.re[c] = fma(-a, av.re[c], ro.re[c]);
                    rn.im[c] = fma(-a, av.im[c], ro.im[c]);
                }
                CVec<R> o = SpinorIO<SF, R>::store(rj, n, s, rn);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[0] += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
                    acc[1] += (double)o.re[c] * (double)ro.re[c] + (double)o.im[c] * (double)ro.im[c];
                }
            }
        }
        block_sum<2>(acc, lds);
        if (threadIdx.x == 0) {
            partial[((size_t)blockIdx.x * nrhs + j) * 2] = acc[0];
            partial[((size_t)blockIdx.x * nrhs + j) * 2 + 1] = acc[1];
        }
        __syncthreads();
    }
}

template <int SF, class R>
__global__ void k_bcg_pupdate(char *pd, const char *r, const char *ps, const SolverCtrl *ctrl, size_t n, size_t fs,
                              int nrhs, Guard gd) {
    if (!gd.pass()) return;
    for (int j = 0; j < nrhs; j++) {
        if (!ctrl->bactive[j]) continue;
        const R ar = (R)ctrl->bpa_re[j], ai = (R)ctrl->bpa_im[j], b = (R)ctrl->bpb[j];
        for (size_t s = gtid(); s < n; s += gstride()) {
            CVec<R> rv = SpinorIO<SF, R>::load(r + j * fs, n, s);
            CVec<R> pv = SpinorIO<SF, R>::load(ps + j * fs, n, s);
            CVec<R> o;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                o.re[c] = fma(ar, rv.re[c], fma(-ai, rv.im[c], b * pv.re[c]));
                o.im[c] = fma(ar, rv.im[c], fma(ai, rv.re[c], b * pv.im[c]));
            }
            SpinorIO<SF, R>::store(pd + j * fs, n, s, o);
        }
    }
}

template <int SF, class R>
__global__ void k_bflush_x(char *x64, size_t fs64, SpinorList p, int count, const SolverCtrl *ctrl, size_t n, size_t fs,
                           int nrhs, Guard gd) {
    if (!gd.pass()) return;
    for (int j = 0; j < nrhs; j++) {
        // a stopped system's buffered gradients were flushed before it stopped
        if (!ctrl->bactive[j]) continue;
        char *xj = x64 + j * fs64;
        for (size_t s = gtid(); s < n; s += gstride()) {
            CVec<double> x = SpinorIO<SF_F64, double>::load(xj, n, s);
            for (int i = 0; i < count; i++) {
                const double a = ctrl->balpha_buf[i][j];
                if (a == 0.0) continue;
                CVec<R> pv = SpinorIO<SF, R>::load(p.p[i] + j * fs, n, s);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    x.re[c] = fma(a, (double)pv.re[c], x.re[c]);
                    x.im[c] = fma(a, (double)pv.im[c], x.im[c]);
                }
            }
            SpinorIO<SF_F64, double>::store(xj, n, s, x);
        }
    }
}

template <int SF, class R>
__global__ void k_bru_convert(char *rs, const char *r64, size_t fs64, const char *p, const char *ap,
                              const SolverCtrl *ctrl, size_t n, size_t fs, int nrhs, double *partial, Guard gd) {
    __shared__ double lds[64];
    if (!gd.pass()) return;
    for (int j = 0; j < nrhs; j++) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const R a = (R)ctrl->balpha[j];
        char *rsj = rs + j * fs;
        // only the systems taking part in the reliable update replace their residual
        const bool part = ctrl->bru[j] && ctrl->bactive[j];
        for (size_t s = gtid(); part && s < n; s += gstride()) {
            CVec<double> rt = SpinorIO<SF_F64, double>::load(r64 + j * fs64, n, s);
            CVec<R> rold;
            if (ap) rold = SpinorIO<SF, R>::load(rsj, n, s);
            CVec<R> rn;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                rn.re[c] = (R)rt.re[c];
                rn.im[c] = (R)rt.im[c];
            }
            CVec<R> o = SpinorIO<SF, R>::store(rsj, n, s, rn);
#pragma unroll
            for (int c = 0; c < 3; c++) acc[0] += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
            if (p) {
                CVec<R> pv = SpinorIO<SF, R>::load(p + j * fs, n, s);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[1] += (double)o.re[c] * (double)pv.re[c] + (double)o.im[c] * (double)pv.im[c];
                    acc[2] += (double)o.re[c] * (double)pv.im[c] - (double)o.im[c] * (double)pv.re[c];
                }
            }
            if (ap) {
                CVec<R> av = SpinorIO<SF, R>::load(ap + j * fs, n, s);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const double pr = (double)rold.re[c] + (double)a * (double)av.re[c];
                    const double pi = (double)rold.im[c] + (double)a * (double)av.im[c];
                    acc[3] += (double)o.re[c] * pr + (double)o.im[c] * pi;
                }
            }
        }
        block_sum<4>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; k++) partial[((size_t)blockIdx.x * nrhs + j) * 4 + k] = acc[k];
        }
        __syncthreads();
    }
}

// dispatch on the sloppy triplet's spinor format and compute precision
#define HISQ_DISPATCH_SC(sf, compute, CALL)                                           \
    do {                                                                              \
        switch ((sf) * 2 + ((compute) == 64)) {                                       \
        case SF_F64 * 2 + 1: { constexpr int SFc = SF_F64; typedef double Rc; CALL; } break;   \
        case SF_F32 * 2 + 0: { constexpr int SFc = SF_F32; typedef float Rc; CALL; } break;    \
        case SF_HALF16 * 2 + 0: { constexpr int SFc = SF_HALF16; typedef float Rc; CALL; } break; \
        case SF_INT20 * 2 + 0: { constexpr int SFc = SF_INT20; typedef float Rc; CALL; } break; \
        case SF_INT30 * 2 + 1: { constexpr int SFc = SF_INT30; typedef double Rc; CALL; } break; \
        case SF_INT30 * 2 + 0: { constexpr int SFc = SF_INT30; typedef float Rc; CALL; } break; \
        case SF_INT24 * 2 + 0: { constexpr int SFc = SF_INT24; typedef float Rc; CALL; } break; \
        default: return hipErrorInvalidValue;                                         \
        }                                                                             \
    } while (0)

#define HISQ_DISPATCH_SF(sf, CALL)                                                    \
    do {                                                                              \
        switch (sf) {                                                                 \
        case SF_F64: { constexpr int SFc = SF_F64; CALL; } break;                    \
        case SF_F32: { constexpr int SFc = SF_F32; CALL; } break;                    \
        case SF_HALF16: { constexpr int SFc = SF_HALF16; CALL; } break;              \
        case SF_INT20: { constexpr int SFc = SF_INT20; CALL; } break;                \
        case SF_INT30: { constexpr int SFc = SF_INT30; CALL; } break;                \
        case SF_INT24: { constexpr int SFc = SF_INT24; CALL; } break;                \
        default: return hipErrorInvalidValue;                                         \
        }                                                                             \
    } while (0)

}  // namespace

hipError_t launch_spinor_pack(char *dst, const double *src, size_t n, int sf, hipStream_t st) {
    if (n == 0) return hipSuccess;
    HISQ_DISPATCH_SF(sf, hipLaunchKernelGGL((k_spinor_pack<SFc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, dst, src, n));
    return hipGetLastError();
}

hipError_t launch_spinor_unpack(double *dst, const char *src, size_t n, int sf, hipStream_t st) {
    if (n == 0) return hipSuccess;
    HISQ_DISPATCH_SF(sf, hipLaunchKernelGGL((k_spinor_unpack<SFc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, dst, src, n));
    return hipGetLastError();
}

namespace {
template <int SFD>
hipError_t convert_from(char *dst, const char *src, int sf_src, size_t n, hipStream_t st) {
    HISQ_DISPATCH_SF(sf_src, hipLaunchKernelGGL((k_spinor_convert<SFD, SFc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, dst, src, n));
    return hipGetLastError();
}
}  // namespace

hipError_t launch_spinor_convert(char *dst, int sf_dst, const char *src, int sf_src, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    switch (sf_dst) {
    case SF_F64: return convert_from<SF_F64>(dst, src, sf_src, n, st);
    case SF_F32: return convert_from<SF_F32>(dst, src, sf_src, n, st);
    case SF_HALF16: return convert_from<SF_HALF16>(dst, src, sf_src, n, st);
    case SF_INT20: return convert_from<SF_INT20>(dst, src, sf_src, n, st);
    case SF_INT30: return convert_from<SF_INT30>(dst, src, sf_src, n, st);
    case SF_INT24: return convert_from<SF_INT24>(dst, src, sf_src, n, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_absmax(const double *src, size_t n, double *partial, int *nblocks, hipStream_t st) {
    const int nb = blas_blocks(n);
    *nblocks = nb;
    hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(BLAS_BLOCK), 0, st, src, n, partial);
    return hipGetLastError();
}

hipError_t launch_reduce_max(const double *partial, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(1024), 0, st, partial, n, out);
    return hipGetLastError();
}

hipError_t launch_gauge_pack(char *dst, const double *src, const Geom &g, int gf, const double *absmax, hipStream_t st) {
    const size_t n = 8 * (size_t)g.vh;
    const int nb = blas_blocks(n);
    switch (gf) {
    case GF_F64: hipLaunchKernelGGL((k_gauge_pack<GF_F64>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, absmax); break;
    case GF_F32: hipLaunchKernelGGL((k_gauge_pack<GF_F32>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, absmax); break;
    case GF_FIX16: hipLaunchKernelGGL((k_gauge_pack<GF_FIX16>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, absmax); break;
    case GF_FIX32: hipLaunchKernelGGL((k_gauge_pack<GF_FIX32>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, absmax); break;
    case GF_SX24: hipLaunchKernelGGL((k_gauge_pack<GF_SX24>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, absmax); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_long_check(const double *src, const Geom &g, double *partial, int *nblocks, hipStream_t st) {
    const int nb = blas_blocks(8 * (size_t)g.vh);
    *nblocks = nb;
    hipLaunchKernelGGL(k_long_check, dim3(nb), dim3(BLAS_BLOCK), 0, st, src, g, partial);
    return hipGetLastError();
}

hipError_t launch_gauge_pack8(char *dst, const double *src, const Geom &g, int gf, double sign, double lmax,
                              hipStream_t st) {
    const int nb = blas_blocks((size_t)8 * g.vh);
    switch (gf) {
    case GF_F64: hipLaunchKernelGGL((k_gauge_pack8<GF_F64>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, sign, lmax); break;
    case GF_FIX32: hipLaunchKernelGGL((k_gauge_pack8<GF_FIX32>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, sign, lmax); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gauge_pack12(char *dst, const double *src, const Geom &g, int gf, double coef, double umax,
                               hipStream_t st) {
    const int nb = blas_blocks(8 * (size_t)g.vh);
    switch (gf) {
    case GF_F64: hipLaunchKernelGGL((k_gauge_pack12<GF_F64>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, coef, umax); break;
    case GF_F32: hipLaunchKernelGGL((k_gauge_pack12<GF_F32>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, coef, umax); break;
    case GF_FIX16: hipLaunchKernelGGL((k_gauge_pack12<GF_FIX16>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, coef, umax); break;
    case GF_FIX32: hipLaunchKernelGGL((k_gauge_pack12<GF_FIX32>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, coef, umax); break;
    case GF_SX24: hipLaunchKernelGGL((k_gauge_pack12<GF_SX24>), dim3(nb), dim3(BLAS_BLOCK), 0, st, dst, src, g, coef, umax); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_norm2_f64(const char *v, size_t n, double *partial, int *nblocks, hipStream_t st) {
    const int nb = blas_blocks(n);
    *nblocks = nb;
    hipLaunchKernelGGL(k_norm2_f64, dim3(nb), dim3(BLAS_BLOCK), 0, st, v, n, partial);
    return hipGetLastError();
}

hipError_t launch_cg_axpy(char *r, const char *ap, const double *alpha, size_t n, int sf, int compute, double *partial,
                          Guard gd, hipStream_t st, char *r_copy) {
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_cg_axpy<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, r, ap, alpha, n, partial, gd, r_copy));
    return hipGetLastError();
}

hipError_t launch_cg_pupdate(char *p_dst, const char *r, const char *p_src, const SolverCtrl *ctrl, double *ppart,
                             size_t n, int sf,
                             int compute, Guard gd, hipStream_t st) {
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_cg_pupdate<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, p_dst, r, p_src, ctrl, n, ppart, gd));
    return hipGetLastError();
}

hipError_t launch_flush_x(char *x64, const SpinorList &p, int count, const double *alpha_buf, size_t n, int sf,
                          int compute, Guard gd, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int nb = flush_x_grid(n, sf, compute);
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_flush_x<SFc, Rc>), dim3(nb), dim3(BLAS_BLOCK), 0, st, x64, p, count, alpha_buf, n, gd));
    return hipGetLastError();
}

hipError_t launch_ru_convert(char *r_s, const char *r64, const char *p, const char *ap, const double *alpha, size_t n,
                             int sf, int compute, double *partial, Guard gd, hipStream_t st) {
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_ru_convert<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, r_s, r64, p, ap, alpha, n, partial, gd));
    return hipGetLastError();
}

namespace {
// blas_blocks(n) capped at the blocks of kernel `fn` the device holds at once
// (queried once per device and kernel)
int resident_grid(const void *fn, size_t n) {
    const int nb = blas_blocks(n);
    int dev = 0;
    if (!fn || hipGetDevice(&dev) != hipSuccess) return nb;
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> resident;
    std::lock_guard<std::mutex> lock(mu);
    auto it = resident.find(std::make_pair(dev, fn));
    if (it == resident.end()) {
        int per_cu = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLAS_BLOCK, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
            ncu < 1) {
            (void)hipGetLastError();
            return nb;
        }
        it = resident.emplace(std::make_pair(dev, fn), per_cu * ncu).first;
    }
    return std::min(nb, it->second);
}
hipError_t shift_replay_kernel(int sf, int compute, const void **fn) {
    HISQ_DISPATCH_SC(sf, compute, *fn = reinterpret_cast<const void *>(&k_shift_replay<SFc, Rc, REPLAY_GROUP>));
    return hipSuccess;
}
hipError_t flush_x_kernel(int sf, int compute, const void **fn) {
    HISQ_DISPATCH_SC(sf, compute, *fn = reinterpret_cast<const void *>(&k_flush_x<SFc, Rc>));
    return hipSuccess;
}
}  // namespace

int shift_replay_grid(size_t n, int sf, int compute) {
    const void *fn = nullptr;
    return resident_grid(shift_replay_kernel(sf, compute, &fn) == hipSuccess ? fn : nullptr, n);
}

int flush_x_grid(size_t n, int sf, int compute) {
    const void *fn = nullptr;
    return resident_grid(flush_x_kernel(sf, compute, &fn) == hipSuccess ? fn : nullptr, n);
}

hipError_t launch_shift_replay(const SpinorList &x64, const SpinorList &p, const SpinorList &rr, const SolverCtrl *ctrl,
                               int nshift, size_t n, int count, int sf, int compute, Guard gd, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (count > HISQ_MAX_GRAD_BUFFER || nshift > HISQ_MAX_SHIFTS) return hipErrorInvalidValue;
    const int nb = shift_replay_grid(n, sf, compute);
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_shift_replay<SFc, Rc, REPLAY_GROUP>), dim3(nb), dim3(BLAS_BLOCK), 0, st, x64, p, rr, ctrl, nshift, n, count, gd));
    return hipGetLastError();
}

hipError_t launch_bcg_axpy(char *r, const char *ap, const SolverCtrl *ctrl, size_t n, size_t stride, int nrhs, int sf,
                           int compute, double *partial, Guard gd, hipStream_t st) {
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_bcg_axpy<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, r, ap, ctrl, n, stride, nrhs, partial, gd));
    return hipGetLastError();
}

hipError_t launch_bcg_pupdate(char *p_dst, const char *r, const char *p_src, const SolverCtrl *ctrl, size_t n,
                              size_t stride, int nrhs, int sf, int compute, Guard gd, hipStream_t st) {
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_bcg_pupdate<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, p_dst, r, p_src, ctrl, n, stride, nrhs, gd));
    return hipGetLastError();
}

hipError_t launch_bflush_x(char *x64, size_t stride64, const SpinorList &p, int count, const SolverCtrl *ctrl,
                           size_t n, size_t stride, int nrhs, int sf, int compute, Guard gd, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_bflush_x<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, x64, stride64, p, count, ctrl, n, stride, nrhs, gd));
    return hipGetLastError();
}

hipError_t launch_bru_convert(char *r_s, const char *r64, size_t stride64, const char *p, const char *ap,
                              const SolverCtrl *ctrl, size_t n, size_t stride, int nrhs, int sf, int compute,
                              double *partial, Guard gd, hipStream_t st) {
    HISQ_DISPATCH_SC(sf, compute, hipLaunchKernelGGL((k_bru_convert<SFc, Rc>), dim3(blas_blocks(n)), dim3(BLAS_BLOCK), 0, st, r_s, r64, stride64, p, ap, ctrl, n, stride, nrhs, partial, gd));
    return hipGetLastError();
}

}  // namespace hisq
