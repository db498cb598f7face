// hisq_dslash_kernels.h -- the even-odd HISQ Dslash kernels for gfx950
// (included once per precision triplet so the instantiations compile in
// parallel translation units).
//
// out(x) = sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^dag in(x-mu)
//                 + L_mu(x) in(x+3mu) - L_mu(x-3mu)^dag in(x-3mu) ]
// for the sites x of one parity (the stencil the paper benchmarks, Secs. 5.2-5.3).
//
// The kernel is bound by HBM bandwidth: every link matrix is read exactly once
// per application (non-temporal loads: it is not reused), while each input
// spinor is read by up to 16 neighbouring sites and comes from L2 / the MALL
// after its first use.  The XCD-aware block order keeps the +-3 neighbours of a
// contiguous site range inside one XCD's L2.
//
// Staging: the 16 hops are processed in stages of STAGE hops.  A stage first
// issues the raw loads of its links and spinors (storage words, no decoding),
// then a scheduling barrier, then unpacks to IEEE registers and accumulates the
// mat-vecs in the compute precision.  STAGE sets how many bytes each lane keeps
// in flight against how many registers it holds, i.e. memory-level parallelism
// against occupancy; the autotuner picks it per triplet and lattice.
//
// Right-hand-side blocks (Sec. 1, "Block solvers"): a lane accumulates NR
// right-hand sides for one site, and rg lanes (adjacent, same wavefront) share
// a site and cover rg*NR right-hand sides, so each link is fetched from memory
// once per block of right-hand sides while the register footprint per lane
// stays bounded.  Single right-hand side: NR = rg = 1.
//
// Epilogue: out = b*D(in) + a*x + c*y, then the packed store and optionally a
// per-block partial of Re<x,out> or |out|^2 on the stored values (per
// right-hand side), which fuses the solver's xpay and first reduction.
#pragma once
#include <type_traits>

#include "hisq_internal.h"

namespace hisq {
namespace dsl {

// ---------------------------------------------------------------------------
// raw storage words of one link / one site
// ---------------------------------------------------------------------------

template <int GF> struct LinkRaw;
template <> struct LinkRaw<GF_F64> { f64x2 w[9]; };
template <> struct LinkRaw<GF_F32> { f32x4 w[4]; f32x2 t; };
template <> struct LinkRaw<GF_FIX16> { u32x4 w[2]; unsigned t; };
template <> struct LinkRaw<GF_FIX32> { u32x4 w[4]; u32x2 t; };
// rows as 24-bit shared-exponent records: words 0-3 of row r in 16-byte plane
// r, word 4 of row r in 4-byte plane r after the three 16-byte planes
template <> struct LinkRaw<GF_SX24> { u32x4 w[3]; unsigned t[3]; };

template <int GF> __device__ __forceinline__ LinkRaw<GF> link_load(const char *sub, size_t vh, size_t s);

template <> __device__ __forceinline__ LinkRaw<GF_F64> link_load<GF_F64>(const char *sub, size_t vh, size_t s) {
    LinkRaw<GF_F64> L;
#pragma unroll
    for (int k = 0; k < 9; k++) L.w[k] = ld_nt<f64x2>(sub + k * 16 * vh + 16 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw<GF_F32> link_load<GF_F32>(const char *sub, size_t vh, size_t s) {
    LinkRaw<GF_F32> L;
#pragma unroll
    for (int k = 0; k < 4; k++) L.w[k] = ld_nt<f32x4>(sub + k * 16 * vh + 16 * s);
    L.t = ld_nt<f32x2>(sub + 64 * vh + 8 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw<GF_FIX16> link_load<GF_FIX16>(const char *sub, size_t vh, size_t s) {
    LinkRaw<GF_FIX16> L;
    L.w[0] = ld_nt<u32x4>(sub + 16 * s);
    L.w[1] = ld_nt<u32x4>(sub + 16 * vh + 16 * s);
    L.t = ld_nt<unsigned>(sub + 32 * vh + 4 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw<GF_FIX32> link_load<GF_FIX32>(const char *sub, size_t vh, size_t s) {
    LinkRaw<GF_FIX32> L;
#pragma unroll
    for (int k = 0; k < 4; k++) L.w[k] = ld_nt<u32x4>(sub + k * 16 * vh + 16 * s);
    L.t = ld_nt<u32x2>(sub + 64 * vh + 8 * s);
    return L;
}

template <> __device__ __forceinline__ LinkRaw<GF_SX24> link_load<GF_SX24>(const char *sub, size_t vh, size_t s) {
    LinkRaw<GF_SX24> L;
#pragma unroll
    for (int r = 0; r < 3; r++) L.w[r] = ld_nt<u32x4>(sub + r * 16 * vh + 16 * s);
#pragma unroll
    for (int r = 0; r < 3; r++) L.t[r] = ld_nt<unsigned>(sub + 48 * vh + r * 4 * vh + 4 * s);
    return L;
}

// one row of a shared-exponent link record
template <class R> __device__ __forceinline__ void sx24_row(Mat<R> &U, int r, u32x4 a, unsigned t) {
    const unsigned w[SxFmt<24>::W] = {a.x, a.y, a.z, a.w, t};
    const CVec<R> v = SxCodec<24, R>::decode(w);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        U.re[3 * r + c] = v.re[c];
        U.im[3 * r + c] = v.im[c];
    }
}

template <class R> __device__ __forceinline__ Mat<R> link_decode(const LinkRaw<GF_F64> &L, R) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        U.re[k] = (R)L.w[k].x;
        U.im[k] = (R)L.w[k].y;
    }
    return U;
}
template <class R> __device__ __forceinline__ Mat<R> link_decode(const LinkRaw<GF_F32> &L, R) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        U.re[2 * k] = L.w[k].x; U.im[2 * k] = L.w[k].y; U.re[2 * k + 1] = L.w[k].z; U.im[2 * k + 1] = L.w[k].w;
    }
    U.re[8] = L.t.x;
    U.im[8] = L.t.y;
    return U;
}
// 16-bit fixed point: u = q * g, g = (compute precision)(max/32767)
template <class R> __device__ __forceinline__ Mat<R> link_decode(const LinkRaw<GF_FIX16> &L, R g) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const unsigned ws[4] = {L.w[k].x, L.w[k].y, L.w[k].z, L.w[k].w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            U.re[4 * k + j] = (R)sext16(ws[j]) * g;
            U.im[4 * k + j] = (R)sext16(ws[j] >> 16) * g;
        }
    }
    U.re[8] = (R)sext16(L.t) * g;
    U.im[8] = (R)sext16(L.t >> 16) * g;
    return U;
}
template <class R> __device__ __forceinline__ Mat<R> link_decode(const LinkRaw<GF_FIX32> &L, R g) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        U.re[2 * k] = (R)(int)L.w[k].x * g; U.im[2 * k] = (R)(int)L.w[k].y * g;
        U.re[2 * k + 1] = (R)(int)L.w[k].z * g; U.im[2 * k + 1] = (R)(int)L.w[k].w * g;
    }
    U.re[8] = (R)(int)L.t.x * g;
    U.im[8] = (R)(int)L.t.y * g;
    return U;
}

// shared-exponent rows carry their own scale
template <class R> __device__ __forceinline__ Mat<R> link_decode(const LinkRaw<GF_SX24> &L, R) {
    Mat<R> U;
#pragma unroll
    for (int r = 0; r < 3; r++) sx24_row(U, r, L.w[r], L.t[r]);
    return U;
}

// Long links stored as two rows (12 reals) of U, where L = c * s * U with U in
// SU(3), c a global real constant and s = +-1 the staggered phase of the link
// (Sec. 1 "Compression": a special unitary matrix is fixed by two of its rows).
// Row 3 is rebuilt as conj(row1 x row2) in the compute precision.
template <int GF> struct LinkRaw12;
template <> struct LinkRaw12<GF_F64> { f64x2 w[6]; };
template <> struct LinkRaw12<GF_F32> { f32x4 w[3]; };
template <> struct LinkRaw12<GF_FIX16> { u32x4 w; u32x2 t; };
template <> struct LinkRaw12<GF_FIX32> { u32x4 w[3]; };
template <> struct LinkRaw12<GF_SX24> { u32x4 w[2]; unsigned t[2]; };

template <int GF> __device__ __forceinline__ LinkRaw12<GF> link_load12(const char *sub, size_t vh, size_t s);
template <> __device__ __forceinline__ LinkRaw12<GF_F64> link_load12<GF_F64>(const char *sub, size_t vh, size_t s) {
    LinkRaw12<GF_F64> L;
#pragma unroll
    for (int k = 0; k < 6; k++) L.w[k] = ld_nt<f64x2>(sub + k * 16 * vh + 16 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw12<GF_F32> link_load12<GF_F32>(const char *sub, size_t vh, size_t s) {
    LinkRaw12<GF_F32> L;
#pragma unroll
    for (int k = 0; k < 3; k++) L.w[k] = ld_nt<f32x4>(sub + k * 16 * vh + 16 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw12<GF_FIX16> link_load12<GF_FIX16>(const char *sub, size_t vh, size_t s) {
    LinkRaw12<GF_FIX16> L;
    L.w = ld_nt<u32x4>(sub + 16 * s);
    L.t = ld_nt<u32x2>(sub + 16 * vh + 8 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw12<GF_FIX32> link_load12<GF_FIX32>(const char *sub, size_t vh, size_t s) {
    LinkRaw12<GF_FIX32> L;
#pragma unroll
    for (int k = 0; k < 3; k++) L.w[k] = ld_nt<u32x4>(sub + k * 16 * vh + 16 * s);
    return L;
}

template <> __device__ __forceinline__ LinkRaw12<GF_SX24> link_load12<GF_SX24>(const char *sub, size_t vh, size_t s) {
    LinkRaw12<GF_SX24> L;
#pragma unroll
    for (int r = 0; r < 2; r++) L.w[r] = ld_nt<u32x4>(sub + r * 16 * vh + 16 * s);
#pragma unroll
    for (int r = 0; r < 2; r++) L.t[r] = ld_nt<unsigned>(sub + 32 * vh + r * 4 * vh + 4 * s);
    return L;
}

// rows 1-2 -> full matrix; third row conj(r0 x r1); rows 1-2 times c, row 3
// times c3
template <class R> __device__ __forceinline__ Mat<R> complete_su3(Mat<R> U, R c, R c3) {
    const R ar[3] = {U.re[0], U.re[1], U.re[2]}, ai[3] = {U.im[0], U.im[1], U.im[2]};
    const R br[3] = {U.re[3], U.re[4], U.re[5]}, bi[3] = {U.im[3], U.im[4], U.im[5]};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int i = (k + 1) % 3, j = (k + 2) % 3;
        // (a_i b_j - a_j b_i), conjugated
        const R re = ar[i] * br[j] - ai[i] * bi[j] - (ar[j] * br[i] - ai[j] * bi[i]);
        const R im = ar[i] * bi[j] + ai[i] * br[j] - (ar[j] * bi[i] + ai[j] * br[i]);
        U.re[6 + k] = re * c3;
        U.im[6 + k] = -im * c3;
    }
#pragma unroll
    for (int k = 0; k < 6; k++) {
        U.re[k] *= c;
        U.im[k] *= c;
    }
    return U;
}

// rows 1-2 of a two-row link (fixed point scaled by g)
template <class R> __device__ __forceinline__ Mat<R> link_rows12(const LinkRaw12<GF_F64> &L, R) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        U.re[k] = (R)L.w[k].x;
        U.im[k] = (R)L.w[k].y;
    }
    return U;
}
template <class R> __device__ __forceinline__ Mat<R> link_rows12(const LinkRaw12<GF_F32> &L, R) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        U.re[2 * k] = L.w[k].x; U.im[2 * k] = L.w[k].y; U.re[2 * k + 1] = L.w[k].z; U.im[2 * k + 1] = L.w[k].w;
    }
    return U;
}
template <class R> __device__ __forceinline__ Mat<R> link_rows12(const LinkRaw12<GF_FIX16> &L, R g) {
    Mat<R> U;
    const unsigned ws[6] = {L.w.x, L.w.y, L.w.z, L.w.w, L.t.x, L.t.y};
#pragma unroll
    for (int k = 0; k < 6; k++) {
        U.re[k] = (R)sext16(ws[k]) * g;
        U.im[k] = (R)sext16(ws[k] >> 16) * g;
    }
    return U;
}
template <class R> __device__ __forceinline__ Mat<R> link_rows12(const LinkRaw12<GF_FIX32> &L, R g) {
    Mat<R> U;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        U.re[2 * k] = (R)(int)L.w[k].x * g; U.im[2 * k] = (R)(int)L.w[k].y * g;
        U.re[2 * k + 1] = (R)(int)L.w[k].z * g; U.im[2 * k + 1] = (R)(int)L.w[k].w * g;
    }
    return U;
}
template <class R> __device__ __forceinline__ Mat<R> link_rows12(const LinkRaw12<GF_SX24> &L, R) {
    Mat<R> U;
#pragma unroll
    for (int r = 0; r < 2; r++) sx24_row(U, r, L.w[r], L.t[r]);
    return U;
}
// the full long link c * U
template <class R, int GF> __device__ __forceinline__ Mat<R> link_decode12(const LinkRaw12<GF> &L, R g, R c) {
    return complete_su3(link_rows12<R>(L, g), c, c);
}

// Long links stored as eight parameters (Sec. 1 "Compression": a special
// unitary matrix has eight real degrees of freedom) of W = |c| U: Re/Im of
// W01, W02, W10, then v_a = tan(arg(W00)/4) and v_c = tan(arg(W20)/4).
// Planes of 16 bytes: F64 four (two parameters each), FIX32 two (four each;
// the entries scaled by the long field's max |real component|, the phase
// parameters by 1).  Only the FP64-arithmetic triplets use this storage.
template <int GF> struct LinkRaw8 { unsigned unused; };   // formats without this storage: never loaded
template <> struct LinkRaw8<GF_F64> { f64x2 w[4]; };
template <> struct LinkRaw8<GF_FIX32> { u32x4 w[2]; };

template <int GF> __device__ __forceinline__ LinkRaw8<GF> link_load8(const char *sub, size_t vh, size_t s);
template <> __device__ __forceinline__ LinkRaw8<GF_F64> link_load8<GF_F64>(const char *sub, size_t vh, size_t s) {
    LinkRaw8<GF_F64> L;
#pragma unroll
    for (int k = 0; k < 4; k++) L.w[k] = ld_nt<f64x2>(sub + k * 16 * vh + 16 * s);
    return L;
}
template <> __device__ __forceinline__ LinkRaw8<GF_FIX32> link_load8<GF_FIX32>(const char *sub, size_t vh, size_t s) {
    LinkRaw8<GF_FIX32> L;
#pragma unroll
    for (int k = 0; k < 2; k++) L.w[k] = ld_nt<u32x4>(sub + k * 16 * vh + 16 * s);
    return L;
}

// the eight parameters in the compute precision (entries times g for fixed point)
template <class R> __device__ __forceinline__ void link_params8(const LinkRaw8<GF_F64> &L, R g, R (&p)[8]) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
        p[2 * k] = (R)L.w[k].x * (k < 3 ? g : R(1));
        p[2 * k + 1] = (R)L.w[k].y * (k < 3 ? g : R(1));
    }
}
template <class R> __device__ __forceinline__ void link_params8(const LinkRaw8<GF_FIX32> &L, R g, R (&p)[8]) {
    const unsigned ws[8] = {L.w[0].x, L.w[0].y, L.w[0].z, L.w[0].w, L.w[1].x, L.w[1].y, L.w[1].z, L.w[1].w};
    const R gv = (R)(1.0 / 2147483647.0);
#pragma unroll
    for (int k = 0; k < 8; k++) p[k] = (R)(int)ws[k] * (k < 6 ? g : gv);
}

// U from its eight parameters.  Rows have unit norm: |u00|^2 = 1 - N with
// N = |u01|^2 + |u02|^2, and the first column: |u20|^2 = N - |u10|^2; the
// phases e^{i theta} = h^2 with h = (1 + i v)^2 / (1 + v^2).  Row 2 solves
// the 2x2 system "orthogonal to row 1" and "u20 = conj(u01 u12 - u02 u11)"
// (determinant N), row 3 the analogous one; in closed form
//   u11 = -(conj(u00) u01 u10 + conj(u02 u20)) / N
//   u12 =  (conj(u01 u20) - conj(u00) u02 u10) / N
//   u21 =  (conj(u02 u10) - conj(u00) u01 u20) / N
//   u22 = -(conj(u00) u02 u20 + conj(u01 u10)) / N
// 1/x (x > 0) and sqrt(x) (0 for x <= 0) in FP64 from the hardware estimates
// refined by two Newton steps each: within a few ulp, far cheaper than the
// correctly rounded division and root, which the rebuild does not need
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double sqrt_nr(double x) {
    const double xp = x > 0.0 ? x : 1.0;
    double y = __builtin_amdgcn_rsq(xp);
    const double h = 0.5 * xp;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return x > 0.0 ? xp * y : 0.0;
}

template <class R> __device__ __forceinline__ Mat<R> su3_from8(const R (&p)[8]) {
    static_assert(std::is_same<R, double>::value, "eight-parameter links are rebuilt in FP64");
    auto cmul = [](R ar, R ai, R br, R bi, R &r, R &i) {
        r = ar * br - ai * bi;
        i = ar * bi + ai * br;
    };
    // e^{i theta} = ((1 + iv)^2 / (1 + v^2))^2
    auto phase = [](R v, R &er, R &ei) {
        const R d = rcp_nr(R(1) + v * v);
        const R hr = (R(1) - v * v) * d, hi = R(2) * v * d;
        er = hr * hr - hi * hi;
        ei = R(2) * hr * hi;
    };
    const R a2r = p[0], a2i = p[1], a3r = p[2], a3i = p[3], b1r = p[4], b1i = p[5];
    const R n = a2r * a2r + a2i * a2i + a3r * a3r + a3i * a3i;
    R ear, eai, ecr, eci;
    phase(p[6], ear, eai);
    phase(p[7], ecr, eci);
    const R ma = sqrt_nr(R(1) - n), mc = sqrt_nr(n - (b1r * b1r + b1i * b1i));
    const R a1r = ma * ear, a1i = ma * eai, c1r = mc * ecr, c1i = mc * eci;
    const R in = rcp_nr(n);
    // conj(a1) a2, conj(a1) a3
    const R xa2r = a1r * a2r + a1i * a2i, xa2i = a1r * a2i - a1i * a2r;
    const R xa3r = a1r * a3r + a1i * a3i, xa3i = a1r * a3i - a1i * a3r;
    R t0r, t0i, t1r, t1i;
    Mat<R> U;
    U.re[0] = a1r; U.im[0] = a1i; U.re[1] = a2r; U.im[1] = a2i; U.re[2] = a3r; U.im[2] = a3i;
    U.re[3] = b1r; U.im[3] = b1i; U.re[6] = c1r; U.im[6] = c1i;
    cmul(xa2r, xa2i, b1r, b1i, t0r, t0i);          // conj(a1) a2 b1
    cmul(a3r, a3i, c1r, c1i, t1r, t1i);            // a3 c1
    U.re[4] = -(t0r + t1r) * in; U.im[4] = -(t0i - t1i) * in;
    cmul(a2r, a2i, c1r, c1i, t0r, t0i);            // a2 c1
    cmul(xa3r, xa3i, b1r, b1i, t1r, t1i);          // conj(a1) a3 b1
    U.re[5] = (t0r - t1r) * in; U.im[5] = (-t0i - t1i) * in;
    cmul(a3r, a3i, b1r, b1i, t0r, t0i);            // a3 b1
    cmul(xa2r, xa2i, c1r, c1i, t1r, t1i);          // conj(a1) a2 c1
    U.re[7] = (t0r - t1r) * in; U.im[7] = (-t0i - t1i) * in;
    cmul(xa3r, xa3i, c1r, c1i, t0r, t0i);          // conj(a1) a3 c1
    cmul(a2r, a2i, b1r, b1i, t1r, t1i);            // a2 b1
    U.re[8] = -(t0r + t1r) * in; U.im[8] = -(t0i - t1i) * in;
    return U;
}

template <int SF> struct SpinRaw;
template <> struct SpinRaw<SF_F64> { f64x2 w[3]; };
template <> struct SpinRaw<SF_F32> { f32x4 a; f32x2 b; };
template <> struct SpinRaw<SF_HALF16> { u32x4 w; };
template <> struct SpinRaw<SF_INT20> { u32x4 w; };
template <> struct SpinRaw<SF_INT30> { u32x4 a; u32x2 b; };
template <> struct SpinRaw<SF_INT24> { u32x4 a; unsigned b; };

template <int SF> __device__ __forceinline__ SpinRaw<SF> spin_load(const char *base, size_t n, size_t s);
template <> __device__ __forceinline__ SpinRaw<SF_F64> spin_load<SF_F64>(const char *base, size_t n, size_t s) {
    SpinRaw<SF_F64> P;
#pragma unroll
    for (int c = 0; c < 3; c++) P.w[c] = ld<f64x2>(base + c * 16 * n + 16 * s);
    return P;
}
template <> __device__ __forceinline__ SpinRaw<SF_F32> spin_load<SF_F32>(const char *base, size_t n, size_t s) {
    SpinRaw<SF_F32> P;
    P.a = ld<f32x4>(base + 16 * s);
    P.b = ld<f32x2>(base + 16 * n + 8 * s);
    return P;
}
template <> __device__ __forceinline__ SpinRaw<SF_HALF16> spin_load<SF_HALF16>(const char *base, size_t, size_t s) {
    SpinRaw<SF_HALF16> P;
    P.w = ld<u32x4>(base + 16 * s);
    return P;
}
template <> __device__ __forceinline__ SpinRaw<SF_INT20> spin_load<SF_INT20>(const char *base, size_t, size_t s) {
    SpinRaw<SF_INT20> P;
    P.w = ld<u32x4>(base + 16 * s);
    return P;
}
template <> __device__ __forceinline__ SpinRaw<SF_INT30> spin_load<SF_INT30>(const char *base, size_t n, size_t s) {
    SpinRaw<SF_INT30> P;
    P.a = ld<u32x4>(base + 16 * s);
    P.b = ld<u32x2>(base + 16 * n + 8 * s);
    return P;
}
template <> __device__ __forceinline__ SpinRaw<SF_INT24> spin_load<SF_INT24>(const char *base, size_t n, size_t s) {
    SpinRaw<SF_INT24> P;
    P.a = ld<u32x4>(base + 16 * s);
    P.b = ld<unsigned>(base + 16 * n + 4 * s);
    return P;
}

template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_F64> &P) {
    CVec<R> v;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        v.re[c] = (R)P.w[c].x;
        v.im[c] = (R)P.w[c].y;
    }
    return v;
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_F32> &P) {
    CVec<R> v;
    v.re[0] = P.a.x; v.im[0] = P.a.y; v.re[1] = P.a.z; v.im[1] = P.a.w; v.re[2] = P.b.x; v.im[2] = P.b.y;
    return v;
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_HALF16> &P) {
    return SpinorIO<SF_HALF16, R>::decode(P.w);
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_INT20> &P) {
    return SpinorIO<SF_INT20, R>::decode(P.w);
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_INT30> &P) {
    return SpinorIO<SF_INT30, R>::decode(P.a, P.b);
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_INT24> &P) {
    const unsigned w[SxFmt<24>::W] = {P.a.x, P.a.y, P.a.z, P.a.w, P.b};
    return SxCodec<24, R>::decode(w);
}

// Link scales folded into the spinor's site scale.  A hop adds link * v.  When
// the spinor format carries a per-site scale, the link is decoded as M with
// link = f * M (fixed-point links: the stored integers; two-row long links: the
// SU(3) matrix without the long-link constant and the phase) and v with its
// site scale times f, so the scales cost one multiply per right-hand side
// instead of one per link element.  Other spinor formats use f = 1.
template <int SF> constexpr bool spinor_scaled() {
    return SF == SF_HALF16 || SF == SF_INT20 || SF == SF_INT30 || SF == SF_INT24;
}
template <int GF> constexpr bool gauge_fixed() { return GF == GF_FIX16 || GF == GF_FIX32; }

template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_F64> &P, R) { return spin_decode<R>(P); }
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_F32> &P, R) { return spin_decode<R>(P); }
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_HALF16> &P, R f) {
    return SpinorIO<SF_HALF16, R>::decode(P.w, (float)f);
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_INT20> &P, R f) {
    return SpinorIO<SF_INT20, R>::decode(P.w, (float)f);
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_INT30> &P, R f) {
    return SpinorIO<SF_INT30, R>::decode(P.a, P.b, f);
}
template <class R> __device__ __forceinline__ CVec<R> spin_decode(const SpinRaw<SF_INT24> &P, R f) {
    const unsigned w[SxFmt<24>::W] = {P.a.x, P.a.y, P.a.z, P.a.w, P.b};
    return SxCodec<24, R>::decode(w, f);
}

// a fat or 18-real long link with scale g: M and f
template <int SF, class R, int GF> __device__ __forceinline__ Mat<R> hop_link(const LinkRaw<GF> &L, R g, R &f) {
    if constexpr (spinor_scaled<SF>() && gauge_fixed<GF>()) {
        f = g;
        return link_decode<R>(L, R(1));
    } else {
        f = R(1);
        return link_decode<R>(L, g);
    }
}
// a two-row long link c * U (rows scaled by g when fixed point): M and f.  For
// fixed point the rows are Q1 = U1/g, Q2 = U2/g and g conj(Q1 x Q2) = U3/g, so
// c U = (c g) M.
template <int SF, class R, int GF>
__device__ __forceinline__ Mat<R> hop_link12(const LinkRaw12<GF> &L, R g, R c, R &f) {
    if constexpr (spinor_scaled<SF>() && gauge_fixed<GF>()) {
        f = c * g;
        return complete_su3(link_rows12<R>(L, R(1)), R(1), g);
    } else if constexpr (spinor_scaled<SF>()) {
        f = c;
        return complete_su3(link_rows12<R>(L, g), R(1), R(1));
    } else {
        f = R(1);
        return link_decode12<R>(L, g, c);
    }
}

// an eight-parameter long link c * U: M and f (the rebuild needs the true
// entries, so fixed-point scales are applied to the parameters; c goes into f
// when the spinor format has a site scale)
template <int SF, class R, int GF>
__device__ __forceinline__ Mat<R> hop_link8(const LinkRaw8<GF> &L, R g, R c, R &f) {
    R prm[8];
    link_params8<R>(L, g, prm);
    Mat<R> U = su3_from8<R>(prm);
    if constexpr (spinor_scaled<SF>()) {
        f = c;
    } else {
        f = R(1);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            U.re[k] *= c;
            U.im[k] *= c;
        }
    }
    return U;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

// checkerboard indices of the +-1, +-3 neighbours of site s along each direction
struct Nbrs {
    int f1[4], b1[4], f3[4], b3[4];
    float lsf[4], lsb[4];  // phase s = +-1 of the forward link L(x) and the backward link L(x-3mu)
};

// staggered phase eta_mu(x) times the antiperiodic time sign of a three-hop
// link starting at time t (negative when the hop crosses t = T)
__device__ __forceinline__ float long_phase(int mu, int x, int y, int z, int t, int T) {
    const int e = mu == 0 ? 0 : mu == 1 ? x : mu == 2 ? x + y : x + y + z;
    const int b = (mu == 3 && t >= T - 3) ? 1 : 0;
    return ((e + b) & 1) ? -1.0f : 1.0f;
}

__device__ __forceinline__ int wrap_add(int c, int h, int L) {
    int v = c + h;
    v -= (v >= L) ? L : 0;
    v += (v < 0) ? L : 0;
    return v;
}

__device__ __forceinline__ Nbrs neighbours(const Geom &g, int s, int parity) {
    int r = fdiv(s, g.dX2);
    const int xcb = s - r * g.X2;
    int r2 = fdiv(r, g.dY);
    const int y = r - r2 * g.Y;
    const int t = fdiv(r2, g.dZ);
    const int z = r2 - t * g.Z;
    const int x = 2 * xcb + ((y + z + t + parity) & 1);
    const int row = s - xcb;
    Nbrs n;
    n.f1[0] = row + (wrap_add(x, 1, g.X) >> 1);
    n.b1[0] = row + (wrap_add(x, -1, g.X) >> 1);
    n.f3[0] = row + (wrap_add(x, 3, g.X) >> 1);
    n.b3[0] = row + (wrap_add(x, -3, g.X) >> 1);
    n.f1[1] = s + (wrap_add(y, 1, g.Y) - y) * g.sy;
    n.b1[1] = s + (wrap_add(y, -1, g.Y) - y) * g.sy;
    n.f3[1] = s + (wrap_add(y, 3, g.Y) - y) * g.sy;
    n.b3[1] = s + (wrap_add(y, -3, g.Y) - y) * g.sy;
    n.f1[2] = s + (wrap_add(z, 1, g.Z) - z) * g.sz;
    n.b1[2] = s + (wrap_add(z, -1, g.Z) - z) * g.sz;
    n.f3[2] = s + (wrap_add(z, 3, g.Z) - z) * g.sz;
    n.b3[2] = s + (wrap_add(z, -3, g.Z) - z) * g.sz;
    n.f1[3] = s + (wrap_add(t, 1, g.T) - t) * g.st;
    n.b1[3] = s + (wrap_add(t, -1, g.T) - t) * g.st;
    n.f3[3] = s + (wrap_add(t, 3, g.T) - t) * g.st;
    n.b3[3] = s + (wrap_add(t, -3, g.T) - t) * g.st;
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        n.lsf[mu] = long_phase(mu, x, y, z, t, g.T);
        n.lsb[mu] = long_phase(mu, x, y, z, wrap_add(t, mu == 3 ? -3 : 0, g.T), g.T);
    }
    return n;
}

// hop h = 4*mu + kind, kind 0: F_mu(x) in(x+mu); 1: -F_mu(x-mu)^dag in(x-mu);
// 2: L_mu(x) in(x+3mu); 3: -L_mu(x-3mu)^dag in(x-3mu)
__device__ __forceinline__ int hop_spinor_site(const Nbrs &n, int h) {
    const int mu = h >> 2, kind = h & 3;
    return kind == 0 ? n.f1[mu] : kind == 1 ? n.b1[mu] : kind == 2 ? n.f3[mu] : n.b3[mu];
}

// site coordinates of checkerboard index s (parity p)
struct Coords {
    int x, y, z, t, row;
};

__device__ __forceinline__ Coords coords_of(const Geom &g, int s, int parity) {
    Coords c;
    const int r = fdiv(s, g.dX2);
    const int xcb = s - r * g.X2;
    const int r2 = fdiv(r, g.dY);
    c.y = r - r2 * g.Y;
    c.t = fdiv(r2, g.dZ);
    c.z = r2 - c.t * g.Z;
    c.x = 2 * xcb + ((c.y + c.z + c.t + parity) & 1);
    c.row = s - xcb;
    return c;
}

// spinor (and backward-link) site of hop h computed at run time
__device__ __forceinline__ int hop_site_rt(const Geom &g, const Coords &c, int s, int h) {
    const int mu = h >> 2, kind = h & 3;
    const int d = ((kind & 2) ? 3 : 1) * ((kind & 1) ? -1 : 1);
    if (mu == 0) return c.row + (wrap_add(c.x, d, g.X) >> 1);
    const int co = mu == 1 ? c.y : mu == 2 ? c.z : c.t;
    const int L = mu == 1 ? g.Y : mu == 2 ? g.Z : g.T;
    const int stride = mu == 1 ? g.sy : mu == 2 ? g.sz : g.st;
    return s + (wrap_add(co, d, L) - co) * stride;
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------

// field column of the launch's right-hand side k, and whether it exists
__device__ __forceinline__ int colmap(const DslashArgs &A, int k) {
    return A.cmapped ? (int)((A.cmap >> (4 * k)) & 15ull) : k;
}
__device__ __forceinline__ bool colvalid(const DslashArgs &A, int k, int ncol) {
    return A.cmapped ? ((A.cvalid >> k) & 1u) != 0 : k < ncol;
}

// The epilogue of one output site: out = b*D(in) + a*x + c*y for each live
// right-hand side j of the lane (field column col(j)), packed and stored, and
// the optional reduction.
template <int SF, class R, int NR, bool RED, class ColF>
__device__ __forceinline__ void site_epilogue(const DslashArgs &A, int s, ColF col, unsigned live,
                                              const R (&acoef)[NR], CVec<R> (&acc)[NR], double (&red)[NR]) {
    const size_t fs = A.field_stride;
    const size_t vh = (size_t)A.g.vh;
    const R b = (R)A.b, cc = (R)A.c;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        if (!((live >> j) & 1u)) continue;
        const size_t off = (size_t)col(j) * fs;
        const R a = acoef[j];
        CVec<R> xv;
        cvec_zero(xv);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc[j].re[c] *= b;
            acc[j].im[c] *= b;
        }
        if (A.x) {
            xv = SpinorIO<SF, R>::load(A.x + off, vh, s);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                acc[j].re[c] = fma(a, xv.re[c], acc[j].re[c]);
                acc[j].im[c] = fma(a, xv.im[c], acc[j].im[c]);
            }
        }
        if (A.y) {
            const CVec<R> yv = SpinorIO<SF, R>::load(A.y + off, vh, s);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                acc[j].re[c] = fma(cc, yv.re[c], acc[j].re[c]);
                acc[j].im[c] = fma(cc, yv.im[c], acc[j].im[c]);
            }
        }
        const CVec<R> o = SpinorIO<SF, R>::store(A.out + off, vh, s, acc[j]);
        if (RED) {
            if (A.red == RED_DOT_X) {
#pragma unroll
                for (int c = 0; c < 3; c++)
                    red[j] += (double)xv.re[c] * (double)o.re[c] + (double)xv.im[c] * (double)o.im[c];
            } else {
#pragma unroll
                for (int c = 0; c < 3; c++)
                    red[j] += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
            }
        }
    }
}

// One output site s for the lane's right-hand sides c0 + j*cs, j < NR (those
// in `live`): the 16 hops, the epilogue out = b*D(in) + a*x + c*y, the packed
// store, and the optional reduction into red[].
template <int GF, int SF, class R, int NR, int STAGE, bool RED, int LR>
__device__ __forceinline__ void dslash_site(const DslashArgs &A, int s, int c0, int cs, unsigned live,
                                            const R (&acoef)[NR], double (&red)[NR]) {
    const Geom &g = A.g;
    const size_t fs = A.field_stride;
    const size_t vh = (size_t)g.vh;
    const int p = A.parity, q = 1 - p;
    static_assert(LR != 8 || (NR == 1 && GF != GF_SX24), "eight-parameter long links: one right-hand side per lane");
    const size_t sub = (size_t)gauge_matrix_bytes(GF) * vh;
    const size_t lsub = LR == 12 ? (size_t)gauge_matrix_bytes12(GF) * vh
                                 : LR == 8 ? (size_t)gauge_matrix_bytes8(GF) * vh : sub;
    const R gf = (R)A.gfat, gl = (R)A.glong, lc = (R)A.lcoef;
    // input field of the lane's right-hand side j
    auto in_col = [&](int j) { return A.in + (size_t)colmap(A, c0 + j * cs) * fs; };
    CVec<R> acc[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) cvec_zero(acc[j]);
    if (NR > 8 && STAGE == 1) {
        // 16 right-hand sides per lane: one hop at a time in a loop (bounded registers)
        const Coords c = coords_of(g, s, p);
#pragma unroll 1
        for (int h = 0; h < 16; h++) {
            const int ss = hop_site_rt(g, c, s, h);
            const int ls = (h & 1) ? ss : s;
            const int lpar = (h & 1) ? q : p;
            Mat<R> U;
            R f;
            SpinRaw<SF> Pr[NR];
            if (LR == 12 && (h & 2)) {
                const int mu = h >> 2;
                const int tl = (mu == 3 && (h & 1)) ? wrap_add(c.t, -3, g.T) : c.t;
                const LinkRaw12<GF> Lr = link_load12<GF>(A.lng + (size_t)(2 * mu + lpar) * lsub, vh, ls);
#pragma unroll
                for (int j = 0; j < NR; j++) Pr[j] = ((live >> j) & 1u) ? spin_load<SF>(in_col(j), vh, ss) : SpinRaw<SF>{};
                U = hop_link12<SF>(Lr, gl, lc * (R)long_phase(mu, c.x, c.y, c.z, tl, g.T), f);
            } else {
                const char *field = (h & 2) ? A.lng : A.fat;
                const LinkRaw<GF> Lr = link_load<GF>(field + (size_t)(2 * (h >> 2) + lpar) * sub, vh, ls);
#pragma unroll
                for (int j = 0; j < NR; j++) Pr[j] = ((live >> j) & 1u) ? spin_load<SF>(in_col(j), vh, ss) : SpinRaw<SF>{};
                U = hop_link<SF>(Lr, (h & 2) ? gl : gf, f);
            }
            if (h & 1) {
#pragma unroll
                for (int j = 0; j < NR; j++)
                    if ((live >> j) & 1u) mdv_sub(acc[j], U, spin_decode<R>(Pr[j], f));
            } else {
#pragma unroll
                for (int j = 0; j < NR; j++)
                    if ((live >> j) & 1u) mv_add(acc[j], U, spin_decode<R>(Pr[j], f));
            }
        }
    }
    // STAGE > 0: the raw words of STAGE hops are loaded, then unpacked and
    // applied; STAGE < 0: -STAGE hops per stage, double-buffered, the next
    // stage's loads issued before this stage's arithmetic so that every wave
    // keeps loads in flight while it computes
    constexpr int SB = STAGE < 0 ? -STAGE : STAGE;
    constexpr bool PIPE = STAGE < 0;
    constexpr int NBUF = PIPE ? 2 : 1;
    constexpr int NST = (NR > 8 && STAGE == 1) ? 0 : 16 / SB;
    const Nbrs n = neighbours(g, s, p);
    LinkRaw<GF> L[NBUF][SB];
    LinkRaw12<GF> L12[NBUF][SB];
    LinkRaw8<GF> L8[NBUF][SB];
    SpinRaw<SF> P[NBUF][SB][NR];
    // input column of each of the lane's right-hand sides, computed once per
    // site; a column the lane does not compute reads its first live column
    // (valid memory, a cache hit, never used), so the loads carry no branches
    // and no zero fill; the arithmetic of a column is skipped when no lane of
    // the wave computes it
    const char *colp[NR];
    {
        const char *first = in_col(NR == 1 ? 0 : __builtin_ctz(live));
#pragma unroll
        for (int j = 0; j < NR; j++) colp[j] = (NR == 1 || ((live >> j) & 1u)) ? in_col(j) : first;
    }
    auto load_stage = [&](int h0, int bf) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < SB; i++) {
            const int h = h0 + i;
            const int ss = hop_spinor_site(n, h);
            const int ls = (h & 1) ? ss : s;
            const int lpar = (h & 1) ? q : p;
            if constexpr (LR == 8) {
                if (h & 2)
                    L8[bf][i] = link_load8<GF>(A.lng + (size_t)(2 * (h >> 2) + lpar) * lsub, vh, ls);
                else
                    L[bf][i] = link_load<GF>(A.fat + (size_t)(2 * (h >> 2) + lpar) * sub, vh, ls);
            } else if (LR == 12 && (h & 2)) {
                L12[bf][i] = link_load12<GF>(A.lng + (size_t)(2 * (h >> 2) + lpar) * lsub, vh, ls);
            } else {
                L[bf][i] = link_load<GF>(((h & 2) ? A.lng : A.fat) + (size_t)(2 * (h >> 2) + lpar) * sub, vh, ls);
            }
#pragma unroll
            for (int j = 0; j < NR; j++) P[bf][i][j] = spin_load<SF>(colp[j], vh, ss);
        }
    };
    auto apply_stage = [&](int h0, int bf) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < SB; i++) {
            const int h = h0 + i;
            R f;
            Mat<R> U;
            if constexpr (LR == 8)
                U = (h & 2) ? hop_link8<SF>(L8[bf][i], gl, lc * (R)((h & 1) ? n.lsb[h >> 2] : n.lsf[h >> 2]), f)
                            : hop_link<SF>(L[bf][i], gf, f);
            else
                U = (LR == 12 && (h & 2))
                        ? hop_link12<SF>(L12[bf][i], gl, lc * (R)((h & 1) ? n.lsb[h >> 2] : n.lsf[h >> 2]), f)
                        : hop_link<SF>(L[bf][i], (h & 2) ? gl : gf, f);
#pragma unroll
            for (int j = 0; j < NR; j++) {
                if (NR > 1 && !((live >> j) & 1u)) continue;
                const CVec<R> v = spin_decode<R>(P[bf][i][j], f);
                if (h & 1)
                    mdv_sub(acc[j], U, v);
                else
                    mv_add(acc[j], U, v);
            }
        }
    };
    if (PIPE && NST > 0) load_stage(0, 0);
#pragma unroll
    for (int k = 0; k < NST; k++) {
        if (!PIPE)
            load_stage(k * SB, 0);
        else if (k + 1 < NST)
            load_stage((k + 1) * SB, (k + 1) % NBUF);
        __builtin_amdgcn_sched_barrier(0);
        apply_stage(k * SB, k % NBUF);
        if (PIPE) __builtin_amdgcn_sched_barrier(0);
    }
    site_epilogue<SF, R, NR, RED>(A, s, [&](int j) { return colmap(A, c0 + j * cs); }, live, acoef, acc, red);
}

// Batched sites on the matrix cores (STAGE == MFMA_STAGE, FP32 compute, four
// lanes per site).  The four lanes of a site form one block of the 16-block
// 4x4x1 FP32 MFMA.  Lane i supplies row i of the operand A, row i of the
// hop's link in real form (the real parts of the output in one tile, the
// imaginary parts in another); lane j supplies column j of B, one component
// of its own right-hand side's neighbour spinor per K step, and receives
// column j of the product in four accumulator registers.  Output rows 0-2
// are colours 0-2; the fourth lane's row is padding whose output is never
// read.  Each lane therefore needs only its own row (forward hops) or column
// (backward hops) of the link: fat and 18-real links select the stored words
// of those three entries and decode only them; two-row long links are
// completed in full (row 3 needs both stored rows) before the selection.
// The lane's right-hand sides are the columns 4 m + lane (m < NR).
constexpr int MFMA_STAGE = 5;
typedef float f32x4v __attribute__((ext_vector_type(4)));

// lane of the site's block: li == 0 (and the padding lane 3), li == 1, else li == 2
struct QuadSel {
    bool c0, c1;
};
template <class T> __device__ __forceinline__ T qsel(const QuadSel &q, T a, T b, T c) {
    return q.c0 ? a : (q.c1 ? b : c);
}

// stored words of complex entry k (row-major) of a fat or 18-real link
__device__ __forceinline__ unsigned entry_word(const LinkRaw<GF_FIX16> &L, int k) {
    return k < 4 ? L.w[0][k] : k < 8 ? L.w[1][k - 4] : L.t;
}
__device__ __forceinline__ u32x2 entry_word(const LinkRaw<GF_FIX32> &L, int k) {
    return k < 8 ? u32x2{L.w[k >> 1][2 * (k & 1)], L.w[k >> 1][2 * (k & 1) + 1]} : L.t;
}
__device__ __forceinline__ f32x2 entry_word(const LinkRaw<GF_F32> &L, int k) {
    return k < 8 ? f32x2{L.w[k >> 1][2 * (k & 1)], L.w[k >> 1][2 * (k & 1) + 1]} : L.t;
}
template <int GF> constexpr bool entry_select() { return GF == GF_FIX16 || GF == GF_FIX32 || GF == GF_F32; }

// row li (BACK false) or column li (BACK true) of a fat or 18-real link with
// scale g, as M and f with the convention of hop_link
template <int SF, int GF, bool BACK>
__device__ __forceinline__ void lane_link(const LinkRaw<GF> &L, float g, const QuadSel &q, float (&ur)[3],
                                          float (&ui)[3], float &f) {
    constexpr bool fold = spinor_scaled<SF>() && gauge_fixed<GF>();
    if constexpr (entry_select<GF>()) {
        f = fold ? g : 1.0f;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int k0 = BACK ? 3 * c : c, k1 = BACK ? 3 * c + 1 : 3 + c, k2 = BACK ? 3 * c + 2 : 6 + c;
            const auto w = qsel(q, entry_word(L, k0), entry_word(L, k1), entry_word(L, k2));
            if constexpr (GF == GF_FIX16) {
                ur[c] = (float)sext16(w);
                ui[c] = (float)sext16(w >> 16);
            } else if constexpr (GF == GF_FIX32) {
                ur[c] = (float)(int)w.x;
                ui[c] = (float)(int)w.y;
            } else {
                ur[c] = w.x;
                ui[c] = w.y;
            }
            if constexpr (gauge_fixed<GF>() && !fold) {
                ur[c] *= g;
                ui[c] *= g;
            }
        }
    } else {
        const Mat<float> U = hop_link<SF>(L, g, f);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int k0 = BACK ? 3 * c : c, k1 = BACK ? 3 * c + 1 : 3 + c, k2 = BACK ? 3 * c + 2 : 6 + c;
            ur[c] = qsel(q, U.re[k0], U.re[k1], U.re[k2]);
            ui[c] = qsel(q, U.im[k0], U.im[k1], U.im[k2]);
        }
    }
}

// the same for a two-row long link c * U
template <int SF, int GF, bool BACK>
__device__ __forceinline__ void lane_link12(const LinkRaw12<GF> &L, float g, float c, const QuadSel &q,
                                            float (&ur)[3], float (&ui)[3], float &f) {
    const Mat<float> U = hop_link12<SF>(L, g, c, f);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int k0 = BACK ? 3 * k : k, k1 = BACK ? 3 * k + 1 : 3 + k, k2 = BACK ? 3 * k + 2 : 6 + k;
        ur[k] = qsel(q, U.re[k0], U.re[k1], U.re[k2]);
        ui[k] = qsel(q, U.im[k0], U.im[k1], U.im[k2]);
    }
}

template <int GF, int SF, int NR, bool RED, int LR>
__device__ __forceinline__ void dslash_site_mfma(const DslashArgs &A, int s, bool valid, int rhs0, int li,
                                                 unsigned live, const float (&acoef)[NR], double (&red)[NR]) {
    const Geom &g = A.g;
    const size_t fs = A.field_stride;
    const size_t vh = (size_t)g.vh;
    const int p = A.parity, q = 1 - p;
    const size_t sub = (size_t)gauge_matrix_bytes(GF) * vh;
    const size_t lsub = LR == 12 ? (size_t)gauge_matrix_bytes12(GF) * vh : sub;
    const float gf = (float)A.gfat, gl = (float)A.glong, lc = (float)A.lcoef;
    const QuadSel qs{li == 0 || li == 3, li == 1};
    const int se = valid ? s : 0;                     // invalid lanes read site 0, results discarded
    const unsigned lv = valid ? live : 0u;
    // input column of each of the lane's right-hand sides; a column the lane
    // does not compute (every column of an invalid lane) reads valid memory
    // whose products reach only this lane's own, unstored, outputs
    const char *colp[NR];
#pragma unroll
    for (int m = 0; m < NR; m++)
        colp[m] = ((lv >> m) & 1u) ? A.in + (size_t)colmap(A, rhs0 + 4 * m + li) * fs : A.in;
    f32x4v acc_re[NR], acc_im[NR];
#pragma unroll
    for (int m = 0; m < NR; m++) {
        acc_re[m] = f32x4v{0.f, 0.f, 0.f, 0.f};
        acc_im[m] = f32x4v{0.f, 0.f, 0.f, 0.f};
    }
    const Nbrs n = neighbours(g, se, p);
#pragma unroll
    for (int h = 0; h < 16; h++) {
        const int ss = hop_spinor_site(n, h);
        const int ls = (h & 1) ? ss : se;
        const int lpar = (h & 1) ? q : p;
        const bool back = (h & 1) != 0;
        float ur[3], ui[3], f;
        if (LR == 12 && (h & 2)) {
            const LinkRaw12<GF> L = link_load12<GF>(A.lng + (size_t)(2 * (h >> 2) + lpar) * lsub, vh, ls);
            const float c = lc * (back ? n.lsb[h >> 2] : n.lsf[h >> 2]);
            if (back)
                lane_link12<SF, GF, true>(L, gl, c, qs, ur, ui, f);
            else
                lane_link12<SF, GF, false>(L, gl, c, qs, ur, ui, f);
        } else {
            const LinkRaw<GF> L = link_load<GF>(((h & 2) ? A.lng : A.fat) + (size_t)(2 * (h >> 2) + lpar) * sub, vh, ls);
            if (back)
                lane_link<SF, GF, true>(L, (h & 2) ? gl : gf, qs, ur, ui, f);
            else
                lane_link<SF, GF, false>(L, (h & 2) ? gl : gf, qs, ur, ui, f);
        }
        // backward hops add -U^dag y: with a site scale the sign goes into it
        // (U^dag applied to -y), otherwise into the link row
        constexpr bool ssign = spinor_scaled<SF>();
        const float fy = (back && ssign) ? -f : f;
        CVec<float> v[NR];
#pragma unroll
        for (int m = 0; m < NR; m++) v[m] = spin_decode<float>(spin_load<SF>(colp[m], vh, ss), fy);
        if (back && !ssign) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                ur[c] = -ur[c];
                ui[c] = -ui[c];
            }
        }
        // A for K index k (k < 3: Re of input colour k, k >= 3: Im of colour k - 3).
        // forward  U y:     Re row: ur yr - ui yi, Im row: ui yr + ur yi
        // backward U^dag y: Re row: ur yr + ui yi, Im row: ur yi - ui yr
        float a_re[6], a_im[6];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            a_re[c] = ur[c];
            a_re[3 + c] = back ? ui[c] : -ui[c];
            a_im[c] = back ? -ui[c] : ui[c];
            a_im[3 + c] = ur[c];
        }
#pragma unroll
        for (int k = 0; k < 6; k++) {
#pragma unroll
            for (int m = 0; m < NR; m++) {
                const float bk = k < 3 ? v[m].re[k] : v[m].im[k - 3];
                acc_re[m] = __builtin_amdgcn_mfma_f32_4x4x1f32(a_re[k], bk, acc_re[m], 0, 0, 0);
                acc_im[m] = __builtin_amdgcn_mfma_f32_4x4x1f32(a_im[k], bk, acc_im[m], 0, 0, 0);
            }
        }
    }
    if (!lv) return;
    CVec<float> acc[NR];
#pragma unroll
    for (int m = 0; m < NR; m++) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc[m].re[c] = acc_re[m][c];
            acc[m].im[c] = acc_im[m][c];
        }
    }
    site_epilogue<SF, float, NR, RED>(A, s, [&](int m) { return colmap(A, rhs0 + 4 * m + li); }, lv, acoef, acc, red);
}

// GUARD: launched inside a solver's block of iterations (may return at once);
// standalone applications use the unguarded instantiation.
// LR: 18 = long links stored in full, 12 = two rows + reconstruction
template <int GF, int SF, class R, int NR, int STAGE, bool RED, bool GUARD, int LR>
__global__ void __launch_bounds__(256) k_dslash(DslashArgs A, int rhs0, int rg, FastDiv drg, int sweep) {
    __shared__ double lds[64];
    if (GUARD && !A.guard.pass()) return;
    const Geom g = A.g;
    double red[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) red[j] = 0.0;
    // The lane's right-hand sides (rg divides blockDim, so a lane keeps its
    // group in every tile): rhs0 + j*rg + grp, one column of each group of rg
    // per lane, so that the live columns of a block (a prefix: the solvers
    // compact them) leave whole groups dead in every lane, whose arithmetic
    // the wave then skips.  Those at or beyond ncol (a block padded to a power
    // of two) and those marked inactive are neither read nor written.
    const int ncol = A.nrhs > 1 ? A.nrhs : 1;
    const int grp0 = (int)(threadIdx.x & (unsigned)(rg - 1));
    auto cofs = [&](int lg, int j) { return j * rg + lg; };
    unsigned live = 0;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const int c = rhs0 + cofs(grp0, j);
        if (colvalid(A, c, ncol) && (!A.cactive || A.cactive[colmap(A, c)])) live |= 1u << j;
    }
    // xpay coefficient of each of the lane's right-hand sides, read once
    R acoef[NR];
#pragma unroll
    for (int j = 0; j < NR; j++)
        acoef[j] = (A.acol && ((live >> j) & 1u)) ? (R)A.acol[colmap(A, rhs0 + cofs(grp0, j))] : (R)A.a;
    // Tiles of blockDim lanes.  sweep 0: XCD k (blocks b with b % 8 == k) sweeps
    // the contiguous tile range [k*ntile/8, (k+1)*ntile/8) in order, each of its
    // gridDim/8 blocks taking every (gridDim/8)-th tile.  sweep 1: block b takes
    // tiles b, b + gridDim, ...  sweep 2: XCD k owns the z-slab [Z k/8, Z (k+1)/8)
    // of every time slice; its tiles run through the slab slice by slice in t
    // order (a slab slice is zs * Y * X/2 consecutive checkerboard sites, padded
    // to whole tiles), each of its gridDim/8 blocks taking every (gridDim/8)-th
    // tile.  One tile per block when the grid covers the lattice, a persistent
    // grid-stride sweep otherwise.
    const int ntile = (int)(((long long)g.vh * rg + blockDim.x - 1) / blockDim.x);
    int tile0, tend, tstep;
    int zs0 = 0, slab = 0, tps = 1;
    if (sweep == 0) {
        const int xcd = blockIdx.x & 7;
        tile0 = (int)(((long long)ntile * xcd) >> 3) + (int)(blockIdx.x >> 3);
        tend = (int)(((long long)ntile * (xcd + 1)) >> 3);
        tstep = gridDim.x >> 3;
    } else if (sweep == 1) {
        tile0 = blockIdx.x;
        tend = ntile;
        tstep = gridDim.x;
    } else {
        const int xcd = blockIdx.x & 7;
        zs0 = (g.Z * xcd) >> 3;
        slab = (((g.Z * (xcd + 1)) >> 3) - zs0) * g.Y * g.X2;
        tps = (slab * rg + (int)blockDim.x - 1) / (int)blockDim.x;
        tile0 = blockIdx.x >> 3;
        tend = g.T * tps;
        tstep = gridDim.x >> 3;
    }
    for (int tile = tile0; tile < tend; tile += tstep) {
    int s, grp;
    bool inside;
    if (sweep == 2) {
        const int t = tile / tps;
        const int off = (tile - t * tps) * (int)blockDim.x + (int)threadIdx.x;
        const int sl = rg == 1 ? off : fdiv(off, drg);
        inside = sl < slab;
        s = (t * g.Z + zs0) * g.Y * g.X2 + sl;
        grp = off - sl * rg;
    } else {
        const int tid = tile * blockDim.x + threadIdx.x;
        s = rg == 1 ? tid : fdiv(tid, drg);
        grp = tid - s * rg;
        inside = s < g.vh;
    }
    if constexpr (STAGE == MFMA_STAGE) {
        // every lane takes part in the matrix instructions of its site's block
        dslash_site_mfma<GF, SF, NR, RED, LR>(A, s, inside, rhs0, grp, live, acoef, red);
    } else {
        if (inside && live) dslash_site<GF, SF, R, NR, STAGE, RED, LR>(A, s, rhs0 + grp, rg, live, acoef, red);
    }
    }
    if (RED) {
        // per right-hand side: sum over the lanes of the same group (lanes l with
        // l % rg == grp; rg is a power of two dividing 64), then over the waves
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            double v = red[j];
            for (int o = 32; o >= rg; o >>= 1) v += __shfl_xor(v, o, 64);
            red[j] = v;
        }
        if (lane < rg) {
#pragma unroll
            for (int j = 0; j < NR; j++) lds[w * rg * NR + cofs(lane, j)] = red[j];
        }
        __syncthreads();
        const int k = threadIdx.x;
        if (k < rg * NR && colvalid(A, rhs0 + k, ncol)) {
            double v = 0.0;
            for (int ww = 0; ww < nw; ww++) v += lds[ww * rg * NR + k];
            A.partial[(size_t)colmap(A, rhs0 + k) * A.pstride + blockIdx.x] = v;
        }
    }
}

// Several lattices in one launch (Sec. 1 "Block solvers": small problems filling
// the device together): block b belongs to the lattice l with boff[l] <= b <
// boff[l+1] and covers its sites (b - boff[l]) * MULTI_BLOCK + lane.
template <int GF, int SF, class R, int STAGE, int LR>
__global__ void __launch_bounds__(MULTI_BLOCK) k_dslash_multi(MultiArgs M) {
    int l = 0;
    while (l + 1 < M.n && (int)blockIdx.x >= M.boff[l + 1]) l++;
    const DslashArgs &A = M.a[l];
    const int s = ((int)blockIdx.x - M.boff[l]) * MULTI_BLOCK + (int)threadIdx.x;
    if (s >= A.g.vh) return;
    const R acoef[1] = {(R)A.a};
    double red[1] = {0.0};
    dslash_site<GF, SF, R, 1, STAGE, false, LR>(A, s, 0, 1, 1u, acoef, red);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int GF, int SF, class R>
hipError_t launch_multi(const MultiArgs &m, int long_recon, hipStream_t st) {
    const int nb = m.boff[m.n];
    if (long_recon != 12 && long_recon != 18) return hipErrorInvalidValue;
    if (long_recon == 12)
        hipLaunchKernelGGL((k_dslash_multi<GF, SF, R, 4, 12>), dim3(nb), dim3(MULTI_BLOCK), 0, st, m);
    else
        hipLaunchKernelGGL((k_dslash_multi<GF, SF, R, 4, 18>), dim3(nb), dim3(MULTI_BLOCK), 0, st, m);
    return hipGetLastError();
}

template <int GF, int SF, class R, int NR, int STAGE>
hipError_t launch_cfg(const DslashArgs &a, int rhs0, int rg, int block, int grid, int sweep, hipStream_t st,
                      int *nblocks) {
    const int nb = dslash_tile_blocks(a.g, DslashTile{NR, rg, STAGE, block, grid, sweep});
    if (nblocks) *nblocks = nb;
    const FastDiv drg = make_fastdiv((unsigned)rg);
    if (a.long_recon == 8) {
        if constexpr (NR == 1 && std::is_same<R, double>::value && (GF == GF_F64 || GF == GF_FIX32) &&
                      STAGE != MFMA_STAGE) {
            if (rg != 1) return hipErrorInvalidValue;
            if (a.red != RED_NONE)
                hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, true, true, 8>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
            else if (a.guard.stop)
                hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, false, true, 8>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
            else
                hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, false, false, 8>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (a.long_recon == 12) {
        if (a.red != RED_NONE)
            hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, true, true, 12>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
        else if (a.guard.stop)
            hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, false, true, 12>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
        else
            hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, false, false, 12>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
    } else {
        if (a.red != RED_NONE)
            hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, true, true, 18>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
        else if (a.guard.stop)
            hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, false, true, 18>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
        else
            hipLaunchKernelGGL((k_dslash<GF, SF, R, NR, STAGE, false, false, 18>), dim3(nb), dim3(block), 0, st, a, rhs0, rg, drg, sweep);
    }
    return hipGetLastError();
}

// one launch covering right-hand sides [rhs0, rhs0 + nr*rg) with the tile (nr, rg, stage);
// rg must be a power of two <= 16 and nr*rg <= 16 (the per-group reduction)
template <int GF, int SF, class R, bool BATCHED>
hipError_t launch_tile(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nblocks) {
    if (t.rg < 1 || t.rg > 16 || (t.rg & (t.rg - 1)) || t.nr * t.rg > 16 || (t.block != 128 && t.block != 256) ||
        t.grid < 0 || (t.grid & 7) || t.sweep < 0 || t.sweep > 2)
        return hipErrorInvalidValue;
    switch (t.nr * 100 + t.stage) {
    case 99: return launch_cfg<GF, SF, R, 1, -1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
    case 98: return launch_cfg<GF, SF, R, 1, -2>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
    case 101: return launch_cfg<GF, SF, R, 1, 1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
    case 102: return launch_cfg<GF, SF, R, 1, 2>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
    case 104: return launch_cfg<GF, SF, R, 1, 4>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
    case 108: return launch_cfg<GF, SF, R, 1, 8>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
    default: break;
    }
    if constexpr (BATCHED && std::is_same<R, float>::value) {
        if (t.stage == MFMA_STAGE) {
            if (t.rg != 4) return hipErrorInvalidValue;
            switch (t.nr) {
            case 1: return launch_cfg<GF, SF, R, 1, MFMA_STAGE>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
            case 2: return launch_cfg<GF, SF, R, 2, MFMA_STAGE>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
            case 4: return launch_cfg<GF, SF, R, 4, MFMA_STAGE>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
            default: return hipErrorInvalidValue;
            }
        }
    }
    if (BATCHED) {
        switch (t.nr * 100 + t.stage) {
        case 201: return launch_cfg<GF, SF, R, 2, 1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        case 401: return launch_cfg<GF, SF, R, 4, 1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        case 801: return launch_cfg<GF, SF, R, 8, 1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        case 199: return launch_cfg<GF, SF, R, 2, -1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        case 399: return launch_cfg<GF, SF, R, 4, -1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        case 799: return launch_cfg<GF, SF, R, 8, -1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        case 1601: return launch_cfg<GF, SF, R, 16, 1>(a, rhs0, t.rg, t.block, t.grid, t.sweep, st, nblocks);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace dsl
}  // namespace hisq
