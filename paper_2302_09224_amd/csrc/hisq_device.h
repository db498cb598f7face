// hisq_device.h -- device-side building blocks of libhisq for gfx950:
// storage codecs (unpack to IEEE registers, pack back), structure-of-arrays
// field addressing, lattice geometry, the XCD-aware block order and the
// deterministic wavefront/block reductions.
//
// Field layouts in HBM (all little-endian):
//  * A spinor field of n sites is stored as planes of 16-byte chunks: chunk k
//    of site s lives at byte k*16*n + 16*s; formats whose site record is not
//    a multiple of 16 bytes keep the last 8 bytes in a trailing plane at
//    K*16*n + 8*s.  Each lane of a wavefront therefore issues 16- or 8-byte
//    loads and a wavefront touches one contiguous 1 KiB (512 B) span.
//      F64    48 B: 3 planes (colour c: re, im)
//      F32    24 B: plane 0 (c0re c0im c1re c1im), tail (c2re c2im)
//      HALF16 16 B: plane 0 (q0|q1<<16, q2|q3<<16, q4|q5<<16, FP32 site max)
//      INT20  16 B: plane 0 (the four words of the 20-bit record)
//      INT30  24 B: plane 0 (words 0-3), tail (words 4-5)
//  * A link field holds 4*V matrices as 8 sub-fields (direction mu, parity p)
//    of Vh matrices each, sub-field index mu*2+p, site = checkerboard index;
//    within a sub-field the 18 reals (row-major, re/im interleaved) are cut
//    into 16-byte planes plus a tail plane:
//      F64   144 B: 9 planes (one complex element each)
//      F32    72 B: 4 planes (2 elements each) + 8-byte tail (element 8)
//      FIX16  36 B: 2 planes (4 elements each) + 4-byte tail (element 8)
//      FIX32  72 B: 4 planes + 8-byte tail
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hisq {

enum SpinorFmt { SF_F64 = 0, SF_F32 = 1, SF_HALF16 = 2, SF_INT20 = 3, SF_INT30 = 4, SF_INT24 = 5 };
enum GaugeFmt { GF_F64 = 0, GF_F32 = 1, GF_FIX16 = 2, GF_FIX32 = 3, GF_SX24 = 4 };

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// bytes per site record / per link matrix
__host__ __device__ constexpr int spinor_site_bytes(int sf) {
    return sf == SF_F64 ? 48 : (sf == SF_F32 || sf == SF_INT30) ? 24 : sf == SF_INT24 ? 20 : 16;
}
__host__ __device__ constexpr int gauge_matrix_bytes(int gf) {
    return gf == GF_F64 ? 144 : gf == GF_FIX16 ? 36 : gf == GF_SX24 ? 60 : 72;
}
// two rows (12 reals) of a long link stored for reconstruction
__host__ __device__ constexpr int gauge_matrix_bytes12(int gf) {
    return gf == GF_F64 ? 96 : gf == GF_FIX16 ? 24 : gf == GF_SX24 ? 40 : 48;
}
// eight parameters of a special unitary long link (F64 and FIX32 only)
__host__ __device__ constexpr int gauge_matrix_bytes8(int gf) {
    return gf == GF_F64 ? 64 : gf == GF_FIX32 ? 32 : 0;
}

// ---------------------------------------------------------------------------
// register types
// ---------------------------------------------------------------------------

template <class R> struct CVec {
    R re[3], im[3];
};

template <class R> struct Mat {
    R re[9], im[9];  // element (a,b) at 3a+b
};

template <class R> __device__ __forceinline__ void cvec_zero(CVec<R> &v) {
#pragma unroll
    for (int a = 0; a < 3; a++) v.re[a] = v.im[a] = R(0);
}

// acc += U v
template <class R> __device__ __forceinline__ void mv_add(CVec<R> &acc, const Mat<R> &U, const CVec<R> &v) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
        for (int b = 0; b < 3; b++) {
            acc.re[a] = fma(U.re[3 * a + b], v.re[b], acc.re[a]);
            acc.re[a] = fma(-U.im[3 * a + b], v.im[b], acc.re[a]);
            acc.im[a] = fma(U.re[3 * a + b], v.im[b], acc.im[a]);
            acc.im[a] = fma(U.im[3 * a + b], v.re[b], acc.im[a]);
        }
    }
}

// acc -= U^dagger v
template <class R> __device__ __forceinline__ void mdv_sub(CVec<R> &acc, const Mat<R> &U, const CVec<R> &v) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
        for (int b = 0; b < 3; b++) {
            // conj(U[b][a]) * v[b] = (ur - i ui)(vr + i vi)
            acc.re[a] = fma(-U.re[3 * b + a], v.re[b], acc.re[a]);
            acc.re[a] = fma(-U.im[3 * b + a], v.im[b], acc.re[a]);
            acc.im[a] = fma(-U.re[3 * b + a], v.im[b], acc.im[a]);
            acc.im[a] = fma(U.im[3 * b + a], v.re[b], acc.im[a]);
        }
    }
}

// ---------------------------------------------------------------------------
// raw loads / stores
// ---------------------------------------------------------------------------

template <class T> __device__ __forceinline__ T ld(const char *p) { return *reinterpret_cast<const T *>(p); }
// streaming load (links are read once per application): non-temporal hint
template <class T> __device__ __forceinline__ T ld_nt(const char *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const T *>(p));
}
template <class T> __device__ __forceinline__ void st(char *p, T v) { *reinterpret_cast<T *>(p) = v; }

__device__ __forceinline__ int sext16(unsigned u) { return (int)(short)(unsigned short)(u & 0xffffu); }
__device__ __forceinline__ int sext20(unsigned u) { return (int)((u & 0xfffffu) ^ 0x80000u) - 0x80000; }
__device__ __forceinline__ int sext30(unsigned u) { return (int)((u & 0x3fffffffu) ^ 0x20000000u) - 0x20000000; }

// 2^(e-127) for an 8-bit biased exponent e in [1,254]
__device__ __forceinline__ float pow2_f32(unsigned e) { return __uint_as_float(e << 23); }
// (a & m) | (b & ~m) in one instruction (the compiler splits the pattern
// into an AND and an AND-OR once it knows the zero bits of b)
__device__ __forceinline__ unsigned bfi32(unsigned m, unsigned a, unsigned b) {
    unsigned r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double pow2_f64(unsigned e) {
    return __longlong_as_double((long long)((unsigned long long)(e + 896u) << 52));
}

// ---------------------------------------------------------------------------
// spinor codecs
// ---------------------------------------------------------------------------

template <int SF, class R> struct SpinorIO;

template <class R> struct SpinorIO<SF_F64, R> {
    static __device__ __forceinline__ CVec<R> load(const char *base, size_t n, size_t s) {
        CVec<R> v;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            f64x2 w = ld<f64x2>(base + c * 16 * n + 16 * s);
            v.re[c] = (R)w.x;
            v.im[c] = (R)w.y;
        }
        return v;
    }
    // stores v; returns the value as stored (what a later load returns)
    static __device__ __forceinline__ CVec<R> store(char *base, size_t n, size_t s, const CVec<R> &v) {
        CVec<R> o;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            f64x2 w;
            w.x = (double)v.re[c];
            w.y = (double)v.im[c];
            st<f64x2>(base + c * 16 * n + 16 * s, w);
            o.re[c] = (R)w.x;
            o.im[c] = (R)w.y;
        }
        return o;
    }
};

template <class R> struct SpinorIO<SF_F32, R> {
    static __device__ __forceinline__ CVec<R> load(const char *base, size_t n, size_t s) {
        f32x4 a = ld<f32x4>(base + 16 * s);
        f32x2 b = ld<f32x2>(base + 16 * n + 8 * s);
        CVec<R> v;
        v.re[0] = a.x; v.im[0] = a.y; v.re[1] = a.z; v.im[1] = a.w; v.re[2] = b.x; v.im[2] = b.y;
        return v;
    }
    static __device__ __forceinline__ CVec<R> store(char *base, size_t n, size_t s, const CVec<R> &v) {
        f32x4 a;
        f32x2 b;
        a.x = (float)v.re[0]; a.y = (float)v.im[0]; a.z = (float)v.re[1]; a.w = (float)v.im[1];
        b.x = (float)v.re[2]; b.y = (float)v.im[2];
        st<f32x4>(base + 16 * s, a);
        st<f32x2>(base + 16 * n + 8 * s, b);
        CVec<R> o;
        o.re[0] = a.x; o.im[0] = a.y; o.re[1] = a.z; o.im[1] = a.w; o.re[2] = b.x; o.im[2] = b.y;
        return o;
    }
};

// QUDA half: q = rint(v * (32767/M)) with M the FP32 site max; v = q * (M/32767),
// the quotient rounded to FP32 once per site (an IEEE division), then one FP32
// product per component.  A site whose M is zero or whose 32767/M overflows
// stores zeros with M = 0.
template <class R> struct SpinorIO<SF_HALF16, R> {
    static __device__ __forceinline__ CVec<R> decode(u32x4 w) {
        return scaled(w, __uint_as_float(w.w) / 32767.0f);
    }
    // The stencil's decode: f, a factor folded into the site scale (the Dslash
    // folds link scales there, one multiply per site instead of one per link
    // element), and M * fl(1/32767) in place of the division: each component
    // differs from f times the exact decode above by a few FP32 roundings.
    static __device__ __forceinline__ CVec<R> decode(u32x4 w, float f) {
        return scaled(w, __uint_as_float(w.w) * (1.0f / 32767.0f) * f);
    }
    static __device__ __forceinline__ CVec<R> scaled(u32x4 w, float d) {
        CVec<R> v;
        v.re[0] = (float)sext16(w.x) * d; v.im[0] = (float)sext16(w.x >> 16) * d;
        v.re[1] = (float)sext16(w.y) * d; v.im[1] = (float)sext16(w.y >> 16) * d;
        v.re[2] = (float)sext16(w.z) * d; v.im[2] = (float)sext16(w.z >> 16) * d;
        return v;
    }
    static __device__ __forceinline__ u32x4 encode(const CVec<R> &vin) {
        float f[6] = {(float)vin.re[0], (float)vin.im[0], (float)vin.re[1],
                      (float)vin.im[1], (float)vin.re[2], (float)vin.im[2]};
        float m = fabsf(f[0]);
#pragma unroll
        for (int k = 1; k < 6; k++) m = fmaxf(m, fabsf(f[k]));
        float c = 32767.0f / m;
        u32x4 w;
        if (!(m > 0.0f) || !__builtin_isfinite(c)) {
            w.x = w.y = w.z = w.w = 0u;
            return w;
        }
        unsigned q[6];
#pragma unroll
        for (int k = 0; k < 6; k++) q[k] = (unsigned)(int)__builtin_rintf(f[k] * c);
        w.x = (q[0] & 0xffffu) | (q[1] << 16);
        w.y = (q[2] & 0xffffu) | (q[3] << 16);
        w.z = (q[4] & 0xffffu) | (q[5] << 16);
        w.w = __float_as_uint(m);
        return w;
    }
    static __device__ __forceinline__ CVec<R> load(const char *base, size_t, size_t s) {
        return decode(ld<u32x4>(base + 16 * s));
    }
    static __device__ __forceinline__ CVec<R> store(char *base, size_t, size_t s, const CVec<R> &v) {
        u32x4 w = encode(v);
        st<u32x4>(base + 16 * s, w);
        return decode(w);
    }
};

// 20-bit shared exponent (Appendix A): E = biased exponent of fl(M/(2^19-1)) + 1,
// q = rint(v * 2^(127-E)), v = q * 2^(E-127).
template <class R> struct SpinorIO<SF_INT20, R> {
    static __device__ __forceinline__ CVec<R> decode(u32x4 w, float f = 1.0f) {
        // A field inside one word is a signed bit-field extract.  A field split
        // over two words has its high bits at the top of the earlier word, so
        // inserting the next word's low bits just below them gives the field
        // times 2^12 as a signed 32-bit integer (exact in FP32); its scale is
        // sc * 2^-12 (exact for f = 1, a subnormal power of two for E < 13).
        // f: an extra factor folded into the site scale.
        const float sc = pow2_f32(w.w >> 24) * f;
        const float sl = sc * 0x1p-12f;
        CVec<R> v;
        v.re[0] = (float)((int)(w.x << 12) >> 12) * sc;
        v.im[0] = (float)(int)bfi32(0xfff00000u, w.x, w.y << 12) * sl;
        v.re[1] = (float)((int)(w.y << 4) >> 12) * sc;
        v.im[1] = (float)(int)bfi32(0xf0000000u, w.y, w.z << 12) * sl;
        v.re[2] = (float)(int)bfi32(0xffff0000u, w.z, w.w << 12) * sl;
        v.im[2] = (float)((int)(w.w << 8) >> 12) * sc;
        return v;
    }
    static __device__ __forceinline__ u32x4 encode(const CVec<R> &vin) {
        float f[6] = {(float)vin.re[0], (float)vin.im[0], (float)vin.re[1],
                      (float)vin.im[1], (float)vin.re[2], (float)vin.im[2]};
        float m = fabsf(f[0]);
#pragma unroll
        for (int k = 1; k < 6; k++) m = fmaxf(m, fabsf(f[k]));
        float t = m / 524287.0f;
        unsigned e = ((__float_as_uint(t) >> 23) & 0xffu) + 1u;
        e = e > 254u ? 254u : e;
        float inv = __uint_as_float((254u - e) << 23);
        unsigned u[6];
#pragma unroll
        for (int k = 0; k < 6; k++) u[k] = (unsigned)(int)__builtin_rintf(f[k] * inv) & 0xfffffu;
        u32x4 w;
        w.x = u[0] | ((u[1] >> 8) << 20);
        w.y = (u[1] & 0xffu) | (u[2] << 8) | ((u[3] >> 16) << 28);
        w.z = (u[3] & 0xffffu) | ((u[4] >> 4) << 16);
        w.w = (u[4] & 0xfu) | (u[5] << 4) | (e << 24);
        return w;
    }
    static __device__ __forceinline__ CVec<R> load(const char *base, size_t, size_t s) {
        return decode(ld<u32x4>(base + 16 * s));
    }
    static __device__ __forceinline__ CVec<R> store(char *base, size_t, size_t s, const CVec<R> &v) {
        u32x4 w = encode(v);
        st<u32x4>(base + 16 * s, w);
        return decode(w);
    }
};

// 30-bit shared exponent: the 20-bit rule with scale 2^29-1 in FP64.
template <class R> struct SpinorIO<SF_INT30, R> {
    static __device__ __forceinline__ CVec<R> decode(u32x4 a, u32x2 b, R f = R(1)) {
        const R sc = (R)pow2_f64((b.y >> 20) & 0xffu) * f;   // f: folded into the site scale
        CVec<R> v;
        v.re[0] = (R)sext30(a.x) * sc;
        v.im[0] = (R)sext30(((a.x >> 30) << 28) | (a.y & 0x0fffffffu)) * sc;
        v.re[1] = (R)sext30(((a.y >> 28) << 26) | (a.z & 0x03ffffffu)) * sc;
        v.im[1] = (R)sext30(((a.z >> 26) << 24) | (a.w & 0x00ffffffu)) * sc;
        v.re[2] = (R)sext30(((a.w >> 24) << 22) | (b.x & 0x003fffffu)) * sc;
        v.im[2] = (R)sext30(((b.x >> 22) << 20) | (b.y & 0x000fffffu)) * sc;
        return v;
    }
    static __device__ __forceinline__ void encode(const CVec<R> &vin, u32x4 &a, u32x2 &b) {
        double f[6] = {(double)vin.re[0], (double)vin.im[0], (double)vin.re[1],
                       (double)vin.im[1], (double)vin.re[2], (double)vin.im[2]};
        double m = fabs(f[0]);
#pragma unroll
        for (int k = 1; k < 6; k++) m = fmax(m, fabs(f[k]));
        double t = m / 536870911.0;
        int e = 1;
        if (t > 0.0) {
            int field = (int)((__double_as_longlong(t) >> 52) & 0x7ff);
            e = field - 895;  // (field - 1023) + 1 + 127
            e = e < 1 ? 1 : (e > 254 ? 254 : e);
        }
        double inv = pow2_f64((unsigned)(254 - e));  // 2^(127-e)
        unsigned u[6];
#pragma unroll
        for (int k = 0; k < 6; k++) u[k] = (unsigned)(int)__builtin_rint(f[k] * inv) & 0x3fffffffu;
        a.x = u[0] | ((u[1] >> 28) << 30);
        a.y = (u[1] & 0x0fffffffu) | ((u[2] >> 26) << 28);
        a.z = (u[2] & 0x03ffffffu) | ((u[3] >> 24) << 26);
        a.w = (u[3] & 0x00ffffffu) | ((u[4] >> 22) << 24);
        b.x = (u[4] & 0x003fffffu) | ((u[5] >> 20) << 22);
        b.y = (u[5] & 0x000fffffu) | ((unsigned)e << 20);
    }
    static __device__ __forceinline__ CVec<R> load(const char *base, size_t n, size_t s) {
        return decode(ld<u32x4>(base + 16 * s), ld<u32x2>(base + 16 * n + 8 * s));
    }
    static __device__ __forceinline__ CVec<R> store(char *base, size_t n, size_t s, const CVec<R> &v) {
        u32x4 a;
        u32x2 b;
        encode(v, a, b);
        st<u32x4>(base + 16 * s, a);
        st<u32x2>(base + 16 * n + 8 * s, b);
        return decode(a, b);
    }
};

// ---------------------------------------------------------------------------
// Shared-exponent format generator (Sec. 4: the 20- and 30-bit formats are two
// members of a family): six B-bit two's-complement components and an 8-bit
// biased exponent E, in the order re0, im0, re1, im1, re2, im2, E, allocated
// LSB-first in 32-bit words; a field that does not fit in the rest of a word
// puts its high bits at the top of that word and its low bits at the bottom of
// the next (the allocation of the appendix's 20-bit struct).  Encoding: M =
// max |component|, E = biased exponent of M / (2^(B-1) - 1) plus one, q =
// rint(v * 2^(127-E)), decode q * 2^(E-127); in FP32 for B <= 24, FP64 above
// (2^(B-1) - 1 must be exact).  B = 20 gives the INT20 words, B = 30 the INT30
// words; SF_INT24 (B = 24: 152 bits in five words) is generated.
// ---------------------------------------------------------------------------

template <int B> struct SxFmt {
    static_assert(B >= 9 && B <= 31, "component width");
    static constexpr int W = (6 * B + 8 + 31) / 32;
    static __host__ __device__ constexpr int width(int f) { return f < 6 ? B : 8; }
    static __host__ __device__ constexpr unsigned mask(int n) { return n >= 32 ? 0xffffffffu : ((1u << n) - 1u); }
    static __host__ __device__ __forceinline__ void put(unsigned (&w)[W], int f, unsigned v) {
        const int n = width(f), p = f * B, k = p >> 5, o = p & 31;
        if (o + n <= 32) {
            w[k] |= (v & mask(n)) << o;
        } else {
            const int l = n - (32 - o);     // low bits that go to the next word
            w[k] |= ((v & mask(n)) >> l) << o;
            w[k + 1] |= v & mask(l);
        }
    }
    static __host__ __device__ __forceinline__ unsigned get(const unsigned (&w)[W], int f) {
        const int n = width(f), p = f * B, k = p >> 5, o = p & 31;
        if (o + n <= 32) return (w[k] >> o) & mask(n);
        const int l = n - (32 - o);
        return ((w[k] >> o) << l) | (w[k + 1] & mask(l));
    }
    static __host__ __device__ __forceinline__ int sext(unsigned u) {
        const unsigned sign = 1u << (B - 1);
        return (int)((u & mask(B)) ^ sign) - (int)sign;
    }
};

template <int B, class R> struct SxCodec {
    typedef SxFmt<B> F;
    static __device__ __forceinline__ void encode(const CVec<R> &vin, unsigned (&w)[F::W]) {
#pragma unroll
        for (int k = 0; k < F::W; k++) w[k] = 0u;
        unsigned e, q[6];
        if (B <= 24) {
            const float f[6] = {(float)vin.re[0], (float)vin.im[0], (float)vin.re[1],
                                (float)vin.im[1], (float)vin.re[2], (float)vin.im[2]};
            float m = fabsf(f[0]);
#pragma unroll
            for (int k = 1; k < 6; k++) m = fmaxf(m, fabsf(f[k]));
            const float t = m / (float)((1 << (B - 1)) - 1);
            e = ((__float_as_uint(t) >> 23) & 0xffu) + 1u;
            e = e > 254u ? 254u : e;
            const float inv = __uint_as_float((254u - e) << 23);
#pragma unroll
            for (int k = 0; k < 6; k++) q[k] = (unsigned)(int)__builtin_rintf(f[k] * inv);
        } else {
            const double f[6] = {(double)vin.re[0], (double)vin.im[0], (double)vin.re[1],
                                 (double)vin.im[1], (double)vin.re[2], (double)vin.im[2]};
            double m = fabs(f[0]);
#pragma unroll
            for (int k = 1; k < 6; k++) m = fmax(m, fabs(f[k]));
            const double t = m / (double)((1u << (B - 1)) - 1u);
            int ei = 1;
            if (t > 0.0) {
                ei = (int)((__double_as_longlong(t) >> 52) & 0x7ff) - 895;
                ei = ei < 1 ? 1 : (ei > 254 ? 254 : ei);
            }
            e = (unsigned)ei;
            const double inv = pow2_f64(254u - e);
#pragma unroll
            for (int k = 0; k < 6; k++) q[k] = (unsigned)(int)__builtin_rint(f[k] * inv);
        }
#pragma unroll
        for (int k = 0; k < 6; k++) F::put(w, k, q[k]);
        F::put(w, 6, e);
    }
    // f: an extra factor folded into the site scale
    static __device__ __forceinline__ CVec<R> decode(const unsigned (&w)[F::W], R f = R(1)) {
        const unsigned e = F::get(w, 6);
        CVec<R> v;
        // FP32 products for B <= 24 in FP32 arithmetic; FP64 otherwise (B-bit
        // integers times a power of two are exact in both, so the values agree)
        if (B <= 24 && sizeof(R) == sizeof(float)) {
            const float sc = pow2_f32(e) * (float)f;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                v.re[c] = (R)((float)F::sext(F::get(w, 2 * c)) * sc);
                v.im[c] = (R)((float)F::sext(F::get(w, 2 * c + 1)) * sc);
            }
        } else {
            const double sc = pow2_f64(e) * (double)f;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                v.re[c] = (R)((double)F::sext(F::get(w, 2 * c)) * sc);
                v.im[c] = (R)((double)F::sext(F::get(w, 2 * c + 1)) * sc);
            }
        }
        return v;
    }
};

// SoA storage of a generated record of W words: words 0-3 in the 16-byte plane
// (16 s), the rest in a tail plane of (W-4)*4 bytes per site after it.
template <class R> struct SpinorIO<SF_INT24, R> {
    typedef SxFmt<24> F;
    static __device__ __forceinline__ CVec<R> load(const char *base, size_t n, size_t s) {
        const u32x4 a = ld<u32x4>(base + 16 * s);
        const unsigned w[F::W] = {a.x, a.y, a.z, a.w, ld<unsigned>(base + 16 * n + 4 * s)};
        return SxCodec<24, R>::decode(w);
    }
    static __device__ __forceinline__ CVec<R> store(char *base, size_t n, size_t s, const CVec<R> &v) {
        unsigned w[F::W];
        SxCodec<24, R>::encode(v, w);
        u32x4 a;
        a.x = w[0]; a.y = w[1]; a.z = w[2]; a.w = w[3];
        st<u32x4>(base + 16 * s, a);
        st<unsigned>(base + 16 * n + 4 * s, w[4]);
        return SxCodec<24, R>::decode(w);
    }
};

// ---------------------------------------------------------------------------
// lattice geometry (checkerboarded, X even)
// ---------------------------------------------------------------------------

// n / d for 0 <= n < 2^31 as (n * m) >> (31 + sh), sh = ceil(log2 d),
// m = ceil(2^(31+sh) / d) < 2^32: the rounding error n*(m - 2^(31+sh)/d) / 2^(31+sh)
// is below 2^-sh <= 1/d, so the quotient is exact.
struct FastDiv {
    unsigned m;
    int sh;
};

__host__ __device__ inline FastDiv make_fastdiv(unsigned d) {
    FastDiv f;
    f.sh = 0;
    while ((1u << f.sh) < d) f.sh++;
    f.m = (unsigned)(((1ull << (31 + f.sh)) + d - 1) / d);
    return f;
}

__device__ __forceinline__ int fdiv(int n, FastDiv f) {
    return (int)(((unsigned long long)(unsigned)n * f.m) >> (31 + f.sh));
}

struct Geom {
    int X, Y, Z, T;
    int X2;        // X/2
    int vh;        // sites per parity
    int sy, sz, st;  // checkerboard strides of +y, +z, +t: X2, X2*Y, X2*Y*Z
    FastDiv dX2, dY, dZ;
};

// ---------------------------------------------------------------------------
// launch order and reductions
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Remap so that every XCD sweeps one contiguous eighth of the sites in order:
// a site's +-1/+-3 neighbours are then read from the same XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nb) {
    return (nb & 7) ? bid : (bid & 7) * (nb >> 3) + (bid >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// deterministic block sum of NV doubles; result valid in thread 0
template <int NV> __device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) lds[w * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double s = 0.0;
            for (int j = 0; j < nw; j++) s += lds[j * NV + k];
            v[k] = s;
        }
    }
}

// Solver iteration guard: a kernel that belongs to iteration j of a block of
// iterations runs iff j < *stop (strict) or j <= *stop; the solver's scalar
// kernels lower *stop to end a block early (reliable update, convergence).
// *stop is written only by earlier kernels of the stream, never during a
// guarded dispatch, and is read first thing: a plain load the compiler turns
// into one scalar load per wave (the packet processor invalidates the scalar
// cache between dispatches), so the wave's vector loads do not queue behind a
// coherent vector load of the flag.
struct Guard {
    const int *stop;
    int j;
    int strict;
    __device__ __forceinline__ bool pass() const {
        if (!stop) return true;
        const int s = *stop;
        return strict ? (j < s) : (j <= s);
    }
};

}  // namespace hisq
