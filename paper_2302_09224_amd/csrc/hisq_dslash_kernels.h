// hisq_dslash_kernels.h -- the even-odd HISQ Dslash kernels for gfx950
// (included once per precision triplet so the instantiations compile in
// parallel translation units).
//
// out(x) = sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^dag in(x-mu)
//                 + L_mu(x) in(x+3mu) - L_mu(x-3mu)^dag in(x-3mu) ]
// for the sites x of one parity (the stencil the paper benchmarks, Secs. 5.2-5.3).
//
// One lane per output site.  The kernel is bound by HBM bandwidth: every link
// matrix is read exactly once per application (non-temporal, it is not reused),
// while each input spinor is read by up to 16 neighbouring sites and must come
// from L2 / the MALL after its first use.  The XCD-aware block order keeps the
// +-3 neighbours of a contiguous site range inside one XCD's L2.  Storage is
// unpacked to IEEE registers, the 16 3x3 complex mat-vecs run in the compute
// precision of the triplet, and the result is packed again before the single
// coalesced store (Sec. 1: the bandwidth-bound stencil gives the computational
// budget for the unpack/pack work).  Optional epilogue: out = b*D(in) + a*x + c*y
// and a per-block partial of Re<x,out> or |out|^2 taken on the stored values,
// which fuses the solver's xpay and the first reduction of each CG step.
#pragma once
#include "hisq_internal.h"

namespace hisq {
namespace dsl {

template <int GF, int SF, class R>
__device__ __forceinline__ void hop4(CVec<R> &acc, const char *in, size_t vh, const char *fat_fwd,
                                     const char *fat_bwd, const char *lng_fwd, const char *lng_bwd, int s,
                                     int f1, int b1, int f3, int b3, R gf, R gl) {
    {
        Mat<R> U = GaugeIO<GF, R>::load(fat_fwd, vh, s, gf);
        CVec<R> v = SpinorIO<SF, R>::load(in, vh, f1);
        mv_add(acc, U, v);
    }
    {
        Mat<R> U = GaugeIO<GF, R>::load(fat_bwd, vh, b1, gf);
        CVec<R> v = SpinorIO<SF, R>::load(in, vh, b1);
        mdv_sub(acc, U, v);
    }
    {
        Mat<R> U = GaugeIO<GF, R>::load(lng_fwd, vh, s, gl);
        CVec<R> v = SpinorIO<SF, R>::load(in, vh, f3);
        mv_add(acc, U, v);
    }
    {
        Mat<R> U = GaugeIO<GF, R>::load(lng_bwd, vh, b3, gl);
        CVec<R> v = SpinorIO<SF, R>::load(in, vh, b3);
        mdv_sub(acc, U, v);
    }
}

// checkerboard indices of the +-1, +-3 neighbours of site s along each direction
struct Nbrs {
    int f1[4], b1[4], f3[4], b3[4];
};

__device__ __forceinline__ int wrap_add(int c, int h, int L) {
    int v = c + h;
    v -= (v >= L) ? L : 0;
    v += (v < 0) ? L : 0;
    return v;
}

__device__ __forceinline__ Nbrs neighbours(const Geom &g, int s, int parity) {
    const int xcb = s % g.X2;
    int r = s / g.X2;
    const int y = r % g.Y;
    r /= g.Y;
    const int z = r % g.Z;
    const int t = r / g.Z;
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
    return n;
}

template <int GF, int SF, class R, bool RED>
__global__ void __launch_bounds__(256) k_dslash(DslashArgs A) {
    __shared__ double lds[16];
    if (!A.guard.pass()) return;
    const Geom g = A.g;
    const int s = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    double red = 0.0;
    if (s < g.vh) {
        const size_t vh = (size_t)g.vh;
        const int p = A.parity, q = 1 - p;
        const size_t sub = (size_t)gauge_matrix_bytes(GF) * vh;
        const R gf = (R)A.gfat, gl = (R)A.glong;
        const Nbrs n = neighbours(g, s, p);
        CVec<R> acc;
        cvec_zero(acc);
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            hop4<GF, SF, R>(acc, A.in, vh, A.fat + (2 * mu + p) * sub, A.fat + (2 * mu + q) * sub,
                            A.lng + (2 * mu + p) * sub, A.lng + (2 * mu + q) * sub, s, n.f1[mu], n.b1[mu],
                            n.f3[mu], n.b3[mu], gf, gl);
        }
        const R b = (R)A.b;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc.re[c] *= b;
            acc.im[c] *= b;
        }
        CVec<R> xv;
        cvec_zero(xv);
        if (A.x) {
            xv = SpinorIO<SF, R>::load(A.x, vh, s);
            const R a = (R)A.a;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                acc.re[c] = fma(a, xv.re[c], acc.re[c]);
                acc.im[c] = fma(a, xv.im[c], acc.im[c]);
            }
        }
        if (A.y) {
            CVec<R> yv = SpinorIO<SF, R>::load(A.y, vh, s);
            const R cc = (R)A.c;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                acc.re[c] = fma(cc, yv.re[c], acc.re[c]);
                acc.im[c] = fma(cc, yv.im[c], acc.im[c]);
            }
        }
        CVec<R> o = SpinorIO<SF, R>::store(A.out, vh, s, acc);
        if (RED) {
            if (A.red == RED_DOT_X) {
#pragma unroll
                for (int c = 0; c < 3; c++) red += (double)xv.re[c] * (double)o.re[c] + (double)xv.im[c] * (double)o.im[c];
            } else {
#pragma unroll
                for (int c = 0; c < 3; c++) red += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
            }
        }
    }
    if (RED) {
        double v[1] = {red};
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) A.partial[blockIdx.x] = v[0];
    }
}

// Block of NR right-hand sides: each link matrix is loaded once and applied to
// all NR spinors of the block (Sec. 1, "Block solvers").  Fields j of in/out/x
// are at byte offset j*field_stride.  Partials: [block][rhs0 + j] with row
// length A.nrhs (the total number of right-hand sides).
template <int GF, int SF, class R, int NR, bool RED>
__global__ void __launch_bounds__(256) k_dslash_batched(DslashArgs A, int rhs0) {
    __shared__ double lds[4 * NR];
    if (!A.guard.pass()) return;
    const Geom g = A.g;
    const int s = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const size_t fs = A.field_stride;
    double red[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) red[j] = 0.0;
    if (s < g.vh) {
        const size_t vh = (size_t)g.vh;
        const int p = A.parity, q = 1 - p;
        const size_t sub = (size_t)gauge_matrix_bytes(GF) * vh;
        const R gf = (R)A.gfat, gl = (R)A.glong;
        const Nbrs n = neighbours(g, s, p);
        const char *in = A.in + (size_t)rhs0 * fs;
        CVec<R> acc[NR];
#pragma unroll
        for (int j = 0; j < NR; j++) cvec_zero(acc[j]);
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const char *fsub[2] = {A.fat + (2 * mu + p) * sub, A.fat + (2 * mu + q) * sub};
            const char *lsub[2] = {A.lng + (2 * mu + p) * sub, A.lng + (2 * mu + q) * sub};
            {
                Mat<R> U = GaugeIO<GF, R>::load(fsub[0], vh, s, gf);
#pragma unroll
                for (int j = 0; j < NR; j++) mv_add(acc[j], U, SpinorIO<SF, R>::load(in + j * fs, vh, n.f1[mu]));
            }
            {
                Mat<R> U = GaugeIO<GF, R>::load(fsub[1], vh, n.b1[mu], gf);
#pragma unroll
                for (int j = 0; j < NR; j++) mdv_sub(acc[j], U, SpinorIO<SF, R>::load(in + j * fs, vh, n.b1[mu]));
            }
            {
                Mat<R> U = GaugeIO<GF, R>::load(lsub[0], vh, s, gl);
#pragma unroll
                for (int j = 0; j < NR; j++) mv_add(acc[j], U, SpinorIO<SF, R>::load(in + j * fs, vh, n.f3[mu]));
            }
            {
                Mat<R> U = GaugeIO<GF, R>::load(lsub[1], vh, n.b3[mu], gl);
#pragma unroll
                for (int j = 0; j < NR; j++) mdv_sub(acc[j], U, SpinorIO<SF, R>::load(in + j * fs, vh, n.b3[mu]));
            }
        }
        const R b = (R)A.b, a = (R)A.a;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            const size_t off = (size_t)(rhs0 + j) * fs;
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
                CVec<R> yv = SpinorIO<SF, R>::load(A.y + off, vh, s);
                const R cc = (R)A.c;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[j].re[c] = fma(cc, yv.re[c], acc[j].re[c]);
                    acc[j].im[c] = fma(cc, yv.im[c], acc[j].im[c]);
                }
            }
            CVec<R> o = SpinorIO<SF, R>::store(A.out + off, vh, s, acc[j]);
            if (RED) {
                if (A.red == RED_DOT_X) {
#pragma unroll
                    for (int c = 0; c < 3; c++) red[j] += (double)xv.re[c] * (double)o.re[c] + (double)xv.im[c] * (double)o.im[c];
                } else {
#pragma unroll
                    for (int c = 0; c < 3; c++) red[j] += (double)o.re[c] * (double)o.re[c] + (double)o.im[c] * (double)o.im[c];
                }
            }
        }
    }
    if (RED) {
        block_sum<NR>(red, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < NR; j++) A.partial[(size_t)blockIdx.x * A.nrhs + rhs0 + j] = red[j];
        }
    }
}

template <int GF, int SF, class R>
hipError_t launch_one(const DslashArgs &a, int block, hipStream_t st) {
    const int nb = dslash_blocks(a.g.vh, block);
    if (a.red != RED_NONE)
        hipLaunchKernelGGL((k_dslash<GF, SF, R, true>), dim3(nb), dim3(block), 0, st, a);
    else
        hipLaunchKernelGGL((k_dslash<GF, SF, R, false>), dim3(nb), dim3(block), 0, st, a);
    return hipGetLastError();
}

template <int GF, int SF, class R, int NR>
hipError_t launch_batched_nr(const DslashArgs &a, int rhs0, int block, hipStream_t st) {
    const int nb = dslash_blocks(a.g.vh, block);
    if (a.red != RED_NONE)
        hipLaunchKernelGGL((k_dslash_batched<GF, SF, R, NR, true>), dim3(nb), dim3(block), 0, st, a, rhs0);
    else
        hipLaunchKernelGGL((k_dslash_batched<GF, SF, R, NR, false>), dim3(nb), dim3(block), 0, st, a, rhs0);
    return hipGetLastError();
}

template <int GF, int SF, class R>
hipError_t launch_batched(const DslashArgs &a, int block, hipStream_t st) {
    // split nrhs into blocks of 16, 8, 4, 2, 1 right-hand sides
    int done = 0;
    while (done < a.nrhs) {
        const int left = a.nrhs - done;
        hipError_t e;
        if (left >= 16) {
            e = launch_batched_nr<GF, SF, R, 16>(a, done, block, st);
            done += 16;
        } else if (left >= 8) {
            e = launch_batched_nr<GF, SF, R, 8>(a, done, block, st);
            done += 8;
        } else if (left >= 4) {
            e = launch_batched_nr<GF, SF, R, 4>(a, done, block, st);
            done += 4;
        } else if (left >= 2) {
            e = launch_batched_nr<GF, SF, R, 2>(a, done, block, st);
            done += 2;
        } else {
            e = launch_batched_nr<GF, SF, R, 1>(a, done, block, st);
            done += 1;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dsl
}  // namespace hisq
