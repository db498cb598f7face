// hisq_internal.h -- declarations shared by the translation units of libhisq
// (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hisq.h"
#include "hisq_device.h"

namespace hisq {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

hisq_status set_error(hisq_status st, const char *fmt, ...);

#define HISQ_TRY_HIP(call)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::hisq::set_error(HISQ_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), \
                                     __FILE__, __LINE__);                                       \
    } while (0)

#define HISQ_TRY(expr)                      \
    do {                                    \
        hisq_status s_ = (expr);            \
        if (s_ != HISQ_OK) return s_;       \
    } while (0)

// ---------------------------------------------------------------------------
// geometry and sizes
// ---------------------------------------------------------------------------

bool dims_ok(const int dims[4]);
Geom make_geom(const int dims[4]);
size_t spinor_field_bytes(size_t nsites, int sf);
size_t gauge_field_bytes(const int dims[4], int gf);
bool triplet_ok(const hisq_fmt &f);
// triplets whose Dslash is also built for blocks of right-hand sides
// (FIX32/INT30/FP32 is not: it exists only as a refinement option)
inline bool has_batched_form(const hisq_fmt &f) { return !(f.spinor == HISQ_SPINOR_INT30 && f.compute == 32); }
bool aligned16(const void *p);
// long-link storage a triplet can use: 18 and 12 reals always; the eight
// parameters only with FP64 arithmetic on F64 or FIX32 links (the rebuild
// amplifies the rounding of its arithmetic, which FP32 would make visible)
// and only for launches of one right-hand side per lane
// (any value but 12 and 8 reads as full storage, as in gauge_args)
inline bool recon_ok(const hisq_fmt &f, int long_recon, bool batched) {
    if (long_recon != HISQ_RECON_8) return true;
    return !batched && f.compute == 64 && (f.gauge == HISQ_GAUGE_F64 || f.gauge == HISQ_GAUGE_FIX32);
}

// ---------------------------------------------------------------------------
// Dslash
// ---------------------------------------------------------------------------

enum { RED_NONE = 0, RED_DOT_X = 1, RED_NORM = 2 };

struct DslashArgs {
    char *out;
    const char *in;
    const char *fat;
    const char *lng;
    const char *x;   // optional: out += a*x (format and parity of out)
    const char *y;   // optional: out += c*y
    double a, b, c;  // out = b*D(in) + a*x + c*y
    double gfat, glong;  // fixed-point decode steps (max/Q), unused for IEEE formats
    Geom g;
    int parity;      // parity of the output sites
    int red;         // RED_*: per-block partial of Re<x,out> or |out|^2 (values as stored)
    double *partial;
    Guard guard;
    size_t field_stride;  // batched: bytes between consecutive right-hand-side fields
    int nrhs;             // right-hand sides of the whole application (partials per block)
    size_t pstride;       // partial of right-hand side j, block b at partial[j*pstride + b]
    int long_recon;       // 18: long links stored in full; 12: two rows, L = lcoef * phase * SU(3);
                          // 8: eight parameters of |lcoef| * U (entries times glong are those of U)
    double lcoef;
    const double *acol;   // optional (device): coefficient a of right-hand side j is acol[j]
    const int *cactive;   // optional (device): right-hand side j is skipped (not read, not written) if !cactive[j]
    // cmapped: the launch's right-hand side k exists if bit k of cvalid is set and is field column
    // (cmap >> 4k) & 15 (fields, acol, cactive and partials are indexed by the field column);
    // otherwise right-hand side k < nrhs is column k
    int cmapped;
    unsigned cvalid;
    unsigned long long cmap;
};

// Launch shape of one Dslash launch: each lane accumulates `nr` right-hand
// sides of one site, `rg` adjacent lanes share a site (nr*rg right-hand sides
// per launch), the 16 hops are loaded in stages of `stage` (negative: stages
// of -stage hops, double-buffered, the next stage's loads issued before this
// stage's arithmetic; one right-hand side per lane only), `block` threads,
// `grid` blocks (0: one tile of lanes per block; otherwise a persistent grid,
// a multiple of 8, sweeping the tiles), `sweep` the order of the tiles: 0 =
// XCD k (blocks b with b % 8 == k) takes the k-th eighth of the lattice, 1 =
// consecutive tiles on consecutive blocks (the eight XCDs advance together,
// sharing the neighbours they read in the memory-side cache), 2 = XCD k owns
// the z-slab [Z k/8, Z (k+1)/8) of every time slice and walks its slabs in t
// order, each slab slice padded to whole tiles (the t and z neighbours of
// the sites an XCD works on stay within its own L2).
struct DslashTile {
    int nr, rg, stage, block, grid, sweep;
};

// A whole application: launches covering right-hand sides [rhs0[i], rhs0[i]+nr*rg)
// with tile[i], or tile_red[i] when the launch fuses a reduction (tuned apart
// for blocks of right-hand sides; the same tile for one right-hand side)
struct DslashPlan {
    int n;
    int rhs0[5];
    DslashTile tile[5];
    DslashTile tile_red[5];
};

// link pointers, fixed-point steps and long-link storage of a packed gauge
void gauge_args(DslashArgs &a, const hisq_gauge *g);

// Several independent lattices in one launch: lattice l owns blocks
// [boff[l], boff[l+1]) of MULTI_BLOCK lanes, one output site per lane.
constexpr int MULTI_BLOCK = 256;
struct MultiArgs {
    DslashArgs a[HISQ_MAX_LATTICES];
    int boff[HISQ_MAX_LATTICES + 1];
    int n;
};
static_assert(sizeof(MultiArgs) <= 4096, "kernel argument block too large");
hipError_t launch_dslash_multi(const MultiArgs &m, const hisq_fmt &f, int long_recon, hipStream_t st);
// link bytes one output site of a Dslash reads (8 fat + 8 long matrices)
inline double dslash_link_bytes(const hisq_gauge *g) {
    const int b18 = gauge_matrix_bytes(g->fmt);
    return 8.0 * b18 + 8.0 * (g->long_recon == HISQ_RECON_12 ? gauge_matrix_bytes12(g->fmt) : b18);
}

// blocks of a Dslash launch over n lanes (multiple of 8 for the XCD order)
int dslash_blocks(int n, int block);
// tiles of `block` lanes per slab slice of the z-slab order (the largest slab)
inline int slab_tiles(const Geom &g, int rg, int block) {
    const int slab = ((g.Z + 7) >> 3) * g.Y * g.X2;
    return (slab * rg + block - 1) / block;
}
// blocks a launch of tile t really uses (a persistent grid smaller than the
// tile count is used as is): the number of per-block partials it writes
inline int dslash_tile_blocks(const Geom &g, const DslashTile &t) {
    const int nb = t.sweep == 2 ? 8 * g.T * slab_tiles(g, t.rg, t.block) : dslash_blocks(g.vh * t.rg, t.block);
    return (t.grid > 0 && t.grid < nb) ? t.grid : nb;
}
// largest block count any plan for the lattice can use, per right-hand side
size_t dslash_max_blocks(const Geom &g);
// plan (autotuned on first use when a probe is given and the stream is not capturing)
DslashPlan dslash_plan(const hisq_fmt &f, const Geom &g, int nrhs, const DslashArgs *probe, hipStream_t st);
// the plan from the shapes already in the table (tuned, fixed or loaded), else
// the default shapes: never tunes, reads no file, allocates nothing
DslashPlan dslash_plan_lookup(const hisq_fmt &f, const Geom &g, int nrhs, int long_recon);
// launch a plan; nblocks[j] receives the block count used for right-hand side j
hipError_t launch_dslash(const DslashArgs &a, const hisq_fmt &f, const DslashPlan &plan, hipStream_t st,
                         int *nblocks);

// ---------------------------------------------------------------------------
// pack / unpack / reductions / solver BLAS
// ---------------------------------------------------------------------------

constexpr int BLAS_BLOCK = 256;
constexpr int BLAS_MAX_BLOCKS = 2048;  // 8 blocks per CU: the best streaming grid on MI355X
int blas_blocks(size_t n);  // grid of the streaming kernels (fixed cap, grid-stride)

hipError_t launch_spinor_pack(char *dst, const double *src, size_t n, int sf, hipStream_t st);
hipError_t launch_spinor_unpack(double *dst, const char *src, size_t n, int sf, hipStream_t st);
hipError_t launch_spinor_convert(char *dst, int sf_dst, const char *src, int sf_src, size_t n, hipStream_t st);
hipError_t launch_absmax(const double *src, size_t n, double *partial, int *nblocks, hipStream_t st);
hipError_t launch_reduce_max(const double *partial, int n, double *out, hipStream_t st);
hipError_t launch_gauge_pack(char *dst, const double *src, const Geom &g, int gf, const double *absmax,
                             hipStream_t st);
hipError_t launch_norm2_f64(const char *v, size_t n, double *partial, int *nblocks, hipStream_t st);
// two-row long links: per-block checks [min lambda, max lambda, #sigma+, #sigma-, defect, |Im det|/|det|, max|U|]
hipError_t launch_long_check(const double *src, const Geom &g, double *partial, int *nblocks, hipStream_t st);
hipError_t launch_gauge_pack12(char *dst, const double *src, const Geom &g, int gf, double coef, double umax,
                               hipStream_t st);
// eight parameters of W = L * phase * sign (sign = +-1, the sign of the long-link
// coefficient); fixed point scaled by lmax (the long field's max |real component|)
hipError_t launch_gauge_pack8(char *dst, const double *src, const Geom &g, int gf, double sign, double lmax,
                              hipStream_t st);

// solver control block, shared by the device scalar kernels and the host
struct SolverCtrl {
    int stop;        // guard value: block-local iteration index where the current block ends
    int reason;      // STOP_*
    int k;           // completed iterations
    int done;        // last true-residual check met the target
    int e_mask;      // multi-shift: shifts updated by this iteration's fused shift kernel
    int active_mask; // multi-shift: shifts still being updated
    int nshift;
    int pr;          // Polak-Ribiere beta
    int reproject;
    int maxiter;
    int breakdown;
    int pad0;
    double rho;      // |r|^2 of the iterated residual (stored values)
    double rho_prev; // |r|^2 before the last iteration's update (beta at a reliable update)
    double rho_new, gamma, pi, alpha, beta;
    double pa_re, pa_im, pb;   // p_new = pa*r + pb*p
    double rmax2;    // max |r|^2 since the last reliable update
    double b2, tol2, delta2;
    double r2_true;  // |b - A x|^2 at the last true-residual computation
    double alpha_prev, beta_prev;
    double floor2;   // multi-shift: sloppy floor^2
    // error-estimate trigger of the reliable updates (instead of the fixed delta)
    int ru_est;
    int pad1;
    double eps_s;       // unit roundoff of the sloppy format
    double anorm;       // running estimate of |A| (largest Rayleigh quotient pAp/|p|^2 seen)
    double dev, dev_init;   // estimated |r_true - r_iterated| and its value after the last update
    double rnorm_prev;      // |r| of the previous iteration
    double alpha_buf[HISQ_MAX_GRAD_BUFFER];
    double sh[HISQ_MAX_SHIFTS];       // shift_i - shift_0
    double tol2_i[HISQ_MAX_SHIFTS];
    double zeta[HISQ_MAX_SHIFTS], zeta_prev[HISQ_MAX_SHIFTS];
    double alpha_i[HISQ_MAX_SHIFTS], beta_i[HISQ_MAX_SHIFTS];
    double ai_buf[HISQ_MAX_GRAD_BUFFER][HISQ_MAX_SHIFTS];  // alpha_i of each iteration (slot) of the block
    double zb_buf[HISQ_MAX_GRAD_BUFFER][HISQ_MAX_SHIFTS];  // zeta_i after each iteration of the block
    double bb_buf[HISQ_MAX_GRAD_BUFFER][HISQ_MAX_SHIFTS];  // beta_i of each iteration of the block
    int eb_buf[HISQ_MAX_GRAD_BUFFER];   // shifts updated in each iteration of the block
    int rmb_buf[HISQ_MAX_GRAD_BUFFER];  // shifts that stopped in each iteration of the block
    int rm_mask;     // multi-shift: shifts that stopped in this iteration
    int shift_stop_k[HISQ_MAX_SHIFTS];
    // batched CG: per right-hand side scalars
    double brho[16], brho_prev[16], brho_new[16], bgamma[16], bpi[16], balpha[16], bbeta[16];
    double bpa_re[16], bpa_im[16], bpb[16], brmax2[16], bb2[16], br2_true[16];
    double balpha_buf[HISQ_MAX_GRAD_BUFFER][16];
    double bc[16], bnc[16];  // 4m^2 + shift of system j, and its negative
    double btol2[16];        // tol_j^2
    int bactive[16];   // 1 while right-hand side j is still iterating
    int bru[16];       // 1: right-hand side j takes part in the pending reliable update
    int bdone[16];
    int bk[16];
    int bwarm[16];     // 1: system j continues a given gradient vector at its first reliable update
};

enum { STOP_NONE = 0, STOP_RU = 1, STOP_CONV = 2, STOP_BREAKDOWN = 3, STOP_MAXITER = 4, STOP_MSDONE = 5 };
constexpr int STOP_NEVER = 0x3fffffff;

struct SpinorList {
    char *p[HISQ_MAX_SHIFTS];
};

// r = r - alpha*ap; partial (|r'|^2, Re<r', r>); r_copy (optional): the new r
// stored a second time there (the multi-shift ring of base residuals)
hipError_t launch_cg_axpy(char *r, const char *ap, const double *alpha, size_t n, int sf, int compute,
                          double *partial, Guard gd, hipStream_t st, char *r_copy = nullptr);
// p_dst = pa*r + pb*p_src, (pa, pb) from the control block
// (ppart: optional per-block |p_dst|^2 of the stored values)
hipError_t launch_cg_pupdate(char *p_dst, const char *r, const char *p_src, const SolverCtrl *ctrl, double *ppart,
                             size_t n, int sf, int compute, Guard gd, hipStream_t st);
// x64 += sum_i alpha_buf[i] p_i, i < count
hipError_t launch_flush_x(char *x64, const SpinorList &p, int count, const double *alpha_buf, size_t n,
                          int sf, int compute, Guard gd, hipStream_t st);
// r_s = pack(r64); partial (|r_s|^2, Re<r_s,p>, Im<r_s,p>, Re<r_s, r_old + alpha ap>)
hipError_t launch_ru_convert(char *r_s, const char *r64, const char *p, const char *ap, const double *alpha,
                             size_t n, int sf, int compute, double *partial, Guard gd, hipStream_t st);
// multi-shift, the shifted systems over a block of `count` iterations, all
// shifts in one launch: shift i's gradient vector p.p[i] holds p_i at the
// block's start; with the base residuals r_{k+1} of the block's iterations in
// rr.p[0..count) and the scalars recorded per iteration (ai_buf, zb_buf,
// bb_buf, eb_buf, rmb_buf), x_i += alpha_i p_i and p_i = zeta_i r + beta_i p_i
// are replayed in registers; p_i is stored again for the shifts still active
hipError_t launch_shift_replay(const SpinorList &x64, const SpinorList &p, const SpinorList &rr, const SolverCtrl *ctrl,
                               int nshift, size_t n, int count, int sf, int compute, Guard gd, hipStream_t st);
// grids of launch_shift_replay and launch_flush_x: blas_blocks(n) capped at
// the blocks of that kernel the device holds at once (a larger grid leaves
// blocks that start only after the first ones finish, on a device that is then
// mostly idle).  The occupancy is queried once per device and triplet; the
// solvers call these before they capture a graph.
int shift_replay_grid(size_t n, int sf, int compute);
int flush_x_grid(size_t n, int sf, int compute);

// batched versions (nrhs consecutive fields of `stride` bytes)
hipError_t launch_bcg_axpy(char *r, const char *ap, const SolverCtrl *ctrl, size_t n, size_t stride, int nrhs,
                           int sf, int compute, double *partial, Guard gd, hipStream_t st);
hipError_t launch_bcg_pupdate(char *p_dst, const char *r, const char *p_src, const SolverCtrl *ctrl, size_t n,
                              size_t stride, int nrhs, int sf, int compute, Guard gd, hipStream_t st);
hipError_t launch_bflush_x(char *x64, size_t stride64, const SpinorList &p, int count, const SolverCtrl *ctrl,
                           size_t n, size_t stride, int nrhs, int sf, int compute, Guard gd, hipStream_t st);
hipError_t launch_bru_convert(char *r_s, const char *r64, size_t stride64, const char *p, const char *ap,
                              const SolverCtrl *ctrl, size_t n, size_t stride, int nrhs, int sf, int compute,
                              double *partial, Guard gd, hipStream_t st);

// A block of independent CG solves (A + c_j) x_j = b_j sharing every Dslash
// (at most 16).  x_j, b_j: canonical FP64 [vh][3] device fields (b_j may
// repeat); x_j holds the initial guess on entry and the solution on exit.
struct BatchedJob {
    int nrhs;
    double *x[16];
    const double *b[16];
    double c[16];
    double tol[16];
    const hisq_gauge *g64, *gs;
    hisq_fmt fmt;
    hisq_solver_params q;   // validated
    void *ws;
    size_t ws_bytes;
    hipStream_t st;
    SolverCtrl *h;          // pinned host copy of the control block
    // optional: called once every launch shape the block can use has been
    // planned (tuned on first use) and before the first iteration, so that
    // work the caller starts there on another stream never overlaps a timing
    void (*after_setup)(void *);
    void *after_setup_ctx;
    // optional: system 0 continues the gradient vector p_warm (the job's
    // storage format) instead of restarting, with beta = |r|^2 / rho_warm at the
    // first reliable update (the multi-shift base system of Sec. 3.2)
    const char *p_warm;
    double rho_warm;
    // results
    long iters, rus, dsl, d64;
    double alg;
    int iters_j[16];
    double resid0_j[16], resid_j[16];
};
bool batched_fmt_ok(const hisq_fmt &f);
size_t batched_ws_bytes(const Geom &g, int nrhs, int sf, int nb);
hisq_status batched_run(BatchedJob &J);

// ---------------------------------------------------------------------------
// library-owned per-device scratch for one-shot calls (reductions)
// ---------------------------------------------------------------------------

struct LibScratch {
    double *dev;       // device doubles
    size_t ndev;
    double *host;      // pinned host doubles
};
hisq_status lib_scratch(LibScratch **out);

}  // namespace hisq
