// hisq_solver.hip -- stabilised mixed-precision CG and multi-shift CG (Sec. 3).
//
// Design (MI355X): every scalar of the recurrences lives on the device in a
// SolverCtrl block and is produced by one-block "finalize" kernels that sum
// the per-block partials of the preceding fused kernel in a fixed order.  No
// iteration needs the host: the host enqueues blocks of `chunk` iterations
// (optionally as one captured hipGraph replayed per block) and polls the
// control block once per block.  A finalize kernel that decides to leave the
// loop (reliable update due, convergence candidate, multi-shift phase done,
// breakdown, iteration cap) lowers ctrl->stop, and every later kernel of the
// block sees its guard fail and returns at once.  The host then performs the
// reliable update (FP64 Dslash on the FP64 solution) and starts a new block.
//
// One CG iteration j of a block (slot jb = j mod N_b of the gradient buffer):
//   t     = D_oe p[jb]                                       (sloppy Dslash)
//   Ap    = c p[jb] - D_eo t,  partial Re<p,Ap>              (sloppy Dslash, fused xpay + dot)
//   alpha = rho / <p,Ap>                                     (finalize)
//   r    -= alpha Ap,  partial |r'|^2, Re<r',r>              (fused axpy + two dots)
//   beta  = (|r'|^2 - Re<r',r>) / |r|^2  (Polak-Ribiere, Sec. 3.1 item 3), RU / stop decisions
//   [multi-shift: x_i += alpha_i p_i, p_i = zeta_i r' + beta_i p_i for all shifts, one launch]
//   [x64 += sum_j alpha_j p_j every N_b iterations: buffered FP64 solution update, Sec. 3.1 item 1]
//   p[jb+1] = r' + beta p[jb]
// Reliable update (Sec. 3 and its footnote, delta = 0.1): flush the buffered
// gradients into x64, r64 = b - A x64 with the FP64 operator, r = pack(r64),
// re-project p against the new r (Sec. 3.1 item 2), then continue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "hisq_internal.h"

namespace hisq {

namespace {

// one block of 16 waves sums the block partials of a whole-lattice launch
// (tens of thousands at 48^3x96); each thread loads its strided share four
// entries at a time (all four in flight) and adds them in index order
constexpr int FIN_THREADS = 1024;

template <int NV>
__device__ __forceinline__ void fin_sums(const double *partial, int n, double (&v)[NV], double *lds) {
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = 0.0;
    const int step = blockDim.x;
    int b = threadIdx.x;
    for (; b + 3 * step < n; b += 4 * step) {
        double q[4][NV];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int k = 0; k < NV; k++) q[u][k] = partial[(size_t)(b + u * step) * NV + k];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int k = 0; k < NV; k++) v[k] += q[u][k];
    }
    for (; b < n; b += step) {
#pragma unroll
        for (int k = 0; k < NV; k++) v[k] += partial[(size_t)b * NV + k];
    }
    block_sum<NV>(v, lds);
}

__global__ void k_fin_b2(SolverCtrl *c, const double *partial, int n) {
    __shared__ double lds[FIN_THREADS / 64];
    double v[1];
    fin_sums<1>(partial, n, v, lds);
    if (threadIdx.x == 0) c->b2 = v[0];
}

// alpha = rho / <p, A p>
__global__ void k_fin_alpha(SolverCtrl *c, const double *partial, int n, int jb, Guard gd) {
    __shared__ double lds[FIN_THREADS / 64];
    if (!gd.pass()) return;
    double v[1];
    fin_sums<1>(partial, n, v, lds);
    if (threadIdx.x) return;
    const double pi = v[0];
    c->pi = pi;
    if (!(pi > 0.0) || !__builtin_isfinite(pi)) {
        c->stop = gd.j - 1;
        c->reason = STOP_BREAKDOWN;
        c->breakdown = 1;
        return;
    }
    const double a = c->rho / pi;
    c->alpha = a;
    c->alpha_buf[jb] = a;
}

// beta and the decisions of one iteration; multi-shift: zeta recurrences
__global__ void k_fin_beta(SolverCtrl *c, const double *partial, int n, Guard gd, int multishift, int jb,
                           const double *ppart, int npp) {
    __shared__ double lds[2 * (FIN_THREADS / 64)], lds2[FIN_THREADS / 64];
    if (!gd.pass()) return;
    double v[2];
    fin_sums<2>(partial, n, v, lds);
    double pv[1] = {0.0};   // |p_k|^2 from the update that produced p_k
    if (c->ru_est) fin_sums<1>(ppart, npp, pv, lds2);
    if (threadIdx.x) return;
    const double rn = v[0], g = v[1];
    const int k = c->k + 1;
    c->k = k;
    c->rho_new = rn;
    c->gamma = g;
    if (!__builtin_isfinite(rn) || !__builtin_isfinite(g)) {
        c->stop = gd.j;
        c->reason = STOP_BREAKDOWN;
        c->breakdown = 1;
        return;
    }
    const double rho = c->rho;
    const double beta = c->pr ? (rn - g) / rho : rn / rho;
    c->beta = beta;
    c->pa_re = 1.0;
    c->pa_im = 0.0;
    c->pb = beta;
    int reason = STOP_NONE;
    if (multishift) {
        const double a = c->alpha, ap = c->alpha_prev, bp = c->beta_prev;
        int amask = c->active_mask, emask = 0, rm = 0;
        for (int i = 1; i < c->nshift; i++) {
            if (!((amask >> i) & 1)) continue;
            const double z = c->zeta[i], zp = c->zeta_prev[i], s = c->sh[i];
            const double zn = z * zp * ap / (ap * zp * (1.0 + a * s) + a * bp * (zp - z));
            const double ratio = zn / z;
            c->alpha_i[i] = a * ratio;
            c->ai_buf[jb][i] = a * ratio;
            c->beta_i[i] = beta * ratio * ratio;
            c->zb_buf[jb][i] = zn;
            c->bb_buf[jb][i] = beta * ratio * ratio;
            c->zeta_prev[i] = z;
            c->zeta[i] = zn;
            emask |= 1 << i;
            if (zn * zn * rn <= fmax(c->tol2_i[i], c->floor2) * c->b2) {
                amask &= ~(1 << i);
                rm |= 1 << i;
                c->shift_stop_k[i] = k;
            }
        }
        c->e_mask = emask;
        c->rm_mask = rm;
        c->eb_buf[jb] = emask;
        c->rmb_buf[jb] = rm;
        c->active_mask = amask;
        c->alpha_prev = a;
        c->beta_prev = beta;
        if ((amask & ~1) == 0) reason = STOP_MSDONE;
    }
    c->rmax2 = fmax(c->rmax2, rn);
    bool ru;
    if (c->ru_est) {
        // Error estimate of the iterated residual (residual replacement in the manner of
        // van der Vorst and Ye): each sloppy update r -= alpha A p makes an error of about
        // eps_s (|r| + |alpha| |A| |p|); the errors of successive iterations are independent,
        // so they are accumulated in quadrature.  A reliable update is due when the estimate
        // crosses sqrt(eps_s) |r| from below and has grown past 1.1x its value after the
        // previous update.
        const double rnorm = sqrt(rn);
        if (pv[0] > 0.0) c->anorm = fmax(c->anorm, c->pi / pv[0]);
        const double e = c->eps_s * (rnorm + fabs(c->alpha) * c->anorm * sqrt(pv[0]));
        const double dnew = sqrt(c->dev * c->dev + e * e);
        const double th = sqrt(c->eps_s);
        ru = c->dev <= th * c->rnorm_prev && dnew > th * rnorm && dnew > 1.1 * c->dev_init;
        c->dev = dnew;
        c->rnorm_prev = rnorm;
    } else {
        ru = c->delta2 > 0.0 && rn < c->delta2 * c->rmax2;
    }
    if (reason == STOP_NONE) {
        if (ru)
            reason = STOP_RU;
        else if (!multishift && rn <= c->tol2 * c->b2)
            reason = STOP_CONV;
    }
    if (reason == STOP_NONE && k >= c->maxiter) reason = STOP_MAXITER;
    c->rho_prev = rho;
    c->rho = rn;
    if (reason != STOP_NONE) {
        c->reason = reason;
        c->stop = gd.j;
    }
}

// |b - A x|^2 from the FP64 operator; done when below tol^2 |b|^2
__global__ void k_fin_ru_check(SolverCtrl *c, const double *partial, int n) {
    __shared__ double lds[FIN_THREADS / 64];
    double v[1];
    fin_sums<1>(partial, n, v, lds);
    if (threadIdx.x) return;
    const double r2 = v[0];
    c->r2_true = r2;
    if (!__builtin_isfinite(r2)) {
        c->breakdown = 1;
        c->done = 0;
        c->stop = -1;
        return;
    }
    const int done = r2 <= c->tol2 * c->b2;
    c->done = done;
    c->stop = done ? -1 : STOP_NEVER;
}

// after r = pack(b - A x): new rho, re-projection and beta of the next p update.
// mode 0: reliable update inside CG (Polak-Ribiere against the previous iterated residual)
// mode 1: fresh start (p = r)
// mode 2: continuation of a gradient vector from another solve (Fletcher-Reeves against rho_prev)
__global__ void k_fin_ru_finish(SolverCtrl *c, const double *partial, int n, int mode, Guard gd) {
    __shared__ double lds[4 * (FIN_THREADS / 64)];
    if (!gd.pass()) return;
    double v[4];
    fin_sums<4>(partial, n, v, lds);
    if (threadIdx.x) return;
    const double rho = v[0];
    double beta = 0.0, cr = 0.0, ci = 0.0;
    if (mode != 1) {
        if (c->reproject && rho > 0.0) {
            cr = v[1] / rho;  // <r,p>/<r,r>: p <- p - (<r,p>/<r,r>) r
            ci = v[2] / rho;
        }
        beta = (mode == 0 && c->pr) ? (rho - v[3]) / c->rho_prev : rho / c->rho_prev;
    }
    c->pa_re = 1.0 - beta * cr;
    c->pa_im = -beta * ci;
    c->pb = beta;
    c->beta = beta;
    c->rho = rho;
    c->rmax2 = rho;
    c->dev = c->dev_init = c->eps_s * sqrt(rho);   // rounding of the freshly stored residual
    c->rnorm_prev = sqrt(rho);
    c->reason = STOP_NONE;
    c->stop = STOP_NEVER;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// library-owned stream (default priority) and pinned mirror of the control block
// ---------------------------------------------------------------------------

struct DevState {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    SolverCtrl *host_ctrl = nullptr;
    // the second stream of the multi-shift refinement (shifted systems batched
    // while the base system is refined on `stream`)
    hipStream_t stream2 = nullptr;
    hipEvent_t ev2 = nullptr;
    SolverCtrl *host_ctrl2 = nullptr;
    std::mutex mu;
};

DevState g_dev[64];

hisq_status dev_state(DevState **out) {
    int d = 0;
    HISQ_TRY_HIP(hipGetDevice(&d));
    if (d < 0 || d >= 64) return set_error(HISQ_EINVAL, "device index %d out of range", d);
    DevState &s = g_dev[d];
    if (!s.stream) {
        HISQ_TRY_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
        HISQ_TRY_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
        HISQ_TRY_HIP(hipHostMalloc((void **)&s.host_ctrl, sizeof(SolverCtrl), hipHostMallocDefault));
        HISQ_TRY_HIP(hipStreamCreateWithFlags(&s.stream2, hipStreamNonBlocking));
        HISQ_TRY_HIP(hipEventCreateWithFlags(&s.ev2, hipEventDisableTiming));
        HISQ_TRY_HIP(hipHostMalloc((void **)&s.host_ctrl2, sizeof(SolverCtrl), hipHostMallocDefault));
    }
    *out = &s;
    return HISQ_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

struct Carver {
    size_t off = 0;
    char *base = nullptr;
    char *take(size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    }
};

size_t partial_doubles(const Geom &g, int nrhs) {
    const size_t a = dslash_max_blocks(g) * std::max(1, nrhs);
    const size_t b = (size_t)4096 * 4 * std::max(1, nrhs);
    return std::max(a, b);
}

struct CgBuffers {
    SolverCtrl *ctrl;
    double *partial;
    double *ppart;                     // per-block |p|^2 of the last p update
    char *x64, *b64, *r64, *t64;
    char *rs, *aps, *ts;
    char *p[HISQ_MAX_GRAD_BUFFER];
    char *pconv;                       // multi-shift: base gradient vector in the refinement format
    char *xs[HISQ_MAX_SHIFTS];         // multi-shift: FP64 shifted solutions (index >= 1)
    char *ps[HISQ_MAX_SHIFTS];         // multi-shift: shifted gradient vectors at the block's start (index >= 1)
    char *rr[HISQ_MAX_GRAD_BUFFER];    // multi-shift: the base residuals of the block's iterations
};

// sloppy_bytes: bytes/site of the largest sloppy format used; ms_bytes: of the
// multi-shift gradient vectors (0: not a multi-shift solve)
size_t carve_cg(CgBuffers *b, char *base, const Geom &g, int sloppy_bytes, int nb, int nshift, int ms_bytes,
                int ref_bytes) {
    Carver cv;
    cv.base = base;
    const size_t vh = g.vh;
    CgBuffers tmp;
    CgBuffers &B = b ? *b : tmp;
    B.ctrl = (SolverCtrl *)cv.take(sizeof(SolverCtrl));
    B.partial = (double *)cv.take(partial_doubles(g, 1) * sizeof(double));
    B.ppart = (double *)cv.take((size_t)BLAS_MAX_BLOCKS * sizeof(double));
    B.x64 = cv.take(48 * vh);
    B.b64 = cv.take(48 * vh);
    B.r64 = cv.take(48 * vh);
    B.t64 = cv.take(48 * vh);
    B.rs = cv.take(sloppy_bytes * vh);
    B.aps = cv.take(sloppy_bytes * vh);
    B.ts = cv.take(sloppy_bytes * vh);
    for (int i = 0; i < HISQ_MAX_GRAD_BUFFER; i++) B.p[i] = i < nb ? cv.take(sloppy_bytes * vh) : nullptr;
    B.pconv = nullptr;
    for (int i = 0; i < HISQ_MAX_SHIFTS; i++) B.xs[i] = B.ps[i] = nullptr;
    for (int i = 0; i < HISQ_MAX_GRAD_BUFFER; i++) B.rr[i] = nullptr;
    if (ms_bytes > 0) {
        B.pconv = cv.take(ref_bytes * vh);
        for (int i = 1; i < nshift; i++) {
            B.xs[i] = cv.take(48 * vh);
            B.ps[i] = cv.take((size_t)ms_bytes * vh);
        }
        if (nshift > 1)
            for (int q = 0; q < nb; q++) B.rr[q] = cv.take((size_t)ms_bytes * vh);
    }
    return cv.off;
}

int sloppy_floor_bits(int sf) {
    switch (sf) {
    case SF_F64: return 52;
    case SF_F32: return 24;
    case SF_HALF16: return 15;
    case SF_INT20: return 19;
    case SF_INT30: return 29;
    case SF_INT24: return 23;
    }
    return 24;
}

// ---------------------------------------------------------------------------
// one CG (or multi-shift) run on prepared buffers
// ---------------------------------------------------------------------------

struct Run {
    Geom g;
    size_t vh;
    hisq_fmt fmt;              // sloppy triplet
    const hisq_gauge *g64, *gs;
    double c;                  // 4m^2 + shift of the system being iterated
    int nb, chunk;
    bool graph;
    bool multishift;
    int nshift;
    CgBuffers *B;
    hipStream_t st;
    DevState *ds;
    // counters
    long dslash_sloppy = 0, dslash_f64 = 0, rus = 0, iters = 0;
    double alg_bytes = 0.0;
    int last_slot = 0;         // slot of the current gradient vector when the run ended
    hipGraphExec_t exec = nullptr;
    DslashPlan plan_s{}, plan_64{};
    int nb_s = 0, nb_64 = 0;

    // launch shapes of the sloppy and FP64 Dslash (autotuned on first use, outside capture)
    void setup_plans() {
        const hisq_fmt f64 = {HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64};
        DslashArgs ps = dargs(gs, B->ts, B->rs, 1);
        plan_s = dslash_plan(fmt, g, 1, &ps, st);
        nb_s = dslash_tile_blocks(g, plan_s.tile[0]);
        DslashArgs p64 = dargs(g64, B->t64, B->x64, 1);
        plan_64 = dslash_plan(f64, g, 1, &p64, st);
        nb_64 = dslash_tile_blocks(g, plan_64.tile[0]);
        // occupancy queries of the capped-grid kernels, before any capture
        (void)flush_x_grid(vh, fmt.spinor, fmt.compute);
        if (multishift) (void)shift_replay_grid(vh, fmt.spinor, fmt.compute);
    }

    DslashArgs dargs(const hisq_gauge *gg, char *out, const char *in, int parity) const {
        DslashArgs a;
        memset(&a, 0, sizeof(a));
        a.out = out;
        a.in = in;
        a.fat = (const char *)gg->fat;
        a.lng = (const char *)gg->lng;
        a.b = 1.0;
        a.g = g;
        a.parity = parity;
        a.red = RED_NONE;
        a.nrhs = 1;
        gauge_args(a, gg);
        return a;
    }

    hisq_status enq_iteration(int j) {
        const int jb = j % nb, jn = (j + 1) % nb;
        SolverCtrl *c = B->ctrl;
        const Guard gns{&c->stop, j, 0}, gs_{&c->stop, j, 1};
        DslashArgs A = dargs(gs, B->ts, B->p[jb], 1);
        A.guard = gns;
        HISQ_TRY_HIP(launch_dslash(A, fmt, plan_s, st, nullptr));
        DslashArgs Bk = dargs(gs, B->aps, B->ts, 0);
        Bk.b = -1.0;
        Bk.x = B->p[jb];
        Bk.a = c_;
        Bk.red = RED_DOT_X;
        Bk.partial = B->partial;
        Bk.guard = gns;
        HISQ_TRY_HIP(launch_dslash(Bk, fmt, plan_s, st, nullptr));
        hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(FIN_THREADS), 0, st, c, B->partial,
                           nb_s, jb, gns);
        HISQ_TRY_HIP(hipGetLastError());
        HISQ_TRY_HIP(launch_cg_axpy(B->rs, B->aps, &c->alpha, vh, fmt.spinor, fmt.compute, B->partial, gns, st,
                                    multishift ? B->rr[jb] : nullptr));
        hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(FIN_THREADS), 0, st, c, B->partial, blas_blocks(vh), gns,
                           multishift ? 1 : 0, jb, B->ppart, blas_blocks(vh));
        HISQ_TRY_HIP(hipGetLastError());
        if (multishift && jb == nb - 1) HISQ_TRY(enq_shift_replay(nb, gns));
        if (jb == nb - 1) {
            SpinorList pl;
            for (int i = 0; i < HISQ_MAX_SHIFTS; i++) pl.p[i] = i < nb ? B->p[i] : nullptr;
            HISQ_TRY_HIP(launch_flush_x(B->x64, pl, nb, c->alpha_buf, vh, fmt.spinor, fmt.compute, gs_, st));
        }
        HISQ_TRY_HIP(launch_cg_pupdate(B->p[jn], B->rs, B->p[jb], c, B->ppart, vh, fmt.spinor, fmt.compute, gs_, st));
        return HISQ_OK;
    }
    double c_ = 0.0;

    // bytes between the gradient slots of one shift's ring
    // the shifted systems' updates of the block's first `count` iterations
    hisq_status enq_shift_replay(int count, Guard gd) {
        SpinorList xl, pl, rl;
        for (int i = 0; i < HISQ_MAX_SHIFTS; i++) {
            xl.p[i] = B->xs[i];
            pl.p[i] = B->ps[i];
            rl.p[i] = i < HISQ_MAX_GRAD_BUFFER ? B->rr[i] : nullptr;
        }
        HISQ_TRY_HIP(launch_shift_replay(xl, pl, rl, B->ctrl, nshift, vh, count, fmt.spinor, fmt.compute, gd, st));
        return HISQ_OK;
    }

    // a block ended early at slot jb (reliable update, end of the phase): the
    // shifted systems take the block's iterations so far, and like the base
    // restart at slot 0
    hisq_status realign_shifts(int jb) {
        if (!multishift || jb == nb - 1) return HISQ_OK;
        return enq_shift_replay(jb + 1, Guard{nullptr, 0, 0});
    }

    // r64 = b - (c x64 - D_eo D_oe x64), |r64|^2 -> done flag (FP64 operator)
    hisq_status enq_true_residual() {
        const hisq_fmt f64 = {HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64};
        DslashArgs A = dargs(g64, B->t64, B->x64, 1);
        HISQ_TRY_HIP(launch_dslash(A, f64, plan_64, st, nullptr));
        DslashArgs Bk = dargs(g64, B->r64, B->t64, 0);
        Bk.b = 1.0;
        Bk.x = B->x64;
        Bk.a = -c_;
        Bk.y = B->b64;
        Bk.c = 1.0;
        Bk.red = RED_NORM;
        Bk.partial = B->partial;
        HISQ_TRY_HIP(launch_dslash(Bk, f64, plan_64, st, nullptr));
        hipLaunchKernelGGL(k_fin_ru_check, dim3(1), dim3(FIN_THREADS), 0, st, B->ctrl, B->partial,
                           nb_64);
        HISQ_TRY_HIP(hipGetLastError());
        dslash_f64 += 2;
        alg_bytes += 2.0 * vh * (dslash_link_bytes(g64) + 2 * 48) + 2.0 * vh * 48;
        return HISQ_OK;
    }

    // flush `count` buffered gradients, true residual, repack r, re-project p
    // and write the next gradient vector into slot 0.
    hisq_status enq_reliable(int mode, int count, const char *p_src) {
        SolverCtrl *c = B->ctrl;
        if (count > 0) {
            SpinorList pl;
            for (int i = 0; i < HISQ_MAX_SHIFTS; i++) pl.p[i] = i < nb ? B->p[i] : nullptr;
            HISQ_TRY_HIP(launch_flush_x(B->x64, pl, count, c->alpha_buf, vh, fmt.spinor, fmt.compute, Guard{nullptr, 0, 0}, st));
            alg_bytes += vh * (count * (double)spinor_site_bytes(fmt.spinor) + 96.0);
        }
        HISQ_TRY(enq_true_residual());
        const Guard g0{&c->stop, 0, 0};
        HISQ_TRY_HIP(launch_ru_convert(B->rs, B->r64, mode == 1 ? nullptr : p_src, mode == 0 ? B->aps : nullptr,
                                       &c->alpha, vh, fmt.spinor, fmt.compute, B->partial, g0, st));
        hipLaunchKernelGGL(k_fin_ru_finish, dim3(1), dim3(FIN_THREADS), 0, st, c, B->partial, blas_blocks(vh), mode, g0);
        HISQ_TRY_HIP(hipGetLastError());
        HISQ_TRY_HIP(launch_cg_pupdate(B->p[0], B->rs, mode == 1 ? B->rs : p_src, c, B->ppart, vh, fmt.spinor,
                                       fmt.compute, g0, st));
        const double bs = spinor_site_bytes(fmt.spinor);
        alg_bytes += vh * (48.0 + 5 * bs) + vh * 3 * bs;
        return HISQ_OK;
    }

    hisq_status read_ctrl(SolverCtrl *h) {
        HISQ_TRY_HIP(hipMemcpyAsync(h, B->ctrl, sizeof(SolverCtrl), hipMemcpyDeviceToHost, st));
        HISQ_TRY_HIP(hipStreamSynchronize(st));
        return HISQ_OK;
    }

    hisq_status enq_chunk() {
        if (graph) {
            if (!exec) {
                hipGraph_t gr = nullptr;
                HISQ_TRY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                hisq_status s = HISQ_OK;
                for (int j = 0; j < chunk && s == HISQ_OK; j++) s = enq_iteration(j);
                hipError_t e = hipStreamEndCapture(st, &gr);
                if (s != HISQ_OK) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return s;
                }
                HISQ_TRY_HIP(e);
                e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                HISQ_TRY_HIP(e);
            }
            HISQ_TRY_HIP(hipGraphLaunch(exec, st));
            return HISQ_OK;
        }
        for (int j = 0; j < chunk; j++) HISQ_TRY(enq_iteration(j));
        return HISQ_OK;
    }

    double iter_bytes() const {
        const double bs = spinor_site_bytes(fmt.spinor), bl = dslash_link_bytes(gs);
        double it = 2.0 * (bl + 2.0 * bs) + bs         // two Dslash + xpay operand
                    + 3.0 * bs                           // r update
                    + 3.0 * bs                           // p update
                    + (nb * bs + 96.0) / nb;             // buffered FP64 solution update
        return it * vh;
    }

    // Iterate until the true residual meets tol (returns OK), or the
    // multi-shift phase ends (OK, *ms_done = 1), or an error.
    hisq_status iterate(SolverCtrl *h, int *ms_done) {
        if (ms_done) *ms_done = 0;
        long k0 = h->k;
        for (;;) {
            HISQ_TRY(enq_chunk());
            HISQ_TRY(read_ctrl(h));
            const long dk = h->k - k0;
            k0 = h->k;
            iters += dk;
            dslash_sloppy += 2 * dk;
            alg_bytes += dk * iter_bytes();
            if (multishift) {
                // the base residual written to the ring and read back once per block; per
                // updated shift, once per block of N_b iterations: its gradient vector read
                // and written and its FP64 solution read and written
                const double bs = spinor_site_bytes(fmt.spinor);
                const int ne = __builtin_popcount((unsigned)h->e_mask);
                alg_bytes += dk * (double)vh * (2.0 * bs + ne * (2.0 * bs + 96.0) / nb);
            }
            if (h->stop == STOP_NEVER) continue;
            if (h->breakdown)
                return set_error(HISQ_EBREAKDOWN, "solver breakdown after %d iterations (pAp = %g, |r|^2 = %g)",
                                 h->k, h->pi, h->rho_new);
            if (h->stop < 0 || h->stop >= chunk)
                return set_error(HISQ_EBREAKDOWN, "inconsistent solver state (stop %d, reason %d)", h->stop, h->reason);
            const int js = h->stop, jb = js % nb;
            last_slot = jb;
            HISQ_TRY(realign_shifts(jb));
            if (h->reason == STOP_MSDONE) {
                SpinorList pl;
                for (int i = 0; i < HISQ_MAX_SHIFTS; i++) pl.p[i] = i < nb ? B->p[i] : nullptr;
                HISQ_TRY_HIP(launch_flush_x(B->x64, pl, jb + 1, B->ctrl->alpha_buf, vh, fmt.spinor, fmt.compute,
                                            Guard{nullptr, 0, 0}, st));
                if (ms_done) *ms_done = 1;
                return HISQ_OK;
            }
            const int reason = h->reason;
            HISQ_TRY(enq_reliable(0, jb + 1, B->p[jb]));
            rus++;
            HISQ_TRY(read_ctrl(h));
            last_slot = 0;
            if (h->breakdown) return set_error(HISQ_EBREAKDOWN, "non-finite true residual");
            if (h->done) return HISQ_OK;
            if (reason == STOP_MAXITER || h->k >= h->maxiter)
                return set_error(HISQ_ENOCONV, "no convergence in %d iterations (true residual %g)", h->k,
                                 std::sqrt(h->r2_true / h->b2));
        }
    }

    ~Run() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

void init_ctrl(SolverCtrl *h, const hisq_solver_params &p, double tol, double b2, int sloppy_spinor) {
    memset(h, 0, sizeof(*h));
    h->ru_est = p.ru_estimate;
    h->eps_s = std::ldexp(1.0, -sloppy_floor_bits(sloppy_spinor));
    h->stop = STOP_NEVER;
    h->pr = p.pr_beta;
    h->reproject = p.reproject;
    h->maxiter = p.maxiter;
    h->tol2 = tol * tol;
    h->delta2 = p.delta > 0 ? p.delta * p.delta : 0.0;
    h->b2 = b2;
    h->alpha_prev = 1.0;
    h->beta_prev = 0.0;
}

hisq_status check_params(const hisq_solver_params *p, hisq_solver_params *out) {
    hisq_solver_params d;
    hisq_solver_params_default(&d);
    *out = p ? *p : d;
    if (out->maxiter <= 0) out->maxiter = d.maxiter;
    if (out->grad_buffer < 1 || out->grad_buffer > HISQ_MAX_GRAD_BUFFER)
        return set_error(HISQ_EINVAL, "grad_buffer must be in [1,%d]", HISQ_MAX_GRAD_BUFFER);
    if (out->poll_every <= 0) out->poll_every = d.poll_every;
    if (out->batch_refine < 0 || out->batch_refine > 3)
        return set_error(HISQ_EINVAL, "batch_refine must be 0, 1, 2 or 3");
    if (out->ru_estimate != 0 && out->ru_estimate != 1) return set_error(HISQ_EINVAL, "ru_estimate must be 0 or 1");
    return HISQ_OK;
}

// multi-shift workspace: the solver buffers, then (batched refinement) the
// buffers of a block of min(16, nshift-1) shifted systems (min(16, nshift)
// when the base system joins the block)
struct MsLayout {
    size_t solver, batched;
    bool batch;
};
MsLayout ms_layout(const Geom &g, int nshift, const hisq_fmt &ms_fmt, const hisq_fmt &refine_fmt,
                   const hisq_solver_params &q) {
    MsLayout L;
    const int bs = std::max(spinor_site_bytes(ms_fmt.spinor), spinor_site_bytes(refine_fmt.spinor));
    L.solver = (carve_cg(nullptr, nullptr, g, bs, q.grad_buffer, nshift, spinor_site_bytes(ms_fmt.spinor),
                         spinor_site_bytes(refine_fmt.spinor)) + 255) & ~(size_t)255;
    L.batch = q.batch_refine && nshift > 1 && batched_fmt_ok(refine_fmt);
    const int nblock = std::min(16, q.batch_refine == 3 ? nshift : nshift - 1);
    L.batched = L.batch ? batched_ws_bytes(g, nblock, refine_fmt.spinor, q.grad_buffer) : 0;
    return L;
}

int chunk_of(const hisq_solver_params &p) {
    const int nb = p.grad_buffer;
    return ((p.poll_every + nb - 1) / nb) * nb;
}

hisq_status check_gauge(const hisq_gauge *gg, const int dims[4], const hisq_fmt &f, const char *what) {
    if (!gg || !gg->fat || !gg->lng) return set_error(HISQ_EINVAL, "%s: null gauge field", what);
    for (int k = 0; k < 4; k++)
        if (gg->dims[k] != dims[k]) return set_error(HISQ_EINVAL, "%s: gauge dims differ from the solve", what);
    if (gg->fmt != f.gauge) return set_error(HISQ_EINVAL, "%s: gauge format %d, triplet wants %d", what, gg->fmt, f.gauge);
    if (!aligned16(gg->fat) || !aligned16(gg->lng)) return set_error(HISQ_EALIGN, "%s: gauge not 16-byte aligned", what);
    if (!recon_ok(f, gg->long_recon, false))
        return set_error(HISQ_EINVAL, "%s: eight-parameter long links need FP64 arithmetic on F64 or FIX32 links", what);
    return HISQ_OK;
}

// |b|^2 of the FP64 SoA b64 into ctrl->b2 (device), returned on the host
hisq_status enq_b2(Run &R) {
    int nbk = 0;
    HISQ_TRY_HIP(launch_norm2_f64(R.B->b64, R.vh, R.B->partial, &nbk, R.st));
    hipLaunchKernelGGL(k_fin_b2, dim3(1), dim3(FIN_THREADS), 0, R.st, R.B->ctrl, R.B->partial, nbk);
    HISQ_TRY_HIP(hipGetLastError());
    return HISQ_OK;
}

// Full CG on prepared buffers (x64, b64 filled).  mode 1: fresh start; mode 2:
// continue the gradient vector p_init (refinement format) with rho_prev.
hisq_status cg_core(Run &R, const hisq_solver_params &p, double tol, int mode, const char *p_init, double rho_prev,
                    SolverCtrl *h, double *resid0) {
    init_ctrl(h, p, tol, 0.0, R.fmt.spinor);
    h->rho_prev = rho_prev;
    HISQ_TRY_HIP(hipMemcpyAsync(R.B->ctrl, h, sizeof(SolverCtrl), hipMemcpyHostToDevice, R.st));
    R.setup_plans();
    HISQ_TRY(enq_b2(R));
    HISQ_TRY(R.enq_reliable(mode, 0, mode == 2 ? p_init : nullptr));
    HISQ_TRY(R.read_ctrl(h));
    if (resid0) *resid0 = h->b2 > 0 ? std::sqrt(h->r2_true / h->b2) : 0.0;
    if (h->breakdown) return set_error(HISQ_EBREAKDOWN, "non-finite initial residual");
    if (h->b2 == 0.0 || h->done) return HISQ_OK;
    return R.iterate(h, nullptr);
}

void fill_common_stats(hisq_solver_stats *s, const Run &R) {
    s->iters += (int)R.iters;
    s->reliable_updates += (int)R.rus;
    s->dslash_sloppy += (int)R.dslash_sloppy;
    s->dslash_f64 += (int)R.dslash_f64;
    s->alg_bytes += R.alg_bytes;
}

struct Entry {
    DevState *ds = nullptr;
    hipStream_t user = nullptr;
    std::unique_lock<std::mutex> lock;
    hisq_status begin(void *stream) {
        HISQ_TRY(dev_state(&ds));
        lock = std::unique_lock<std::mutex>(ds->mu);
        user = (hipStream_t)stream;
        HISQ_TRY_HIP(hipEventRecord(ds->ev, user));
        HISQ_TRY_HIP(hipStreamWaitEvent(ds->stream, ds->ev, 0));
        return HISQ_OK;
    }
    hisq_status end() {
        HISQ_TRY_HIP(hipStreamSynchronize(ds->stream));
        return HISQ_OK;
    }
};

}  // namespace

}  // namespace hisq

using namespace hisq;

extern "C" void hisq_solver_params_default(hisq_solver_params *p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->delta = 0.1;
    p->maxiter = 100000;
    p->grad_buffer = 8;
    p->pr_beta = 1;
    p->reproject = 1;
    p->poll_every = 32;
    p->use_graph = 1;
    p->shift_floor = 0.0;
    p->batch_refine = 3;
    p->ru_estimate = 0;
}

extern "C" size_t hisq_cg_workspace_bytes(const int dims[4], hisq_fmt sloppy, const hisq_solver_params *p) {
    if (!dims || !dims_ok(dims) || !triplet_ok(sloppy)) return 0;
    hisq_solver_params q;
    if (check_params(p, &q) != HISQ_OK) return 0;
    const Geom g = make_geom(dims);
    return carve_cg(nullptr, nullptr, g, spinor_site_bytes(sloppy.spinor), q.grad_buffer, 0, 0, 0);
}

extern "C" hisq_status hisq_cg_solve(double *x, const double *b, const hisq_gauge *g64, const hisq_gauge *gs,
                                     double mass, double shift, double tol, hisq_fmt sloppy,
                                     const hisq_solver_params *p, void *ws, size_t ws_bytes,
                                     hisq_solver_stats *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    hisq_solver_stats tmp;
    hisq_solver_stats *st = stats ? stats : &tmp;
    memset(st, 0, sizeof(*st));
    st->status = HISQ_EINVAL;
    if (!x || !b || !g64 || !gs || !ws) return set_error(HISQ_EINVAL, "hisq_cg_solve: null argument");
    if (!aligned16(x) || !aligned16(b) || !aligned16(ws)) return set_error(HISQ_EALIGN, "hisq_cg_solve: unaligned pointer");
    if (!triplet_ok(sloppy)) return set_error(HISQ_EINVAL, "hisq_cg_solve: unsupported sloppy triplet");
    if (!(tol > 0.0)) return set_error(HISQ_EINVAL, "hisq_cg_solve: tol must be > 0");
    const int *dims = g64->dims;
    if (!dims_ok(dims)) return set_error(HISQ_EINVAL, "hisq_cg_solve: bad lattice dims");
    HISQ_TRY(check_gauge(g64, dims, hisq_fmt{HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64}, "g64"));
    HISQ_TRY(check_gauge(gs, dims, sloppy, "gs"));
    hisq_solver_params q;
    HISQ_TRY(check_params(p, &q));
    const Geom g = make_geom(dims);
    CgBuffers B;
    const size_t need = carve_cg(&B, (char *)ws, g, spinor_site_bytes(sloppy.spinor), q.grad_buffer, 0, 0, 0);
    if (ws_bytes < need) return set_error(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    Entry E;
    HISQ_TRY(E.begin(stream));
    Run R;
    R.g = g;
    R.vh = g.vh;
    R.fmt = sloppy;
    R.g64 = g64;
    R.gs = gs;
    R.c_ = 4.0 * mass * mass + shift;
    R.nb = q.grad_buffer;
    R.chunk = chunk_of(q);
    R.graph = q.use_graph != 0;
    R.multishift = false;
    R.nshift = 1;
    R.B = &B;
    R.st = E.ds->stream;
    R.ds = E.ds;
    HISQ_TRY_HIP(launch_spinor_pack(B.x64, x, g.vh, SF_F64, R.st));
    HISQ_TRY_HIP(launch_spinor_pack(B.b64, b, g.vh, SF_F64, R.st));
    SolverCtrl *h = E.ds->host_ctrl;
    hisq_status s = cg_core(R, q, tol, 1, nullptr, 0.0, h, nullptr);
    if (s == HISQ_OK || s == HISQ_ENOCONV || s == HISQ_EBREAKDOWN) {
        hipError_t e = launch_spinor_unpack(x, B.x64, g.vh, SF_F64, R.st);
        if (e != hipSuccess && s == HISQ_OK) s = set_error(HISQ_EHIP, "unpack: %s", hipGetErrorString(e));
    }
    hisq_status s2 = E.end();
    if (s == HISQ_OK) s = s2;
    fill_common_stats(st, R);
    st->true_resid = h->b2 > 0 ? std::sqrt(h->r2_true / h->b2) : 0.0;
    st->nshift = 1;
    st->shift_resid[0] = st->true_resid;
    st->status = s;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

extern "C" size_t hisq_multishift_workspace_bytes(const int dims[4], int nshift, hisq_fmt ms_fmt, hisq_fmt refine_fmt,
                                                  const hisq_solver_params *p) {
    if (!dims || !dims_ok(dims) || !triplet_ok(ms_fmt) || !triplet_ok(refine_fmt)) return 0;
    if (nshift < 1 || nshift > HISQ_MAX_SHIFTS) return 0;
    hisq_solver_params q;
    if (check_params(p, &q) != HISQ_OK) return 0;
    const MsLayout L = ms_layout(make_geom(dims), nshift, ms_fmt, refine_fmt, q);
    return L.solver + L.batched;
}

extern "C" hisq_status hisq_multishift_cg_solve(double *const *x, const double *b, const double *shifts, int nshift,
                                                const double *tol, const hisq_gauge *g64, const hisq_gauge *g_ms,
                                                const hisq_gauge *g_ref, double mass, hisq_fmt ms_fmt,
                                                hisq_fmt refine_fmt, const hisq_solver_params *p, void *ws,
                                                size_t ws_bytes, hisq_solver_stats *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    hisq_solver_stats tmp;
    hisq_solver_stats *st = stats ? stats : &tmp;
    memset(st, 0, sizeof(*st));
    st->status = HISQ_EINVAL;
    if (!x || !b || !shifts || !tol || !g64 || !g_ms || !g_ref || !ws)
        return set_error(HISQ_EINVAL, "hisq_multishift_cg_solve: null argument");
    if (nshift < 1 || nshift > HISQ_MAX_SHIFTS)
        return set_error(HISQ_EINVAL, "nshift must be in [1,%d]", HISQ_MAX_SHIFTS);
    for (int i = 0; i < nshift; i++) {
        if (!x[i] || !aligned16(x[i])) return set_error(HISQ_EALIGN, "x[%d] null or unaligned", i);
        if (!(tol[i] > 0.0)) return set_error(HISQ_EINVAL, "tol[%d] must be > 0", i);
        if (i == 0 && !(shifts[0] >= 0.0)) return set_error(HISQ_EINVAL, "shifts[0] must be >= 0");
        if (i > 0 && !(shifts[i] > shifts[i - 1])) return set_error(HISQ_EINVAL, "shifts must be strictly ascending");
    }
    if (!aligned16(b) || !aligned16(ws)) return set_error(HISQ_EALIGN, "unaligned pointer");
    if (!triplet_ok(ms_fmt) || !triplet_ok(refine_fmt)) return set_error(HISQ_EINVAL, "unsupported triplet");
    const int *dims = g64->dims;
    if (!dims_ok(dims)) return set_error(HISQ_EINVAL, "bad lattice dims");
    HISQ_TRY(check_gauge(g64, dims, hisq_fmt{HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64}, "g64"));
    HISQ_TRY(check_gauge(g_ms, dims, ms_fmt, "g_ms"));
    HISQ_TRY(check_gauge(g_ref, dims, refine_fmt, "g_ref"));
    hisq_solver_params q;
    HISQ_TRY(check_params(p, &q));
    const Geom g = make_geom(dims);
    const int bs = std::max(spinor_site_bytes(ms_fmt.spinor), spinor_site_bytes(refine_fmt.spinor));
    MsLayout L = ms_layout(g, nshift, ms_fmt, refine_fmt, q);
    // eight-parameter long links have no batched Dslash: shifts refined one after another
    L.batch = L.batch && g_ref->long_recon != HISQ_RECON_8;
    if (ws_bytes < L.solver + L.batched)
        return set_error(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.solver + L.batched);
    CgBuffers B;
    carve_cg(&B, (char *)ws, g, bs, q.grad_buffer, nshift, spinor_site_bytes(ms_fmt.spinor),
             spinor_site_bytes(refine_fmt.spinor));
    Entry E;
    HISQ_TRY(E.begin(stream));
    hipStream_t s_ = E.ds->stream;
    SolverCtrl *h = E.ds->host_ctrl;
    st->nshift = nshift;
    hisq_status status = HISQ_OK;
    const double m2 = 4.0 * mass * mass;

    // ---- multi-shift phase (ms_fmt), base = shift 0 ----
    HISQ_TRY_HIP(launch_spinor_pack(B.b64, b, g.vh, SF_F64, s_));
    HISQ_TRY_HIP(hipMemsetAsync(B.x64, 0, 48 * (size_t)g.vh, s_));
    for (int i = 1; i < nshift; i++) HISQ_TRY_HIP(hipMemsetAsync(B.xs[i], 0, 48 * (size_t)g.vh, s_));
    double rho_ms = 0.0;
    int base_slot = 0;
    {
        Run R;
        R.g = g;
        R.vh = g.vh;
        R.fmt = ms_fmt;
        R.g64 = g64;
        R.gs = g_ms;
        R.c_ = m2 + shifts[0];
        R.nb = q.grad_buffer;
        R.chunk = chunk_of(q);
        R.graph = q.use_graph != 0;
        R.multishift = nshift > 1;
        R.nshift = nshift;
        R.B = &B;
        R.st = s_;
        R.ds = E.ds;
        init_ctrl(h, q, tol[0], 0.0, ms_fmt.spinor);
        h->nshift = nshift;
        // where a shifted system's iterated residual stops tracking its true
        // residual: with FP32 arithmetic near the storage format's epsilon;
        // with FP64 arithmetic (INT30 or SX24/INT30 storage included) below
        // any tolerance the FP64 reliable updates certify, so only tol_i stops it
        const double fl = q.shift_floor > 0     ? q.shift_floor
                          : ms_fmt.compute == 64 ? 0.0
                                                 : std::ldexp(1.0, -sloppy_floor_bits(ms_fmt.spinor));
        h->floor2 = fl * fl;
        h->active_mask = 0;
        for (int i = 0; i < nshift; i++) {
            h->sh[i] = shifts[i] - shifts[0];
            h->tol2_i[i] = tol[i] * tol[i];
            h->zeta[i] = h->zeta_prev[i] = 1.0;
            h->active_mask |= 1 << i;
        }
        HISQ_TRY_HIP(hipMemcpyAsync(B.ctrl, h, sizeof(SolverCtrl), hipMemcpyHostToDevice, s_));
        R.setup_plans();
        HISQ_TRY(enq_b2(R));
        HISQ_TRY(R.enq_reliable(1, 0, nullptr));  // x = 0: r = b, p_0 = r
        // every shifted gradient vector starts as p_i = b (stored in the sloppy format)
        for (int i = 1; i < nshift; i++)
            HISQ_TRY_HIP(launch_spinor_convert(B.ps[i], ms_fmt.spinor, B.rs, ms_fmt.spinor, g.vh, s_));
        HISQ_TRY(R.read_ctrl(h));
        if (h->b2 == 0.0) {
            for (int i = 0; i < nshift; i++) HISQ_TRY_HIP(hipMemsetAsync(x[i], 0, 48 * (size_t)g.vh, s_));
            HISQ_TRY(E.end());
            st->status = HISQ_OK;
            return HISQ_OK;
        }
        int ms_done = 0;
        if (!h->done) {
            // one shift: plain CG with reliable updates in the multi-shift triplet
            status = R.iterate(h, &ms_done);
            if (status == HISQ_ENOCONV) status = HISQ_OK;  // the refinement continues from here
        }
        fill_common_stats(st, R);
        for (int i = 1; i < nshift; i++) st->shift_iters[i] = h->shift_stop_k[i] ? h->shift_stop_k[i] : h->k;
        st->shift_iters[0] = h->k;
        rho_ms = h->rho_prev;  // |r_k|^2 of the gradient vector p_k carried into the refinement
        st->phase_seconds[0] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        base_slot = R.last_slot;
        if (status != HISQ_OK) {
            (void)E.end();
            st->status = status;
            return status;
        }
    }

    // ---- refinement (refine_fmt): the base keeps its gradient vector, every shift
    // restarts from its multi-shift solution.  The base first, then the shifts in
    // ascending order or together as a batch; with batch_refine == 2 the batch
    // runs on the second stream while a host thread refines the base on the
    // first (the two are independent once the multi-shift phase is over; every
    // launch shape either uses is planned before they overlap). ----
    auto t1 = std::chrono::steady_clock::now();
    struct Refined {
        hisq_status status = HISQ_OK;
        double r0 = 0.0, r1 = 0.0, seconds = 0.0;
        std::string msg;   // the error message (set in the thread that ran it)
        Run R;
    };
    // refinement run of system i on stream sr with host control block hc
    auto setup_run = [&](Run &R, CgBuffers &Bi, int i, hipStream_t sr) {
        R.g = g;
        R.vh = g.vh;
        R.fmt = refine_fmt;
        R.g64 = g64;
        R.gs = g_ref;
        R.c_ = m2 + shifts[i];
        R.nb = q.grad_buffer;
        R.chunk = chunk_of(q);
        R.graph = q.use_graph != 0;
        R.multishift = false;
        R.nshift = 1;
        Bi = B;
        if (i > 0) Bi.x64 = B.xs[i];
        R.B = &Bi;
        R.st = sr;
        R.ds = E.ds;
    };
    auto refine_one = [&](int i, Refined &out, SolverCtrl *hc) {
        auto ts = std::chrono::steady_clock::now();
        CgBuffers Bi;
        setup_run(out.R, Bi, i, s_);
        if (i == 0 && nshift > 1)
            out.status = cg_core(out.R, q, tol[0], 2, B.pconv, rho_ms, hc, &out.r0);
        else
            out.status = cg_core(out.R, q, tol[i], 1, nullptr, 0.0, hc, &out.r0);
        out.r1 = hc->b2 > 0 ? std::sqrt(hc->r2_true / hc->b2) : 0.0;
        hipError_t e = launch_spinor_unpack(x[i], Bi.x64, g.vh, SF_F64, s_);
        if (e == hipSuccess) e = hipStreamSynchronize(s_);
        if (e != hipSuccess && out.status == HISQ_OK)
            out.status = set_error(HISQ_EHIP, "refinement of system %d: %s", i, hipGetErrorString(e));
        if (out.status != HISQ_OK) out.msg = hisq_last_error();
        out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
    };
    auto account = [&](int i, const Refined &o) {
        st->shift_resid_ms[i] = o.r0;
        st->refine_iters[i] = (int)o.R.iters;
        st->shift_resid[i] = o.r1;
        st->reliable_updates += (int)o.R.rus;
        st->dslash_sloppy += (int)o.R.dslash_sloppy;
        st->dslash_f64 += (int)o.R.dslash_f64;
        st->alg_bytes += o.R.alg_bytes;
    };
    if (nshift > 1 && status == HISQ_OK)
        HISQ_TRY_HIP(launch_spinor_convert(B.pconv, refine_fmt.spinor, B.p[base_slot], ms_fmt.spinor, g.vh, s_));
    const bool overlap = L.batch && nshift > 1 && q.batch_refine == 2;
    const bool joint = L.batch && nshift > 1 && q.batch_refine == 3;
    // one batched block of the systems [i0, i0 + n): the base (i0 == 0) continues its gradient vector
    auto run_block = [&](int i0, int n, hipStream_t sr, SolverCtrl *hc, BatchedJob &J) {
        memset(&J, 0, sizeof(J));
        J.nrhs = n;
        for (int j = 0; j < n; j++) {
            J.x[j] = x[i0 + j];
            J.b[j] = b;
            J.c[j] = m2 + shifts[i0 + j];
            J.tol[j] = tol[i0 + j];
        }
        J.g64 = g64;
        J.gs = g_ref;
        J.fmt = refine_fmt;
        J.q = q;
        J.ws = (char *)ws + L.solver;
        J.ws_bytes = L.batched;
        J.st = sr;
        J.h = hc;
        if (i0 == 0) {
            J.p_warm = B.pconv;
            J.rho_warm = rho_ms;
        }
    };
    auto account_block = [&](int i0, const BatchedJob &J) {
        for (int j = 0; j < J.nrhs; j++) {
            st->shift_resid_ms[i0 + j] = J.resid0_j[j];
            st->refine_iters[i0 + j] = J.iters_j[j];
            st->shift_resid[i0 + j] = J.resid_j[j];
        }
        st->reliable_updates += (int)J.rus;
        st->dslash_sloppy += (int)J.dsl;
        st->dslash_f64 += (int)J.d64;
        st->alg_bytes += J.alg;
    };
    if (joint) {
        // the base joins the shifts' batch as system 0 of the first block,
        // continuing its gradient vector; every system converges on its own
        if (status == HISQ_OK) HISQ_TRY_HIP(launch_spinor_unpack(x[0], B.x64, g.vh, SF_F64, s_));
        for (int i = 1; i < nshift && status == HISQ_OK; i++)
            HISQ_TRY_HIP(launch_spinor_unpack(x[i], B.xs[i], g.vh, SF_F64, s_));
        for (int i0 = 0; i0 < nshift && status == HISQ_OK; i0 += 16) {
            BatchedJob J;
            run_block(i0, std::min(16, nshift - i0), s_, h, J);
            status = batched_run(J);
            account_block(i0, J);
        }
        st->phase_seconds[1] = 0.0;
    } else if (!overlap) {
        // the base, then the shifts: one after another, or together as a batch
        for (int i = 0; i < (L.batch ? 1 : nshift) && status == HISQ_OK; i++) {
            Refined o;
            refine_one(i, o, h);
            status = o.status;
            account(i, o);
            if (i == 0) {
                t1 = std::chrono::steady_clock::now();
                st->phase_seconds[1] = o.seconds;
            }
        }
        if (L.batch && status == HISQ_OK) {
            for (int i = 1; i < nshift; i++) HISQ_TRY_HIP(launch_spinor_unpack(x[i], B.xs[i], g.vh, SF_F64, s_));
            for (int i0 = 1; i0 < nshift && status == HISQ_OK; i0 += 16) {
                BatchedJob J;
                run_block(i0, std::min(16, nshift - i0), s_, h, J);
                status = batched_run(J);
                account_block(i0, J);
            }
        }
    } else if (status == HISQ_OK) {
        // the multi-shift solutions are the shifted systems' initial guesses
        for (int i = 1; i < nshift; i++) HISQ_TRY_HIP(launch_spinor_unpack(x[i], B.xs[i], g.vh, SF_F64, s_));
        // the base run's launch shapes, planned before anything overlaps
        {
            Run Rp;
            CgBuffers Bp;
            setup_run(Rp, Bp, 0, s_);
            Rp.setup_plans();
        }
        HISQ_TRY_HIP(hipEventRecord(E.ds->ev2, s_));
        hipStream_t s2 = E.ds->stream2;
        HISQ_TRY_HIP(hipStreamWaitEvent(s2, E.ds->ev2, 0));
        Refined base;
        std::thread worker;
        struct Start {
            std::thread *w;
            std::function<void()> fn;
        } start{&worker, [&] { refine_one(0, base, h); }};
        for (int i0 = 1; i0 < nshift && status == HISQ_OK; i0 += 16) {
            BatchedJob J;
            run_block(i0, std::min(16, nshift - i0), s2, E.ds->host_ctrl2, J);
            if (!worker.joinable()) {
                // the base starts once the block's launch shapes are planned
                J.after_setup = [](void *c) {
                    Start *sp = static_cast<Start *>(c);
                    try {
                        *sp->w = std::thread(sp->fn);
                    } catch (...) {
                        // no thread: the base is refined after the batch
                    }
                };
                J.after_setup_ctx = &start;
            }
            status = batched_run(J);
            account_block(i0, J);
        }
        if (worker.joinable()) {
            worker.join();
        } else {
            refine_one(0, base, h);   // the batched block stopped before it started the base
        }
        account(0, base);
        st->phase_seconds[1] = base.seconds;
        if (status == HISQ_OK && base.status != HISQ_OK)
            status = set_error(base.status, "base refinement: %s", base.msg.c_str());
    }
    hisq_status s2 = E.end();
    if (status == HISQ_OK) status = s2;
    st->phase_seconds[2] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
    double worst = 0.0;
    for (int i = 0; i < nshift; i++) worst = std::max(worst, st->shift_resid[i] / tol[i] * tol[0]);
    st->true_resid = worst;
    st->status = status;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}
