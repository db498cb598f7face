// hisq_batched.hip -- a block of independent mixed-precision CG solves that
// share every Dslash launch (Sec. 1, "Block solvers": the link traffic of the
// stencil is amortised over the right-hand sides).
//
// Each right-hand side j keeps its own scalars (rho_j, alpha_j, beta_j, ...)
// in the control block; the Dslash applies one load of each link matrix to all
// nrhs spinors.  The iteration is the single-system one of hisq_solver.hip
// (buffered FP64 solution, Polak-Ribiere beta, reliable updates with
// re-projection) done for every j at once.  When a right-hand side asks for a
// reliable update (or its iterated residual meets tol) the block stops; only
// the right-hand sides that asked compute their true residual (the FP64 Dslash
// skips the others), replace r and re-project p, while the others take their
// ordinary CG step; every buffered gradient is flushed.  A right-hand side
// whose true residual meets tol stops updating and costs no more Dslash work.
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

// finalize kernels: 16 waves per block; each thread loads its strided share
// of the block partials four entries at a time (all four in flight) and adds
// them in index order
constexpr int FIN_THREADS = 1024;

// sum over blocks b of partial[(b*nrhs + j)*NV + k], k < NV; valid in thread 0
template <int NV>
__device__ __forceinline__ void bsum(const double *partial, int nb, int nrhs, int j, double (&v)[NV], double *lds) {
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = 0.0;
    const int step = blockDim.x;
    int b = threadIdx.x;
    for (; b + 3 * step < nb; b += 4 * step) {
        double q[4][NV];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int k = 0; k < NV; k++) q[u][k] = partial[((size_t)(b + u * step) * nrhs + j) * NV + k];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int k = 0; k < NV; k++) v[k] += q[u][k];
    }
    for (; b < nb; b += step) {
#pragma unroll
        for (int k = 0; k < NV; k++) v[k] += partial[((size_t)b * nrhs + j) * NV + k];
    }
    block_sum<NV>(v, lds);
    __syncthreads();
}

// Dslash partials: right-hand side j owns column partial[j*pstride + b], b < nb[j]
struct NbList {
    int nb[16];
    size_t pstride;
};

__device__ __forceinline__ void csum(const double *col, int nb, double (&v)[1], double *lds) {
    v[0] = 0.0;
    const int step = blockDim.x;
    int b = threadIdx.x;
    for (; b + 3 * step < nb; b += 4 * step) {
        const double q0 = col[b], q1 = col[b + step], q2 = col[b + 2 * step], q3 = col[b + 3 * step];
        v[0] += q0;
        v[0] += q1;
        v[0] += q2;
        v[0] += q3;
    }
    for (; b < nb; b += step) v[0] += col[b];
    block_sum<1>(v, lds);
    __syncthreads();
}

// one block per right-hand side j (launched with nrhs blocks): the columns are
// independent, and a Dslash over rg lanes per site leaves rg times more partials
// per column than sites per block; each column is summed in a fixed order
__global__ void k_bfin_alpha(SolverCtrl *c, const double *partial, NbList nl, int nrhs, int jb, Guard gd) {
    __shared__ double lds[FIN_THREADS / 64];
    const int j = blockIdx.x;
    if (j >= nrhs || !gd.pass()) return;
    double v[1];
    csum(partial + (size_t)j * nl.pstride, nl.nb[j], v, lds);
    if (threadIdx.x) return;
    const double pi = v[0];
    c->bpi[j] = pi;
    if (!c->bactive[j]) {
        c->balpha[j] = 0.0;
        c->balpha_buf[jb][j] = 0.0;
        return;
    }
    if (!(pi > 0.0) || !__builtin_isfinite(pi)) {
        // every block that finds a breakdown writes the same stop record
        c->stop = gd.j - 1;
        c->reason = STOP_BREAKDOWN;
        c->breakdown = 1;
        c->balpha[j] = 0.0;
        c->balpha_buf[jb][j] = 0.0;
        return;
    }
    const double a = c->brho[j] / pi;
    c->balpha[j] = a;
    c->balpha_buf[jb][j] = a;
}

__global__ void k_bfin_beta(SolverCtrl *c, const double *partial, int nb, int nrhs, Guard gd) {
    __shared__ double lds[2 * (FIN_THREADS / 64)];
    if (!gd.pass()) return;
    int reason = STOP_NONE;
    for (int j = 0; j < nrhs; j++) {
        double v[2];
        bsum<2>(partial, nb, nrhs, j, v, lds);
        if (threadIdx.x || !c->bactive[j]) continue;
        const double rn = v[0], g = v[1];
        c->bk[j] += 1;
        if (!__builtin_isfinite(rn) || !__builtin_isfinite(g)) {
            reason = STOP_BREAKDOWN;
            c->breakdown = 1;
            continue;
        }
        const double rho = c->brho[j];
        const double beta = c->pr ? (rn - g) / rho : rn / rho;
        c->bbeta[j] = beta;
        c->bpa_re[j] = 1.0;
        c->bpa_im[j] = 0.0;
        c->bpb[j] = beta;
        c->brmax2[j] = fmax(c->brmax2[j], rn);
        const bool ru = c->delta2 > 0.0 && rn < c->delta2 * c->brmax2[j];
        const bool conv = rn <= c->btol2[j] * c->bb2[j];
        if (ru) reason = reason ? reason : STOP_RU;
        if (conv) reason = reason ? reason : STOP_CONV;
        if (ru || conv) c->bru[j] = 1;
        c->brho_prev[j] = rho;
        c->brho[j] = rn;
    }
    if (threadIdx.x) return;
    const int k = c->k + 1;
    c->k = k;
    if (reason == STOP_NONE && k >= c->maxiter) {
        reason = STOP_MAXITER;
        for (int j = 0; j < nrhs; j++) c->bru[j] = c->bactive[j];   // report every true residual
    }
    if (reason == STOP_RU || reason == STOP_CONV) {
        // systems whose residual norm is within a factor of about 3 (10 in its square) of
        // their own trigger join this reliable update
        // (one FP64 application serves them all instead of one each shortly after)
        for (int j = 0; j < nrhs; j++)
            if (c->bactive[j] && c->delta2 > 0.0 && c->brho[j] < 10.0 * c->delta2 * c->brmax2[j]) c->bru[j] = 1;
    }
    if (reason != STOP_NONE) {
        c->reason = reason;
        c->stop = gd.j;
    }
}

__global__ void k_bfin_ru_check(SolverCtrl *c, const double *partial, NbList nl, int nrhs) {
    __shared__ double lds[FIN_THREADS / 64];
    int all = 1;
    for (int j = 0; j < nrhs; j++) {
        double v[1];
        csum(partial + (size_t)j * nl.pstride, nl.nb[j], v, lds);
        if (threadIdx.x) continue;
        if (c->bru[j] && c->bactive[j]) {
            const double r2 = v[0];
            c->br2_true[j] = r2;
            if (!__builtin_isfinite(r2)) c->breakdown = 1;
            if (r2 <= c->btol2[j] * c->bb2[j]) {
                c->bactive[j] = 0;
                c->bdone[j] = 1;
            }
        }
        all &= !c->bactive[j];
    }
    if (threadIdx.x) return;
    c->done = all;
    c->stop = (all || c->breakdown) ? -1 : STOP_NEVER;
}

__global__ void k_bfin_ru_finish(SolverCtrl *c, const double *partial, int nb, int nrhs, int mode, Guard gd) {
    __shared__ double lds[4 * (FIN_THREADS / 64)];
    if (!gd.pass()) return;
    for (int j = 0; j < nrhs; j++) {
        double v[4];
        bsum<4>(partial, nb, nrhs, j, v, lds);
        if (threadIdx.x || !c->bactive[j] || !c->bru[j]) continue;   // the others keep their CG step
        const double rho = v[0];
        double beta = 0.0, cr = 0.0, ci = 0.0;
        // the first reliable update restarts every system, except one that
        // continues a given gradient vector (re-projected, Fletcher-Reeves beta:
        // there is no previous iterated residual to form Polak-Ribiere's)
        if (mode != 1 || c->bwarm[j]) {
            if (c->reproject && rho > 0.0) {
                cr = v[1] / rho;
                ci = v[2] / rho;
            }
            beta = c->pr ? (rho - v[3]) / c->brho_prev[j] : rho / c->brho_prev[j];
        }
        c->bpa_re[j] = 1.0 - beta * cr;
        c->bpa_im[j] = -beta * ci;
        c->bpb[j] = beta;
        c->bbeta[j] = beta;
        c->brho[j] = rho;
        c->brmax2[j] = rho;
        c->bwarm[j] = 0;
    }
    if (threadIdx.x) return;
    for (int j = 0; j < nrhs; j++) c->bru[j] = 0;
    c->reason = STOP_NONE;
    c->stop = STOP_NEVER;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BBuf {
    SolverCtrl *ctrl;
    double *partial;
    char *x64, *b64, *r64, *t64;
    char *rs, *aps, *ts;
    char *p[HISQ_MAX_GRAD_BUFFER];
};

size_t partial_len(const Geom &g, int nrhs) {
    const size_t a = dslash_max_blocks(g) * nrhs;
    const size_t b = (size_t)4096 * 4 * nrhs;
    return std::max(a, b);
}

size_t carve(BBuf *B, char *base, const Geom &g, int nrhs, int bs, int nb) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    BBuf tmp;
    BBuf &b = B ? *B : tmp;
    const size_t vh = g.vh;
    b.ctrl = (SolverCtrl *)take(sizeof(SolverCtrl));
    b.partial = (double *)take(partial_len(g, nrhs) * sizeof(double));
    b.x64 = take(48 * vh * nrhs);
    b.b64 = take(48 * vh * nrhs);
    b.r64 = take(48 * vh * nrhs);
    b.t64 = take(48 * vh * nrhs);
    b.rs = take((size_t)bs * vh * nrhs);
    b.aps = take((size_t)bs * vh * nrhs);
    b.ts = take((size_t)bs * vh * nrhs);
    for (int i = 0; i < HISQ_MAX_GRAD_BUFFER; i++) b.p[i] = i < nb ? take((size_t)bs * vh * nrhs) : nullptr;
    return off;
}

struct BRun {
    Geom g;
    size_t vh;
    int nrhs;
    hisq_fmt fmt;
    const hisq_gauge *g64, *gs;
    int nb, chunk;
    bool graph;
    BBuf *B;
    hipStream_t st;
    size_t fs, fs64;
    long iters = 0, rus = 0, dsl = 0, d64 = 0;
    double alg = 0.0;
    hipGraphExec_t exec = nullptr;
    // A Dslash launch over a set of field columns: the plan for the block padded
    // to a power of two and the column map that deals the columns round-robin
    // over the lane groups (column i of the set -> group i % rg, slot i / rg),
    // so that the lanes of a site share the work of the longest-running systems.
    // Launches with a fused reduction have their own tile, hence their own map;
    // they write the partials that nl describes.
    struct Mapped {
        DslashPlan plan{};
        unsigned mask = 0;            // field columns in the launch
        unsigned cvalid = 0, cvalid_red = 0;
        unsigned long long cmap = 0, cmap_red = 0;
        NbList nl{};
    };
    Mapped ms_{}, m64_{};

    Mapped map_columns(const hisq_fmt &f, const hisq_gauge *gg, char *out, const char *in, unsigned mask) {
        Mapped m;
        m.mask = mask;
        int cols[16], n = 0;
        for (int j = 0; j < nrhs; j++)
            if ((mask >> j) & 1u) cols[n++] = j;
        // tune (first use of a key) on a dense map of the same columns
        DslashArgs probe = dargs(gg, f, out, in, 1);
        probe.nrhs = n;
        probe.cmapped = 1;
        probe.cvalid = n >= 16 ? 0xffffu : ((1u << n) - 1u);
        probe.cmap = 0;
        for (int k = 0; k < n; k++) probe.cmap |= (unsigned long long)cols[k] << (4 * k);
        m.plan = dslash_plan(f, g, n, &probe, st);
        const DslashTile &t = m.plan.tile[0], &tr = m.plan.tile_red[0];
        for (int i = 0; i < n; i++) {
            const int k = (i % t.rg) * t.nr + i / t.rg;
            m.cmap |= (unsigned long long)cols[i] << (4 * k);
            m.cvalid |= 1u << k;
            const int kr = (i % tr.rg) * tr.nr + i / tr.rg;
            m.cmap_red |= (unsigned long long)cols[i] << (4 * kr);
            m.cvalid_red |= 1u << kr;
        }
        m.nl.pstride = dslash_max_blocks(g);
        for (int j = 0; j < 16; j++) m.nl.nb[j] = dslash_tile_blocks(g, tr);
        return m;
    }

    // the column map of plan m for launch a (set a.red first)
    void apply(DslashArgs &a, const Mapped &m) const {
        const bool red = a.red != RED_NONE;
        a.nrhs = __builtin_popcount(m.mask);
        a.cmapped = 1;
        a.cvalid = red ? m.cvalid_red : m.cvalid;
        a.cmap = red ? m.cmap_red : m.cmap;
    }

    // plan every block the solve can shrink to (a power of two of columns up to
    // nrhs), for the sloppy and the FP64 operator: the autotuner runs here, not
    // later while the solve shares the device with other work
    void pretune() {
        const hisq_fmt f64 = {HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64};
        for (int c = 1;; c <<= 1) {
            const int n = std::min(c, nrhs);
            const unsigned mask = n >= 16 ? 0xffffu : ((1u << n) - 1u);
            (void)map_columns(fmt, gs, B->ts, B->rs, mask);
            (void)map_columns(f64, g64, B->t64, B->x64, mask);
            if (n == nrhs) break;
        }
    }

    // the sloppy launches cover the systems still iterating; a change of that set
    // re-plans them and drops the captured block of iterations
    hisq_status remap_sloppy(const SolverCtrl *h) {
        unsigned mask = 0;
        for (int j = 0; j < nrhs; j++)
            if (h->bactive[j]) mask |= 1u << j;
        if (mask == 0 || mask == ms_.mask) return HISQ_OK;
        ms_ = map_columns(fmt, gs, B->ts, B->rs, mask);
        if (exec) {
            HISQ_TRY_HIP(hipGraphExecDestroy(exec));
            exec = nullptr;
        }
        return HISQ_OK;
    }

    ~BRun() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }

    DslashArgs dargs(const hisq_gauge *gg, const hisq_fmt &f, char *out, const char *in, int parity) const {
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
        a.nrhs = nrhs;
        a.field_stride = spinor_field_bytes(vh, f.spinor);
        gauge_args(a, gg);
        return a;
    }

    hisq_status enq_iteration(int j) {
        const int jb = j % nb, jn = (j + 1) % nb;
        SolverCtrl *c = B->ctrl;
        const Guard gns{&c->stop, j, 0}, gsn{&c->stop, j, 1};
        DslashArgs A = dargs(gs, fmt, B->ts, B->p[jb], 1);
        apply(A, ms_);
        A.guard = gns;
        A.cactive = c->bactive;   // stopped systems cost no Dslash work
        HISQ_TRY_HIP(launch_dslash(A, fmt, ms_.plan, st, nullptr));
        DslashArgs Bk = dargs(gs, fmt, B->aps, B->ts, 0);
        Bk.red = RED_DOT_X;
        apply(Bk, ms_);
        Bk.b = -1.0;
        Bk.x = B->p[jb];
        Bk.acol = c->bc;
        Bk.cactive = c->bactive;
        Bk.partial = B->partial;
        Bk.pstride = ms_.nl.pstride;
        Bk.guard = gns;
        HISQ_TRY_HIP(launch_dslash(Bk, fmt, ms_.plan, st, nullptr));
        hipLaunchKernelGGL(k_bfin_alpha, dim3(nrhs), dim3(FIN_THREADS), 0, st, c, B->partial, ms_.nl, nrhs, jb, gns);
        HISQ_TRY_HIP(hipGetLastError());
        HISQ_TRY_HIP(launch_bcg_axpy(B->rs, B->aps, c, vh, fs, nrhs, fmt.spinor, fmt.compute, B->partial, gns, st));
        hipLaunchKernelGGL(k_bfin_beta, dim3(1), dim3(FIN_THREADS), 0, st, c, B->partial, blas_blocks(vh), nrhs, gns);
        HISQ_TRY_HIP(hipGetLastError());
        if (jb == nb - 1) {
            SpinorList pl;
            for (int i = 0; i < HISQ_MAX_SHIFTS; i++) pl.p[i] = i < nb ? B->p[i] : nullptr;
            HISQ_TRY_HIP(launch_bflush_x(B->x64, fs64, pl, nb, c, vh, fs, nrhs, fmt.spinor, fmt.compute, gsn, st));
        }
        HISQ_TRY_HIP(launch_bcg_pupdate(B->p[jn], B->rs, B->p[jb], c, vh, fs, nrhs, fmt.spinor, fmt.compute, gsn, st));
        return HISQ_OK;
    }

    // ru_mask: the systems taking part (the FP64 launches cover those only)
    hisq_status enq_reliable(int mode, int count, const char *p_src, unsigned ru_mask) {
        SolverCtrl *c = B->ctrl;
        const hisq_fmt f64 = {HISQ_GAUGE_F64, HISQ_SPINOR_F64, 64};
        const int nru = __builtin_popcount(ru_mask);
        if (ru_mask != m64_.mask) m64_ = map_columns(f64, g64, B->t64, B->x64, ru_mask);
        if (count > 0) {
            SpinorList pl;
            for (int i = 0; i < HISQ_MAX_SHIFTS; i++) pl.p[i] = i < nb ? B->p[i] : nullptr;
            HISQ_TRY_HIP(launch_bflush_x(B->x64, fs64, pl, count, c, vh, fs, nrhs, fmt.spinor, fmt.compute,
                                         Guard{nullptr, 0, 0}, st));
        }
        // true residuals of the systems taking part (c->bru) only
        DslashArgs A = dargs(g64, f64, B->t64, B->x64, 1);
        apply(A, m64_);
        A.cactive = c->bru;
        HISQ_TRY_HIP(launch_dslash(A, f64, m64_.plan, st, nullptr));
        DslashArgs Bk = dargs(g64, f64, B->r64, B->t64, 0);
        Bk.red = RED_NORM;
        apply(Bk, m64_);
        Bk.cactive = c->bru;
        Bk.x = B->x64;
        Bk.acol = c->bnc;
        Bk.y = B->b64;
        Bk.c = 1.0;
        Bk.partial = B->partial;
        Bk.pstride = m64_.nl.pstride;
        HISQ_TRY_HIP(launch_dslash(Bk, f64, m64_.plan, st, nullptr));
        hipLaunchKernelGGL(k_bfin_ru_check, dim3(1), dim3(FIN_THREADS), 0, st, c, B->partial, m64_.nl, nrhs);
        HISQ_TRY_HIP(hipGetLastError());
        d64 += 2;
        alg += 2.0 * vh * (dslash_link_bytes(g64) + nru * 2.0 * 48) + 2.0 * vh * nru * 48;
        const Guard g0{&c->stop, 0, 0};
        HISQ_TRY_HIP(launch_bru_convert(B->rs, B->r64, fs64, p_src, mode == 0 ? B->aps : nullptr,
                                        c, vh, fs, nrhs, fmt.spinor, fmt.compute, B->partial, g0, st));
        hipLaunchKernelGGL(k_bfin_ru_finish, dim3(1), dim3(FIN_THREADS), 0, st, c, B->partial, blas_blocks(vh), nrhs,
                           mode, g0);
        HISQ_TRY_HIP(hipGetLastError());
        HISQ_TRY_HIP(launch_bcg_pupdate(B->p[0], B->rs, p_src ? p_src : B->rs, c, vh, fs, nrhs, fmt.spinor,
                                        fmt.compute, g0, st));
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
};

struct BDev {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    SolverCtrl *host = nullptr;
    std::mutex mu;
};
BDev g_bdev[64];

}  // namespace

bool batched_fmt_ok(const hisq_fmt &f) {
    return triplet_ok(f) && has_batched_form(f);
}

size_t batched_ws_bytes(const Geom &g, int nrhs, int sf, int nb) {
    return carve(nullptr, nullptr, g, nrhs, spinor_site_bytes(sf), nb);
}

hisq_status batched_run(BatchedJob &J) {
    const int nrhs = J.nrhs;
    const hisq_solver_params &q = J.q;
    const Geom g = make_geom(J.g64->dims);
    hipStream_t s_ = J.st;
    J.iters = J.rus = J.dsl = J.d64 = 0;
    J.alg = 0.0;
    BBuf B;
    const size_t need = carve(&B, (char *)J.ws, g, nrhs, spinor_site_bytes(J.fmt.spinor), q.grad_buffer);
    if (J.ws_bytes < need) return set_error(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", J.ws_bytes, need);

    BRun R;
    R.g = g;
    R.vh = g.vh;
    R.nrhs = nrhs;
    R.fmt = J.fmt;
    R.g64 = J.g64;
    R.gs = J.gs;
    R.nb = q.grad_buffer;
    R.chunk = ((q.poll_every + q.grad_buffer - 1) / q.grad_buffer) * q.grad_buffer;
    R.graph = q.use_graph != 0;
    R.B = &B;
    R.st = s_;
    R.fs = spinor_field_bytes(g.vh, J.fmt.spinor);
    R.fs64 = spinor_field_bytes(g.vh, SF_F64);

    for (int j = 0; j < nrhs; j++) {
        HISQ_TRY_HIP(launch_spinor_pack(B.x64 + j * R.fs64, J.x[j], g.vh, SF_F64, s_));
        HISQ_TRY_HIP(launch_spinor_pack(B.b64 + j * R.fs64, J.b[j], g.vh, SF_F64, s_));
    }
    SolverCtrl *h = J.h;
    memset(h, 0, sizeof(*h));
    h->stop = STOP_NEVER;
    h->pr = q.pr_beta;
    h->reproject = q.reproject;
    h->maxiter = q.maxiter;
    h->delta2 = q.delta > 0 ? q.delta * q.delta : 0.0;
    for (int j = 0; j < nrhs; j++) {
        h->bactive[j] = 1;
        h->bru[j] = 1;   // the first reliable update computes every initial residual
        h->bc[j] = J.c[j];
        h->bnc[j] = -J.c[j];
        h->btol2[j] = J.tol[j] * J.tol[j];
    }
    if (J.p_warm) {
        // system 0 continues the given gradient vector: it goes to column 0 of
        // the first ring slot (the other columns are zero, so the fused update
        // p = r + 0 p of the restarting systems stays finite)
        h->bwarm[0] = 1;
        h->brho_prev[0] = J.rho_warm;
        HISQ_TRY_HIP(hipMemsetAsync(B.p[0], 0, (size_t)nrhs * R.fs, s_));
        HISQ_TRY_HIP(hipMemcpyAsync(B.p[0], J.p_warm, R.fs, hipMemcpyDeviceToDevice, s_));
    }
    HISQ_TRY_HIP(hipMemcpyAsync(B.ctrl, h, sizeof(SolverCtrl), hipMemcpyHostToDevice, s_));
    // |b_j|^2: the F64 norm kernel per right-hand side, each into its own partial column
    for (int j = 0; j < nrhs; j++) {
        int nbk = 0;
        HISQ_TRY_HIP(launch_norm2_f64(B.b64 + j * R.fs64, g.vh, B.partial + (size_t)j * 4096, &nbk, s_));
    }
    // gather b2 on the host (once per solve) and store it in the control block
    {
        const int nbk = blas_blocks(g.vh);
        std::vector<double> part((size_t)nrhs * 4096);
        HISQ_TRY_HIP(hipMemcpyAsync(part.data(), B.partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
        HISQ_TRY_HIP(hipStreamSynchronize(s_));
        for (int j = 0; j < nrhs; j++) {
            double acc = 0.0;
            for (int k = 0; k < nbk; k++) acc += part[(size_t)j * 4096 + k];
            h->bb2[j] = acc;
            if (acc == 0.0) {   // b_j = 0: x_j = 0 whatever the initial guess
                h->bactive[j] = 0;
                h->bdone[j] = 1;
                HISQ_TRY_HIP(hipMemsetAsync(B.x64 + j * R.fs64, 0, R.fs64, s_));
            }
        }
        HISQ_TRY_HIP(hipMemcpyAsync(B.ctrl, h, sizeof(SolverCtrl), hipMemcpyHostToDevice, s_));
    }
    if (J.after_setup) {
        R.pretune();
        HISQ_TRY_HIP(hipStreamSynchronize(s_));
        J.after_setup(J.after_setup_ctx);
    }
    unsigned m0 = 0;   // systems with b != 0: their initial true residuals
    for (int j = 0; j < nrhs; j++)
        if (h->bactive[j]) m0 |= 1u << j;
    hisq_status status = HISQ_OK;
    if (m0) {
        status = R.enq_reliable(1, 0, J.p_warm ? B.p[0] : nullptr, m0);
        if (status == HISQ_OK) status = R.read_ctrl(h);
    } else {
        h->done = 1;
    }
    for (int j = 0; j < nrhs; j++) J.resid0_j[j] = h->bb2[j] > 0 ? std::sqrt(h->br2_true[j] / h->bb2[j]) : 0.0;
    if (status == HISQ_OK && !h->done) status = R.remap_sloppy(h);
    long k0 = 0;
    while (status == HISQ_OK && !h->done) {
        if (h->breakdown) {
            status = set_error(HISQ_EBREAKDOWN, "batched CG breakdown");
            break;
        }
        status = R.enq_chunk();
        if (status != HISQ_OK) break;
        status = R.read_ctrl(h);
        if (status != HISQ_OK) break;
        const long dk = h->k - k0;
        k0 = h->k;
        R.iters += dk;
        R.dsl += 2 * dk;
        {
            // links once per Dslash; spinor traffic of the systems still iterating
            int na = 0;
            for (int j = 0; j < nrhs; j++) na += h->bactive[j] ? 1 : 0;
            const double bs = spinor_site_bytes(J.fmt.spinor), bl = dslash_link_bytes(J.gs);
            R.alg += dk * (double)g.vh * (2.0 * (bl + na * 2.0 * bs) + na * (7.0 * bs + (R.nb * bs + 96.0) / R.nb));
        }
        if (h->stop == STOP_NEVER) continue;
        if (h->breakdown) {
            status = set_error(HISQ_EBREAKDOWN, "batched CG breakdown after %d iterations", h->k);
            break;
        }
        if (h->stop < 0 || h->stop >= R.chunk) {
            status = set_error(HISQ_EBREAKDOWN, "inconsistent batched solver state (stop %d)", h->stop);
            break;
        }
        const int jb = h->stop % R.nb;
        const int reason = h->reason;
        unsigned rum = 0, act = 0;
        for (int j = 0; j < nrhs; j++) {
            if (h->bru[j] && h->bactive[j]) rum |= 1u << j;
            if (h->bactive[j]) act |= 1u << j;
        }
        status = R.enq_reliable(0, jb + 1, B.p[jb], rum ? rum : act);
        if (status != HISQ_OK) break;
        R.rus++;
        status = R.read_ctrl(h);
        if (status != HISQ_OK) break;
        if (h->done) break;
        status = R.remap_sloppy(h);
        if (status != HISQ_OK) break;
        if (reason == STOP_MAXITER || h->k >= q.maxiter) {
            status = set_error(HISQ_ENOCONV, "batched CG: no convergence in %d iterations", h->k);
            break;
        }
    }
    for (int j = 0; j < nrhs; j++) {
        hipError_t e = launch_spinor_unpack(J.x[j], B.x64 + j * R.fs64, g.vh, SF_F64, s_);
        if (e != hipSuccess && status == HISQ_OK) status = set_error(HISQ_EHIP, "unpack: %s", hipGetErrorString(e));
    }
    hipError_t e = hipStreamSynchronize(s_);
    if (e != hipSuccess && status == HISQ_OK) status = set_error(HISQ_EHIP, "sync: %s", hipGetErrorString(e));
    J.iters = R.iters;
    J.rus = R.rus;
    J.dsl = R.dsl;
    J.d64 = R.d64;
    J.alg = R.alg;
    for (int j = 0; j < nrhs; j++) {
        J.resid_j[j] = h->bb2[j] > 0 ? std::sqrt(h->br2_true[j] / h->bb2[j]) : 0.0;
        J.iters_j[j] = h->bk[j];
    }
    return status;
}

}  // namespace hisq

using namespace hisq;

extern "C" size_t hisq_cg_batched_workspace_bytes(const int dims[4], int nrhs, hisq_fmt sloppy,
                                                  const hisq_solver_params *p) {
    if (!dims || !dims_ok(dims) || !triplet_ok(sloppy) || nrhs < 1 || nrhs > 16) return 0;
    hisq_solver_params q;
    hisq_solver_params_default(&q);
    if (p) q = *p;
    if (q.grad_buffer < 1 || q.grad_buffer > HISQ_MAX_GRAD_BUFFER) return 0;
    return batched_ws_bytes(make_geom(dims), nrhs, sloppy.spinor, q.grad_buffer);
}

extern "C" hisq_status hisq_cg_solve_batched(double *x, const double *b, int nrhs, const hisq_gauge *g64,
                                             const hisq_gauge *gs, double mass, double shift, double tol,
                                             hisq_fmt sloppy, const hisq_solver_params *p, void *ws, size_t ws_bytes,
                                             hisq_solver_stats *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    hisq_solver_stats tmp;
    hisq_solver_stats *st = stats ? stats : &tmp;
    memset(st, 0, sizeof(*st));
    st->status = HISQ_EINVAL;
    if (!x || !b || !g64 || !gs || !ws) return set_error(HISQ_EINVAL, "hisq_cg_solve_batched: null argument");
    if (nrhs < 1 || nrhs > 16) return set_error(HISQ_EINVAL, "hisq_cg_solve_batched: nrhs must be in [1,16]");
    if (!aligned16(x) || !aligned16(b) || !aligned16(ws)) return set_error(HISQ_EALIGN, "unaligned pointer");
    if (!batched_fmt_ok(sloppy)) return set_error(HISQ_EINVAL, "hisq_cg_solve_batched: unsupported sloppy triplet");
    if (!(tol > 0.0)) return set_error(HISQ_EINVAL, "tol must be > 0");
    const int *dims = g64->dims;
    if (!dims_ok(dims)) return set_error(HISQ_EINVAL, "bad lattice dims");
    if (!gs->fat || !gs->lng || gs->fmt != sloppy.gauge || g64->fmt != HISQ_GAUGE_F64 || !g64->fat || !g64->lng)
        return set_error(HISQ_EINVAL, "gauge format mismatch or null gauge");
    if (gs->long_recon == HISQ_RECON_8 || g64->long_recon == HISQ_RECON_8)
        return set_error(HISQ_EINVAL, "hisq_cg_solve_batched: eight-parameter long links have no batched Dslash");
    for (int k = 0; k < 4; k++)
        if (gs->dims[k] != dims[k]) return set_error(HISQ_EINVAL, "gauge dims differ");
    hisq_solver_params q;
    hisq_solver_params_default(&q);
    if (p) q = *p;
    if (q.grad_buffer < 1 || q.grad_buffer > HISQ_MAX_GRAD_BUFFER) return set_error(HISQ_EINVAL, "bad grad_buffer");
    if (q.maxiter <= 0) q.maxiter = 100000;
    if (q.poll_every <= 0) q.poll_every = 32;
    const Geom g = make_geom(dims);
    const size_t need = batched_ws_bytes(g, nrhs, sloppy.spinor, q.grad_buffer);
    if (ws_bytes < need) return set_error(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);

    int d = 0;
    HISQ_TRY_HIP(hipGetDevice(&d));
    BDev &dv = g_bdev[d & 63];
    std::unique_lock<std::mutex> lk(dv.mu);
    if (!dv.stream) {
        HISQ_TRY_HIP(hipStreamCreateWithFlags(&dv.stream, hipStreamNonBlocking));
        HISQ_TRY_HIP(hipEventCreateWithFlags(&dv.ev, hipEventDisableTiming));
        HISQ_TRY_HIP(hipHostMalloc((void **)&dv.host, sizeof(SolverCtrl), hipHostMallocDefault));
    }
    HISQ_TRY_HIP(hipEventRecord(dv.ev, (hipStream_t)stream));
    HISQ_TRY_HIP(hipStreamWaitEvent(dv.stream, dv.ev, 0));

    BatchedJob J;
    memset(&J, 0, sizeof(J));
    J.nrhs = nrhs;
    for (int j = 0; j < nrhs; j++) {
        J.x[j] = x + 6 * (size_t)g.vh * j;
        J.b[j] = b + 6 * (size_t)g.vh * j;
        J.c[j] = 4.0 * mass * mass + shift;
        J.tol[j] = tol;
    }
    J.g64 = g64;
    J.gs = gs;
    J.fmt = sloppy;
    J.q = q;
    J.ws = ws;
    J.ws_bytes = ws_bytes;
    J.st = dv.stream;
    J.h = dv.host;
    hisq_status status = batched_run(J);
    st->iters = (int)J.iters;
    st->reliable_updates = (int)J.rus;
    st->dslash_sloppy = (int)J.dsl;
    st->dslash_f64 = (int)J.d64;
    st->alg_bytes = J.alg;
    st->nshift = nrhs;
    double worst = 0.0;
    for (int j = 0; j < nrhs; j++) {
        st->shift_resid_ms[j] = J.resid0_j[j];
        st->shift_resid[j] = J.resid_j[j];
        st->refine_iters[j] = J.iters_j[j];
        worst = std::max(worst, st->shift_resid[j]);
    }
    st->true_resid = worst;
    st->status = status;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}
