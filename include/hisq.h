/*
 * hisq.h -- C ABI of libhisq: the even-odd HISQ staggered Dslash in low-bit
 * storage formats and the stabilised mixed-precision CG / multi-shift CG
 * solvers built on it, for AMD Instinct MI355X (gfx950).
 *
 * Paper: M. A. Clark, D. Howarth, J. Tu, M. Wagner, E. Weinberg,
 * "Maximizing the Bang Per Bit", arXiv:2302.09224 (Lattice 2022).
 *
 * Conventions for every call
 *  - Pointers marked (device) are HIP device pointers owned by the caller; the
 *    library never frees or reallocates them.  Pointers marked (host) are
 *    ordinary host memory.  Device pointers must be 16-byte aligned
 *    (HISQ_EALIGN otherwise).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Packing, unpacking and the Dslash calls (hisq_dslash, _xpay, _batched,
 *    _multi, hisq_normal_op) enqueue their device work on `stream` and return
 *    without waiting for it, with one exception: the first application of a
 *    launch-shape key (triplet, long-link storage, lattice, right-hand-side
 *    block) runs the autotuner, which times candidate shapes on `stream` into
 *    library-allocated scratch memory (hipMalloc/hipFree, so the device is
 *    synchronised) and waits for each timing before the real launch is
 *    enqueued.  HISQ_TUNE=0, hisq_tune_set and hisq_tune_load avoid it.
 *    Gauge packing synchronises `stream` (the scales are returned on the host).
 *    The solvers (hisq_cg_solve, hisq_multishift_cg_solve,
 *    hisq_cg_solve_batched, hisq_bicgstab_solve) run on a library-owned
 *    non-blocking stream of the current device (default priority), ordered
 *    after the work enqueued on `stream` before the call by an event (graphs
 *    cannot be captured on the null stream), and return after that stream has
 *    drained: the results are complete on return.  Calls of one solver on one
 *    device are serialised by a lock.
 *  - Errors are returned as hisq_status; no C++ exception crosses the ABI.
 *    hisq_last_error() gives a message for the calling thread's last error.
 *  - Lattice: dims = {X, Y, Z, T}, each even and >= 4; site index
 *    i = ((t*Z + z)*Y + y)*X + x; parity (x+y+z+t) & 1; the checkerboard
 *    index of a site within its parity is i >> 1; V = X*Y*Z*T, Vh = V/2.
 *  - Canonical FP64 fields (the interchange format at the ABI):
 *      links:   complex128 [4][V][3][3]  (direction mu = x,y,z,t; site; row; col)
 *      spinor:  complex128 [Vh][3]       (one parity, checkerboard order)
 *    complex128 = two doubles (re, im).  The staggered phases and the
 *    boundary signs are expected to be folded into the links already.
 *  - Packed fields (the formats the kernels stream) have a library-defined
 *    layout; create them only with hisq_gauge_pack / hisq_spinor_pack and read
 *    them back with hisq_spinor_unpack.  Their sizes are given by
 *    hisq_gauge_bytes / hisq_spinor_bytes.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HISQ_OK = 0,
    HISQ_EINVAL = -1,      /* bad argument (dims, format, sizes, null pointer) */
    HISQ_EALIGN = -2,      /* a device pointer is not 16-byte aligned */
    HISQ_EHIP = -3,        /* a HIP runtime call failed */
    HISQ_ENOCONV = -4,     /* solver hit maxiter; stats are filled, x is the best iterate */
    HISQ_EBREAKDOWN = -5,  /* solver breakdown: <p,Ap> <= 0 or a non-finite residual */
    HISQ_EWORKSPACE = -6,  /* workspace too small (see the *_workspace_bytes queries) */
    HISQ_ERANGE = -7,      /* a value exceeds what the storage format can hold */
    HISQ_EIO = -8          /* a field file cannot be opened, read or written, or is inconsistent */
} hisq_status;

/* Spinor (fermion) storage formats. */
enum {
    HISQ_SPINOR_F64 = 0,     /* IEEE FP64, 48 B/site */
    HISQ_SPINOR_F32 = 1,     /* IEEE FP32, 24 B/site */
    HISQ_SPINOR_HALF16 = 2,  /* QUDA half: 6 x int16 + FP32 site max, 16 B/site (Sec. 2, Listing 1) */
    HISQ_SPINOR_INT20 = 3,   /* 6 x 20-bit + 8-bit shared exponent, 16 B/site (Sec. 4, Listing 2, App. A) */
    HISQ_SPINOR_INT30 = 4,   /* 6 x 30-bit + 8-bit shared exponent, 24 B/site (Sec. 4, Listing 3) */
    HISQ_SPINOR_INT24 = 5    /* 6 x 24-bit + 8-bit shared exponent, 20 B/site: a member of the
                                Sec. 4 family generated from the same rule (FP32 encode, the
                                Appendix A word allocation); words 0-3 in a 16-B plane, word 4
                                in a 4-B plane after it.  Paired with FIX32 links, FP32 compute. */
};

/* Gauge (link) storage formats. */
enum {
    HISQ_GAUGE_F64 = 0,      /* IEEE FP64, 144 B/matrix */
    HISQ_GAUGE_F32 = 1,      /* IEEE FP32, 72 B/matrix */
    HISQ_GAUGE_FIX16 = 2,    /* 16-bit fixed point, global scale, 36 B/matrix (Sec. 2 footnote, Sec. 4) */
    HISQ_GAUGE_FIX32 = 3,    /* 32-bit fixed point, global scale, 72 B/matrix (Sec. 4) */
    HISQ_GAUGE_SX24 = 4      /* each row a 24-bit shared-exponent record (the spinor generator of
                                HISQ_SPINOR_INT24 applied to the three colour rows), 60 B/matrix:
                                words 0-3 of row r in 16-B plane r, word 4 in 4-B plane r after the
                                three 16-B planes; two-row long links 40 B.  No global scale. */
};

/* Precision triplet gauge / fermion / compute of one stencil application
 * (Sec. 4).  compute is 32 (FP32) or 64 (FP64).  Supported triplets:
 *   F64/F64/64, F32/F32/32, FIX16/HALF16/32, FIX16/INT20/32,
 *   FIX32/INT30/64, FIX32/INT30/32, FIX32/INT24/32, SX24/INT24/32, SX24/INT30/64. */
typedef struct {
    int gauge;
    int spinor;
    int compute;
} hisq_fmt;

/* Storage of the long (Naik) links: all 18 reals, two rows (12 reals) from
 * which the third is rebuilt, or eight parameters (Sec. 1, "Compression":
 * special unitary matrices have eight real degrees of freedom). */
#define HISQ_RECON_18 18
#define HISQ_RECON_12 12
#define HISQ_RECON_8 8

/* A packed pair of link fields, filled by hisq_gauge_pack / hisq_gauge_pack_recon. */
typedef struct {
    int dims[4];
    int fmt;              /* HISQ_GAUGE_* */
    const void *fat;      /* (device) packed one-link (fat) field */
    const void *lng;      /* (device) packed three-link (Naik) field */
    double fat_max;       /* global max |real component| of the fat field (fixed-point scale) */
    double long_max;      /* same for the long field (two-row storage: max |component| of U) */
    int long_recon;       /* HISQ_RECON_18, HISQ_RECON_12 or HISQ_RECON_8 */
    double long_coeff;    /* two-row storage: L_mu(x) = long_coeff * phase_mu(x) * U, U in SU(3) */
} hisq_gauge;

/* Bytes of ONE packed link field (fat or long): 4*V matrices. */
size_t hisq_gauge_bytes(const int dims[4], int gauge_fmt);

/* Bytes of the packed long field with HISQ_RECON_18, _12 or _8 storage (0 for
 * a format that has no such storage). */
size_t hisq_gauge_long_bytes(const int dims[4], int gauge_fmt, int long_recon);

/* Bytes of one packed single-parity spinor of `nsites` sites (Vh for a field). */
size_t hisq_spinor_bytes(long nsites, int spinor_fmt);

/* Pack canonical FP64 links into `gauge_fmt` and fill *g.
 * fat_src, long_src: (device) canonical complex128 [4][V][3][3].
 * fat_dst, long_dst: (device) hisq_gauge_bytes(dims, gauge_fmt) bytes each.
 * Fixed-point formats scale each field by its own global max real component
 * (Sec. 2 footnote); q = round-half-even(u * Q / max), Q = 2^15-1 or 2^31-1.
 * FP32 rounds to nearest.  Synchronises `stream` (the scales are returned in *g).
 * Errors: EINVAL (dims/format/null), EALIGN, ERANGE (non-finite link), EHIP. */
hisq_status hisq_gauge_pack(hisq_gauge *g, void *fat_dst, void *long_dst,
                            const double *fat_src, const double *long_src,
                            const int dims[4], int gauge_fmt, void *stream);

/* As hisq_gauge_pack, with the long links stored as two rows when
 * long_recon == HISQ_RECON_12 (long_dst: hisq_gauge_long_bytes bytes).  This
 * requires L_mu(x) = lambda * sigma * phase_mu(x) * U_mu(x) with U in SU(3),
 * lambda > 0 and sigma = +-1 global, phase_mu(x) the staggered phase
 * eta_mu(x) (eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 =
 * (-1)^(x+y+z)) times -1 for mu = t when t >= T-3 (antiperiodic time); HISQ
 * Naik links (-1/24 times a product of three SU(3) links) with the phases and
 * boundary folded in have this form.  The pack step verifies it (relative
 * tolerance: 1e-13 for F64, 1e-7 for F32, 1e-5 for FIX16, 1e-9 for FIX32 storage)
 * and returns HISQ_EINVAL otherwise.  The Dslash rebuilds row 3 = conj(row 1 x
 * row 2) in its compute precision, cutting the long-link traffic by a third.
 * long_recon == HISQ_RECON_8 (gauge_fmt F64 or FIX32 only, for the triplets
 * with FP64 arithmetic, F64/F64/64 and FIX32/INT30/64, and one right-hand side
 * per launch: hisq_dslash, _xpay, hisq_normal_op, the CG, multi-shift and
 * BiCGStab operators; batched and multi-lattice calls give HISQ_EINVAL): each
 * link keeps eight parameters of W = sigma * phase * L = lambda * U: Re/Im of
 * W01, W02, W10, then tan(arg(W00)/4) and tan(arg(W20)/4), each phase
 * parameter computed by a fixed sequence of correctly rounded operations
 * (cos = x/|z|, sin = y/|z|; cos >= 0: c2 = sqrt((1+cos)/2), s2 = sin/(2 c2);
 * else s2 = +-sqrt((1-cos)/2) with the sign of sin, c2 = |sin|/(2|s2|);
 * result s2/(1+c2)); FIX32 scales the entries by the long field's max |real
 * component| (long_max) and the phase parameters by 1.  F64: 64 B per link,
 * FIX32: 32 B (two 16-B planes: W01, W02 | W10, phases).  The Dslash rebuilds
 * U in FP64: |U00|^2 = 1 - N (N = |U01|^2 + |U02|^2), |U20|^2 = N - |U10|^2,
 * and the other four entries from the unitarity conditions divided by N, so
 * links with small N or small |U20| amplify the storage rounding (about 1/N
 * and 1/|U20|^2). */
hisq_status hisq_gauge_pack_recon(hisq_gauge *g, void *fat_dst, void *long_dst,
                                  const double *fat_src, const double *long_src,
                                  const int dims[4], int gauge_fmt, int long_recon, void *stream);

/* Pack `nsites` canonical FP64 colour vectors (device complex128 [nsites][3])
 * into `spinor_fmt` at dst (device, hisq_spinor_bytes bytes).
 * HALF16, INT20 and INT24 first round the values to FP32 (their compute
 * precision), INT30 works in FP64.  HALF16: per-site max M, q = rint(v * (32767/M)).
 * INT20/INT24/INT30: shared exponent E = (FP exponent of M/(2^(B-1)-1)) + 1,
 * q = rint(v * 2^(127-E)) (the packing of Appendix A; INT30 per Sec. 4). */
hisq_status hisq_spinor_pack(void *dst, const double *src, long nsites, int spinor_fmt, void *stream);

/* Inverse of hisq_spinor_pack: decode to device complex128 [nsites][3]. */
hisq_status hisq_spinor_unpack(double *dst, const void *src, long nsites, int spinor_fmt, void *stream);

/* The even-odd HISQ Dslash (the stencil of Secs. 1 and 5; Figs. 2-3):
 *   out(x) = sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^dag in(x-mu)
 *                   + L_mu(x) in(x+3mu) - L_mu(x-3mu)^dag in(x-3mu) ]
 * for every site x of parity `parity`; `in` holds the sites of parity
 * 1-parity.  in/out: (device) packed spinors in fmt.spinor (Vh sites each;
 * must not alias).  g: packed links, g->fmt == fmt.gauge.  The arithmetic is
 * done in fmt.compute after unpacking in registers; the result is packed
 * again into fmt.spinor.  Errors: EINVAL, EALIGN, EHIP. */
hisq_status hisq_dslash(void *out, const void *in, const hisq_gauge *g, int parity,
                        hisq_fmt fmt, void *stream);

/* out = a * x + b * Dslash(in), x (device, packed, parity `parity`) may be
 * NULL (then out = b * Dslash(in)).  Same rules as hisq_dslash. */
hisq_status hisq_dslash_xpay(void *out, const void *in, const hisq_gauge *g, int parity,
                             hisq_fmt fmt, double a, const void *x, double b, void *stream);

/* The even-site normal operator of the solvers (Sec. 3):
 *   out = (4 m^2 + shift) in - D_eo D_oe in
 * in/out: (device) packed even-parity spinors; tmp: (device) packed odd-parity
 * spinor of the same format (overwritten). */
hisq_status hisq_normal_op(void *out, const void *in, void *tmp, const hisq_gauge *g,
                           double mass, double shift, hisq_fmt fmt, void *stream);

/* hisq_normal_op for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operator without the tmp argument.  The odd-parity intermediate
 * D_oe in is kept in a library-owned device array of
 * HISQ_NOALLOC_SCRATCH_BYTES, which each device holds from the loading of the
 * library's device code until the process ends.  The call allocates nothing
 * (no hipMalloc/hipFree, no host memory), never runs the autotuner (launch
 * shapes already chosen by an earlier call, hisq_tune_set or hisq_tune_load,
 * else the default shapes) and reads no tune cache file.  Requires
 * hisq_spinor_bytes(Vh, fmt.spinor) <= HISQ_NOALLOC_SCRATCH_BYTES, which every
 * format of at most 24 B/site meets up to 48^3x96; HISQ_EINVAL otherwise,
 * before any device work.  Every call on one device shares that device's
 * array: calls that overlap in time on one device (other streams, other
 * threads) race and give wrong results, so serialise them.  Results equal
 * those of hisq_normal_op with the same launch shapes.  out, in: as for
 * hisq_normal_op (out must not alias in). */
#define HISQ_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
hisq_status hisq_normal_op_noalloc(void *out, const void *in, const hisq_gauge *g, double mass, double shift,
                                   hisq_fmt fmt, void *stream);

/* Batched Dslash (block of right-hand sides, Sec. 1 "Block solvers"): nrhs
 * consecutive packed fields in `in` and `out` (each hisq_spinor_bytes(Vh))
 * share one pass over the links.  1 <= nrhs <= 16.  Every triplet but
 * FIX32/INT30/32 (a refinement option only) has this form; that one, and
 * links with HISQ_RECON_8 long links, give HISQ_EINVAL. */
hisq_status hisq_dslash_batched(void *out, const void *in, const hisq_gauge *g, int parity,
                                hisq_fmt fmt, int nrhs, void *stream);

/* Several independent lattices in ONE launch (Sec. 1 "Block solvers": small
 * problems sharing the device, e.g. 8^4 + 12^4 + 16^4 + 24^4): lattice i gets
 * out[i] = D in[i] with its own packed links g[i] (its own dims), the same
 * triplet, parity and long-link storage for all.  out, in: (host) arrays of n
 * (device) packed spinors of lattice i's Vh sites; g: (host) array of n
 * descriptors.  1 <= n <= HISQ_MAX_LATTICES; every lattice has at most 2^31
 * sites.  Results are identical to n hisq_dslash calls. */
#define HISQ_MAX_LATTICES 8
hisq_status hisq_dslash_multi(int n, void *const *out, const void *const *in, const hisq_gauge *const *g,
                              int parity, hisq_fmt fmt, void *stream);

/* ------------------------------------------------------------------------ */
/* Solvers (Sec. 3)                                                          */
/* ------------------------------------------------------------------------ */

#define HISQ_MAX_SHIFTS 32
#define HISQ_MAX_GRAD_BUFFER 16

typedef struct {
    double delta;        /* reliable update when |r| < delta * max|r| since the last one (Sec. 3 footnote: 0.1);
                            <= 0 disables reliable updates (the residual is only checked at the end) */
    int maxiter;         /* iteration cap per solve (per phase for multi-shift) */
    int grad_buffer;     /* gradient vectors buffered before the FP64 solution update (Sec. 3.1 item 1), 1..16;
                            default 8 */
    int pr_beta;         /* 1: Polak-Ribiere beta (Sec. 3.1 item 3); 0: Fletcher-Reeves */
    int reproject;       /* 1: re-project the gradient vector at each reliable update (Sec. 3.1 item 2) */
    int poll_every;      /* iterations enqueued between host polls of the device state (rounded up to a
                            multiple of grad_buffer); 0 = default */
    int use_graph;       /* 1: replay each block of iterations as a captured hipGraph */
    double shift_floor;  /* multi-shift: a shifted system stops updating once its iterated residual is below
                            max(tol_i, shift_floor) (Sec. 3.2: the shifts stop at the sloppy precision's
                            limit); <= 0 selects that limit: none (tol_i alone) for triplets with FP64
                            arithmetic, the spinor format's epsilon for FP32 arithmetic */
    int batch_refine;    /* multi-shift: refine the shifted systems together, one Dslash per iteration shared
                            by up to 16 of them (1), or one after another (0), the base refined first.
                            2: as 1, but the batch runs on a second library stream while a host thread refines
                            the base concurrently on the first (every launch shape planned beforehand);
                            phase_seconds[1] and [2] then overlap; 3: the base joins the first block as its
                            system 0, still continuing its gradient vector (phase_seconds[1] is then 0) */
    int ru_estimate;     /* CG and the multi-shift base: 0 = reliable update when |r| drops below delta times its
                            maximum since the last one; 1 = when an estimate of |r_true - r_iterated| (each
                            iteration's sloppy roundoff, accumulated in quadrature: residual replacement in the
                            manner of van der Vorst and Ye; Sec. 3 footnote) crosses sqrt(eps_sloppy) |r|.  The batched CG and BiCGStab
                            use the delta rule. */
} hisq_solver_params;

typedef struct {
    int status;                 /* hisq_status of the solve */
    int iters;                  /* sloppy iterations (multi-shift: multi-shift phase) */
    int reliable_updates;
    int dslash_sloppy;          /* sloppy Dslash applications */
    int dslash_f64;             /* FP64 Dslash applications */
    double true_resid;          /* final |b - A x| / |b| (multi-shift: max over shifts of resid/tol_i * tol_0) */
    double seconds;             /* wall-clock of the solve */
    double alg_bytes;           /* algorithmic HBM bytes of all kernels of the solve */
    int nshift;
    int shift_iters[HISQ_MAX_SHIFTS];        /* multi-shift phase iteration at which shift i stopped */
    double shift_resid_ms[HISQ_MAX_SHIFTS];  /* true residual of shift i after the multi-shift phase */
    int refine_iters[HISQ_MAX_SHIFTS];       /* refinement CG iterations of shift i */
    double shift_resid[HISQ_MAX_SHIFTS];     /* final true residual of shift i */
    double phase_seconds[3];                 /* multi-shift: wall time of the multi-shift phase, of the base's
                                                refinement and of the shifted systems' refinement */
} hisq_solver_stats;

/* Default parameters: delta 0.1, maxiter 100000, grad_buffer 8, PR beta,
 * re-projection on, poll_every 32, graphs on, shift_floor 0 (auto), batch_refine 3, ru_estimate 0. */
void hisq_solver_params_default(hisq_solver_params *p);

/* Workspace bytes for hisq_cg_solve on `dims` with sloppy format `sloppy`. */
size_t hisq_cg_workspace_bytes(const int dims[4], hisq_fmt sloppy, const hisq_solver_params *p);

/* Mixed-precision CG (Sec. 3.1) for (4m^2 + shift - D_eo D_oe) x = b on the
 * even sites:  the iterated residual and gradient vectors live in
 * sloppy.spinor, the Dslash runs in the sloppy triplet; the solution is
 * accumulated in FP64 from buffered gradient vectors; reliable updates
 * recompute the true residual with the FP64 operator (g64, F64/F64/64) and
 * re-project the gradient vector; beta is Polak-Ribiere.  Stops when the
 * true relative residual |b - A x|/|b| <= tol.
 * x: (device) canonical complex128 [Vh][3], initial guess in, solution out.
 * b: (device) canonical complex128 [Vh][3].
 * g64: links packed as HISQ_GAUGE_F64; gs: links packed as sloppy.gauge.
 * ws: (device) workspace of at least hisq_cg_workspace_bytes bytes.
 * stats: (host) filled on return, may be NULL.
 * Errors: EINVAL, EALIGN, EWORKSPACE, ENOCONV, EBREAKDOWN, EHIP. */
hisq_status hisq_cg_solve(double *x, const double *b, const hisq_gauge *g64, const hisq_gauge *gs,
                          double mass, double shift, double tol, hisq_fmt sloppy,
                          const hisq_solver_params *p, void *ws, size_t ws_bytes,
                          hisq_solver_stats *stats, void *stream);

/* Workspace bytes for hisq_multishift_cg_solve. */
size_t hisq_multishift_workspace_bytes(const int dims[4], int nshift, hisq_fmt ms_fmt,
                                       hisq_fmt refine_fmt, const hisq_solver_params *p);

/* Mixed-precision multi-shift CG with post-solve refinement (Sec. 3.2):
 * x_i = (4m^2 + shift_i - D_eo D_oe)^-1 b for i = 0..nshift-1.  One Krylov
 * space of the base system (shift_0, the smallest) built in the ms_fmt
 * triplet with reliable updates on the base only; the shifted solutions
 * (FP64) and gradient vectors are updated once per block of grad_buffer
 * iterations, all shifts in one launch, from the block's base residuals;
 * shift i stops updating when its iterated residual reaches
 * max(tol_i, shift_floor); the phase ends when every shift i >= 1 has
 * stopped.  Then CG refinement in the refine_fmt triplet: the base keeping
 * its gradient vector, every shift from a clean restart, each to its own
 * tol_i (true residual).  By default (p->batch_refine 3, refine triplets other
 * than FIX32/INT30/FP32) all of them as blocks of up to 16 independent CGs
 * sharing every Dslash (each the iteration of a lone solve, with its own
 * reliable updates), the base in the first block; otherwise the base first,
 * then the shifts in ascending order (batch_refine 0) or as such blocks
 * (1, or 2 concurrently with the base).
 * x: (host) array of nshift (device) canonical complex128 [Vh][3] outputs.
 * shifts, tol: (host) arrays of nshift doubles, shifts strictly ascending,
 * shifts[0] >= 0 and 1 <= nshift <= HISQ_MAX_SHIFTS.
 * g64: F64 links; g_ms: links in ms_fmt.gauge; g_ref: links in refine_fmt.gauge.
 * Errors as hisq_cg_solve. */
hisq_status hisq_multishift_cg_solve(double *const *x, const double *b, const double *shifts,
                                     int nshift, const double *tol, const hisq_gauge *g64,
                                     const hisq_gauge *g_ms, const hisq_gauge *g_ref, double mass,
                                     hisq_fmt ms_fmt, hisq_fmt refine_fmt,
                                     const hisq_solver_params *p, void *ws, size_t ws_bytes,
                                     hisq_solver_stats *stats, void *stream);

/* Workspace bytes for hisq_bicgstab_solve (0 for unsupported arguments). */
#define HISQ_MAX_BICGSTAB_L 8
size_t hisq_bicgstab_workspace_bytes(const int dims[4], int l, hisq_fmt sloppy);

/* Mixed-precision BiCGStab(l) (Sec. 6.1, the solver of Sleijpen and Fokkema)
 * for M x = b on the WHOLE lattice, M = 2m + D (D the HISQ Dslash of both
 * parities; M^dag M restricted to even sites is the CG operator above).
 * x, b: (device) canonical complex128 [V][3], all sites in lexicographic order
 * (x: initial guess in, solution out).  The Krylov vectors r_0..r_l, u_0..u_l
 * and the shadow residual are stored in the sloppy triplet (links gs); the
 * solution is accumulated in FP64; a reliable update replaces r_0 by b - M x
 * from the FP64 operator (links g64) whenever |r_0| drops below p->delta times
 * its maximum since the previous one, or meets tol.  Converged when the FP64
 * true residual |b - M x| <= tol |b|.  1 <= l <= HISQ_MAX_BICGSTAB_L, mass > 0.
 * stats: iters = operator applications (2 per BiCG step), reliable_updates,
 * true_resid, seconds.  p->maxiter bounds the operator applications
 * (HISQ_ENOCONV beyond, x is the last iterate); HISQ_EBREAKDOWN when a BiCG
 * or minimal-residual denominator vanishes.  Runs on a library-owned stream
 * ordered after `stream` and returns when x is written: every scalar of the
 * method is formed on the device, each cycle (l BiCG steps and the
 * minimal-residual step) is enqueued as a whole (replayed as a captured
 * hipGraph when p->use_graph) and followed by one synchronisation, where the
 * reliable-update decision is taken. */
hisq_status hisq_bicgstab_solve(double *x, const double *b, const hisq_gauge *g64, const hisq_gauge *gs,
                                double mass, double tol, int l, hisq_fmt sloppy,
                                const hisq_solver_params *p, void *ws, size_t ws_bytes,
                                hisq_solver_stats *stats, void *stream);

/* Workspace bytes for hisq_cg_solve_batched. */
size_t hisq_cg_batched_workspace_bytes(const int dims[4], int nrhs, hisq_fmt sloppy,
                                       const hisq_solver_params *p);

/* nrhs independent mixed-precision CG solves (same operator, different right-hand
 * sides) that share every Dslash launch, so each link is loaded once per
 * application for the whole block (Sec. 1 "Block solvers").  x, b: (device)
 * nrhs consecutive canonical complex128 [Vh][3] fields.  Each right-hand side
 * converges to tol on its own, with its own reliable updates, and stops
 * costing Dslash work once converged; stats describe the slowest one
 * (shift_resid[j], refine_iters[j]: right-hand side j).  1 <= nrhs <= 16. */
hisq_status hisq_cg_solve_batched(double *x, const double *b, int nrhs, const hisq_gauge *g64,
                                  const hisq_gauge *gs, double mass, double shift, double tol,
                                  hisq_fmt sloppy, const hisq_solver_params *p, void *ws,
                                  size_t ws_bytes, hisq_solver_stats *stats, void *stream);

/* Launch shapes chosen by the Dslash autotuner so far (one text line per
 * triplet, long-link storage, lattice and right-hand-side block: right-hand sides per lane, lanes
 * per site, hops per load stage, block size, measured time).  Writes at most
 * len bytes (NUL-terminated) into buf if buf is not NULL; returns the size the
 * full report needs.  The autotuner times each candidate shape with HIP events
 * on the first application of a shape key (never inside stream capture);
 * environment HISQ_TUNE=0 selects fixed defaults instead. */
size_t hisq_tune_report(char *buf, size_t len);

/* ---------------------------------------------------------------------------
 * Offline storage of packed fields (Sec. 7 outlook: gauge fields and
 * propagators kept on disk in the bit-packed formats).  A file holds a
 * 128-byte header (magic "HISQPK01", field kind, format, lattice extents or
 * site count, long-link storage, the gauge scales, payload sizes and an
 * FNV-1a checksum over 64-bit words of the payload) followed by the packed
 * device bytes verbatim (gauge: fat links, then long links), so a field
 * comes back bit for bit without being unpacked.  Copies go through a
 * 64 MiB pinned staging buffer on `stream`; the calls return when the file
 * is complete (save) or the device holds the field (load).  A file whose
 * header is malformed, whose length differs from its header or whose
 * checksum does not match gives HISQ_EIO (after a checksum mismatch the
 * destination holds the file's bytes); a file that is well formed but holds
 * another kind, format or size than asked gives HISQ_EINVAL.
 * ------------------------------------------------------------------------- */
enum { HISQ_FIELD_SPINOR = 1, HISQ_FIELD_GAUGE = 2 };

typedef struct {
    int kind;        /* HISQ_FIELD_SPINOR or HISQ_FIELD_GAUGE */
    int fmt;         /* spinor or gauge storage format */
    int dims[4];     /* gauge: lattice extents; spinor: zeros */
    long nsites;     /* spinor: sites; gauge: lattice volume */
    int long_recon;  /* gauge: HISQ_RECON_18 or HISQ_RECON_12 */
    size_t bytes0;   /* spinor payload or fat-link payload */
    size_t bytes1;   /* long-link payload (0 for a spinor) */
} hisq_field_header;

/* Read the header of `path` (host string) into *info: what to allocate
 * before hisq_spinor_load / hisq_gauge_load. */
hisq_status hisq_field_info(const char *path, hisq_field_header *info);

/* Write the packed spinor field src (device, hisq_spinor_bytes(nsites,
 * spinor_fmt) bytes) to `path`, replacing the file. */
hisq_status hisq_spinor_save(const char *path, const void *src, long nsites, int spinor_fmt, void *stream);

/* Read a spinor file into dst (device, hisq_spinor_bytes(nsites, spinor_fmt)
 * bytes); the file must hold exactly nsites sites in spinor_fmt. */
hisq_status hisq_spinor_load(const char *path, void *dst, long nsites, int spinor_fmt, void *stream);

/* Write the packed links of g (filled by hisq_gauge_pack or hisq_gauge_load)
 * with their scales and long-link storage to `path`. */
hisq_status hisq_gauge_save(const char *path, const hisq_gauge *g, void *stream);

/* Read a gauge file into fat_dst and long_dst (device buffers of fat_bytes
 * and long_bytes, at least the file's bytes0 and bytes1) and fill *g as
 * hisq_gauge_pack would have. */
hisq_status hisq_gauge_load(const char *path, hisq_gauge *g, void *fat_dst, size_t fat_bytes,
                            void *long_dst, size_t long_bytes, void *stream);

/* Fix the launch shape of the Dslash for triplet fmt on lattice dims with long
 * links stored as long_recon (HISQ_RECON_18, _12 or _8; _8 with rhs_block 1) and a block of
 * rhs_block right-hand sides (1, 2, 4, 8 or 16), replacing what the
 * autotuner chose or would choose: nr right-hand sides per lane and rg lanes
 * per site (nr * rg == rhs_block, both powers of two), stage hops per load
 * stage (1, 2, 4, 8, -1 or -2 when nr == 1; 1 or -1 when 1 < nr <= 8; 1 when
 * nr == 16; -1 and -2: one or two hops per stage, double-buffered, the next
 * stage's loads issued before the current stage's arithmetic; 5: the
 * matrix-core path, rg == 4 and nr <= 4, FP32-arithmetic triplets only),
 * block threads (128 or 256),
 * grid blocks (0: one tile of lanes per block; otherwise a multiple of 8,
 * a persistent grid when smaller than the tile count) and sweep, the order in
 * which the blocks take the tiles of lanes (0: the blocks of XCD k, b % 8 ==
 * k, take the k-th eighth of the lattice; 1: consecutive tiles on consecutive
 * blocks, so all XCDs work on neighbouring sites; 2: XCD k owns the z-slab
 * [Z k/8, Z (k+1)/8) of every time slice and walks it slice by slice in t
 * order).  For rhs_block > 1 the
 * shape serves both the plain launches and those that fuse a reduction (which
 * the autotuner otherwise tunes apart).  For reproducible launch shapes and
 * for tests.  HISQ_EINVAL for an unsupported shape. */
hisq_status hisq_tune_set(hisq_fmt fmt, const int dims[4], int long_recon, int rhs_block, int nr, int rg,
                          int stage, int block, int grid, int sweep);

/* As hisq_tune_set, but only for the launches that fuse a reduction (the
 * second Dslash of a batched solver's normal operator, the reliable-update
 * residual norms), which the autotuner otherwise tunes apart from the plain
 * launches of the same block; rhs_block 2..16.  Call it after hisq_tune_set
 * for the same key (hisq_tune_set pins both).  HISQ_EINVAL for an unsupported
 * shape or rhs_block 1. */
hisq_status hisq_tune_set_fused(hisq_fmt fmt, const int dims[4], int long_recon, int rhs_block, int nr, int rg,
                                int stage, int block, int grid, int sweep);

/* Forget every tuned or fixed launch shape (the next application tunes again). */
void hisq_tune_clear(void);

/* Tune cache files.  hisq_tune_save writes every launch shape of the table
 * (tuned, fixed or loaded) to `path` (host string), one text line per key:
 *   hisq-tune 1 <arch> <HIP runtime version> <key: gauge*10000 + spinor*1000 +
 *   (compute == 64)*100 + long_recon> X Y Z T <rhs block> <fused 0|1> :
 *   nr rg stage block grid sweep <microseconds, -1000 if not timed>
 * hisq_tune_load reads such a file and enters the lines whose architecture
 * and HIP runtime version match the current device (others are skipped) into
 * the table, replacing entries of the same key; *nloaded (may be NULL)
 * receives their count.  Both need a current HIP device (HISQ_EHIP
 * otherwise); HISQ_EIO for a file that cannot be read or written, a
 * malformed line or a shape the kernels do not have (then nothing is loaded).
 * With the environment variable HISQ_TUNE_CACHE=<path>, the file is loaded at
 * the first shape lookup of the process (if it exists; keys already fixed by
 * hisq_tune_set or hisq_tune_load keep their shapes) and every shape the
 * autotuner chooses afterwards is appended to it, so later processes on the
 * same device and runtime do not tune again. */
hisq_status hisq_tune_save(const char *path);
hisq_status hisq_tune_load(const char *path, int *nloaded);

/* Thread-local message of the calling thread's last non-OK status. */
const char *hisq_last_error(void);

/* Library version string. */
const char *hisq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
