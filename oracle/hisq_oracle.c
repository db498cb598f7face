/*
 * hisq_oracle.c -- plain, slow, FP64 CPU oracle for the HISQ hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this file; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no code, header, table or helper with the HIP implementation.
 *
 * Contents, each written from its definition:
 *   - the HISQ staggered operator D (one-link "fat" + three-link "Naik" hops,
 *     phases folded into the links) and its even-odd normal operator
 *     A = 4m^2 + sigma - D_pq D_qp.  The paper names this operator (abstract,
 *     Sec. 1, Sec. 5.2 and the captions of Figs. 2-3) but does not print it;
 *     the standard form is used:
 *       (D psi)(x) = sum_mu [ F_mu(x) psi(x+mu) - F_mu(x-mu)^dag psi(x-mu)
 *                           + L_mu(x) psi(x+3mu) - L_mu(x-3mu)^dag psi(x-3mu) ]
 *     with periodic site arithmetic (boundary signs live in the links);
 *   - plain FP64 conjugate gradient on A (its result is x = A^-1 b);
 *   - FP64 multi-shift CG (Sec. 3.2: one Krylov space, shifted residuals kept
 *     co-linear with the base residual; recurrences of the reference the
 *     paper cites for multi-shift solvers);
 *   - the storage codecs: QUDA half (Sec. 2, Listing 1), the 20-bit
 *     shared-exponent spinor (Sec. 4 Listing 2, packing rules of Appendix A),
 *     the 30-bit shared-exponent spinor (Sec. 4 Listing 3) and the 16/32-bit
 *     fixed-point gauge formats (Sec. 2 footnote, Sec. 4).
 *
 * Layouts (canonical, shared with the library's ABI by definition only):
 *   dims = {X,Y,Z,T}, all even; site i = ((t*Z+z)*Y+y)*X+x;
 *   parity (x+y+z+t)&1; links complex [4][V][3][3]; spinors complex [V][3].
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* lattice geometry                                                          */
/* ------------------------------------------------------------------------ */

static void site_to_coords(long i, const int *d, int *c)
{
    c[0] = (int)(i % d[0]); i /= d[0];
    c[1] = (int)(i % d[1]); i /= d[1];
    c[2] = (int)(i % d[2]); i /= d[2];
    c[3] = (int)i;
}

static long coords_to_site(const int *c, const int *d)
{
    return ((long)(c[3] * d[2] + c[2]) * d[1] + c[1]) * d[0] + c[0];
}

/* site reached from i by `hop` steps (hop in {-3,-1,+1,+3}) along mu */
static long hop_site(long i, int mu, int hop, const int *d)
{
    int c[4];
    site_to_coords(i, d, c);
    c[mu] = ((c[mu] + hop) % d[mu] + d[mu]) % d[mu];
    return coords_to_site(c, d);
}

static int site_parity(long i, const int *d)
{
    int c[4];
    site_to_coords(i, d, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static long lattice_volume(const int *d) { return (long)d[0] * d[1] * d[2] * d[3]; }

/* threads the site loops use (OpenMP) */
int hisq_oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

/* tan(arg(x + iy)/4), 0 at the origin: the phase parameter of the
 * eight-parameter long-link storage, by one fixed sequence of correctly
 * rounded operations (r = sqrt(fma(x, x, y*y)), cos = x/r, sin = y/r; cos >= 0:
 * c2 = sqrt((1 + cos)/2), s2 = sin/(2 c2); else s2 = sqrt((1 - cos)/2) with the
 * sign of sin, c2 = |sin|/(2|s2|); result s2/(1 + c2)), from the half-angle
 * identities, so that every implementation stores the same bits. */
void hisq_oracle_phase_params(const double *x, const double *y, double *v, long n)
{
    for (long k = 0; k < n; k++) {
        double r = sqrt(fma(x[k], x[k], y[k] * y[k]));
        if (r == 0.0) {
            v[k] = 0.0;
            continue;
        }
        double c = x[k] / r, sn = y[k] / r, ch, sh;
        if (c >= 0.0) {
            ch = sqrt((1.0 + c) * 0.5);
            sh = sn / (2.0 * ch);
        } else {
            double sa = sqrt((1.0 - c) * 0.5);
            sh = copysign(sa, sn);
            ch = fabs(sn) / (2.0 * sa);
        }
        v[k] = sh / (1.0 + ch);
    }
}

/* set the number of threads of the site loops (n >= 1) */
void hisq_oracle_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

/* link matrix of direction mu at site i: row-major 3x3 */
static const cplx *link(const cplx *field, int mu, long i, long V)
{
    return field + ((long)mu * V + i) * 9;
}

/* y += s * U v */
static void add_mv(cplx *y, double s, const cplx *U, const cplx *v)
{
    for (int a = 0; a < 3; a++) {
        cplx acc = 0;
        for (int b = 0; b < 3; b++) acc += U[3 * a + b] * v[b];
        y[a] += s * acc;
    }
}

/* y += s * U^dagger v */
static void add_mdv(cplx *y, double s, const cplx *U, const cplx *v)
{
    for (int a = 0; a < 3; a++) {
        cplx acc = 0;
        for (int b = 0; b < 3; b++) acc += conj(U[3 * b + a]) * v[b];
        y[a] += s * acc;
    }
}

/* (D psi)(x) at one site, written out term by term */
static void dslash_site(cplx *out3, const cplx *fat, const cplx *lng, const cplx *in,
                        long x, const int *d, long V)
{
    cplx acc[3] = {0, 0, 0};
    for (int mu = 0; mu < 4; mu++) {
        long xp1 = hop_site(x, mu, +1, d);
        long xm1 = hop_site(x, mu, -1, d);
        long xp3 = hop_site(x, mu, +3, d);
        long xm3 = hop_site(x, mu, -3, d);
        add_mv(acc, +1.0, link(fat, mu, x, V), in + 3 * xp1);
        add_mdv(acc, -1.0, link(fat, mu, xm1, V), in + 3 * xm1);
        add_mv(acc, +1.0, link(lng, mu, x, V), in + 3 * xp3);
        add_mdv(acc, -1.0, link(lng, mu, xm3, V), in + 3 * xm3);
    }
    for (int a = 0; a < 3; a++) out3[a] = acc[a];
}

/* out = D in on the sites of `parity` (all sites if parity < 0); sites of the
 * other parity are left untouched. */
void hisq_oracle_dslash(cplx *out, const cplx *fat, const cplx *lng, const cplx *in,
                        const int *dims, int parity)
{
    long V = lattice_volume(dims);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) {
        if (parity >= 0 && site_parity(x, dims) != parity) continue;
        dslash_site(out + 3 * x, fat, lng, in, x, dims, V);
    }
}

/* out[k] = (D in)(sites[k]) for an explicit list of sites (sampled checks) */
void hisq_oracle_dslash_sites(cplx *out, const cplx *fat, const cplx *lng, const cplx *in,
                              const int *dims, const int64_t *sites, long n)
{
    long V = lattice_volume(dims);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; k++) dslash_site(out + 3 * k, fat, lng, in, (long)sites[k], dims, V);
}

/* ------------------------------------------------------------------------ */
/* even-odd normal operator and FP64 solvers                                 */
/* ------------------------------------------------------------------------ */

/* out = c*in - D_pq D_qp in, with c = 4m^2 + sigma, on parity p; `in` must
 * vanish off parity p; tmp holds D_qp in.  Sites off parity p are zeroed. */
void hisq_oracle_normal(cplx *out, const cplx *in, cplx *tmp, const cplx *fat, const cplx *lng,
                        const int *dims, int parity, double c)
{
    long V = lattice_volume(dims);
    hisq_oracle_dslash(tmp, fat, lng, in, dims, 1 - parity);
    hisq_oracle_dslash(out, fat, lng, tmp, dims, parity);
    for (long x = 0; x < V; x++) {
        int on = site_parity(x, dims) == parity;
        for (int a = 0; a < 3; a++)
            out[3 * x + a] = on ? c * in[3 * x + a] - out[3 * x + a] : 0.0;
    }
}

static double norm2(const cplx *a, long n)
{
    double s = 0.0;
    for (long k = 0; k < n; k++) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return s;
}

static double redot(const cplx *a, const cplx *b, long n)
{
    double s = 0.0;
    for (long k = 0; k < n; k++) s += creal(a[k]) * creal(b[k]) + cimag(a[k]) * cimag(b[k]);
    return s;
}

/* relative true residual |b - (A+shift) x| / |b| */
double hisq_oracle_true_residual(const cplx *x, const cplx *b, const cplx *fat, const cplx *lng,
                                 const int *dims, int parity, double mass, double shift)
{
    long V = lattice_volume(dims), n = 3 * V;
    cplx *ax = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    memset(tmp, 0, sizeof(cplx) * n);
    memset(ax, 0, sizeof(cplx) * n);
    hisq_oracle_normal(ax, x, tmp, fat, lng, dims, parity, 4.0 * mass * mass + shift);
    double r2 = 0.0;
    for (long k = 0; k < n; k++) {
        cplx r = b[k] - ax[k];
        r2 += creal(r) * creal(r) + cimag(r) * cimag(r);
    }
    double b2 = norm2(b, n);
    free(ax);
    free(tmp);
    return b2 > 0 ? sqrt(r2 / b2) : sqrt(r2);
}

/* Plain FP64 CG on (A + shift) x = b, parity p.  x: initial guess in,
 * solution out.  Stops when the iterated |r| <= tol |b|.  Returns 0 if the
 * true residual then meets tol, 1 otherwise (maxiter or drift). */
int hisq_oracle_cg(cplx *x, const cplx *b, const cplx *fat, const cplx *lng, const int *dims,
                   int parity, double mass, double shift, double tol, int maxiter,
                   int *iters_out, double *true_resid_out)
{
    long V = lattice_volume(dims), n = 3 * V;
    double c = 4.0 * mass * mass + shift;
    cplx *r = calloc(n, sizeof(cplx)), *p = calloc(n, sizeof(cplx));
    cplx *ap = calloc(n, sizeof(cplx)), *tmp = calloc(n, sizeof(cplx));
    hisq_oracle_normal(ap, x, tmp, fat, lng, dims, parity, c);
    for (long k = 0; k < n; k++) { r[k] = b[k] - ap[k]; p[k] = r[k]; }
    double b2 = norm2(b, n), rr = norm2(r, n), stop = tol * tol * b2;
    int it = 0;
    while (rr > stop && it < maxiter) {
        hisq_oracle_normal(ap, p, tmp, fat, lng, dims, parity, c);
        double alpha = rr / redot(p, ap, n);
        for (long k = 0; k < n; k++) { x[k] += alpha * p[k]; r[k] -= alpha * ap[k]; }
        double rr_new = norm2(r, n);
        double beta = rr_new / rr;
        for (long k = 0; k < n; k++) p[k] = r[k] + beta * p[k];
        rr = rr_new;
        it++;
    }
    double res = hisq_oracle_true_residual(x, b, fat, lng, dims, parity, mass, shift);
    if (iters_out) *iters_out = it;
    if (true_resid_out) *true_resid_out = res;
    free(r); free(p); free(ap); free(tmp);
    return res <= tol ? 0 : 1;
}

/* FP64 multi-shift CG: x_i = (A + shift_i)^-1 b for i = 0..nshift-1, all from
 * the Krylov space of the base system A + shift_0 (shift_0 = smallest).
 * Shift i stops updating once |zeta_i| |r| <= tol_i |b|; the solve ends when
 * every system has stopped or after maxiter iterations.
 *
 * Base iteration (any two-term CG):  r' = r - a A0 p,  p' = r' + b p.
 * Shifted systems, s_i = shift_i - shift_0, residual r_i = zeta_i r:
 *   zeta_i' = zeta_i zeta_i_prev a_prev /
 *             ( a_prev zeta_i_prev (1 + a s_i) + a b_prev (zeta_i_prev - zeta_i) )
 *   a_i = a zeta_i'/zeta_i,   x_i += a_i p_i,
 *   b_i = b (zeta_i'/zeta_i)^2,  p_i = zeta_i' r' + b_i p_i
 * with zeta_i = zeta_i_prev = 1, a_prev = 1, b_prev = 0 at the start, x_i = 0.
 *
 * Optional outputs: zeta_out[i] (final zeta_i), r_out (final base iterated
 * residual), iters_out[i] (iteration at which shift i stopped). */
int hisq_oracle_multishift_cg(cplx **x, const cplx *b, const cplx *fat, const cplx *lng,
                              const int *dims, int parity, double mass, const double *shifts,
                              int nshift, const double *tol, int maxiter, int *iters_out,
                              double *true_resid_out, double *zeta_out, cplx *r_out)
{
    long V = lattice_volume(dims), n = 3 * V;
    double c0 = 4.0 * mass * mass + shifts[0];
    cplx *r = calloc(n, sizeof(cplx)), *ap = calloc(n, sizeof(cplx)), *tmp = calloc(n, sizeof(cplx));
    cplx **p = malloc(sizeof(cplx *) * nshift);
    double *z = malloc(sizeof(double) * nshift), *zp = malloc(sizeof(double) * nshift);
    int *active = malloc(sizeof(int) * nshift);
    for (int i = 0; i < nshift; i++) {
        p[i] = malloc(sizeof(cplx) * n);
        memcpy(p[i], b, sizeof(cplx) * n);
        memset(x[i], 0, sizeof(cplx) * n);
        z[i] = zp[i] = 1.0;
        active[i] = 1;
        if (iters_out) iters_out[i] = 0;
    }
    memcpy(r, b, sizeof(cplx) * n);
    double b2 = norm2(b, n), rr = b2, a_prev = 1.0, b_prev = 0.0;
    int it = 0, nactive = nshift;
    while (nactive > 0 && it < maxiter) {
        /* base step: p[0] is the base gradient vector */
        hisq_oracle_normal(ap, p[0], tmp, fat, lng, dims, parity, c0);
        double a = rr / redot(p[0], ap, n);
        for (long k = 0; k < n; k++) r[k] -= a * ap[k];
        double rr_new = norm2(r, n);
        double bb = rr_new / rr;
        for (int i = 0; i < nshift; i++) {
            /* the base gradient vector p[0] drives the Krylov space and is
             * updated until the end, even after x[0] has converged */
            if (!active[i] && i != 0) continue;
            int upd_x = active[i];
            double s = shifts[i] - shifts[0];
            double znew = z[i] * zp[i] * a_prev /
                          (a_prev * zp[i] * (1.0 + a * s) + a * b_prev * (zp[i] - z[i]));
            double ai = a * znew / z[i];
            double bi = bb * (znew / z[i]) * (znew / z[i]);
            for (long k = 0; k < n; k++) {
                if (upd_x) x[i][k] += ai * p[i][k];
                p[i][k] = znew * r[k] + bi * p[i][k];
            }
            zp[i] = z[i];
            z[i] = znew;
        }
        a_prev = a;
        b_prev = bb;
        rr = rr_new;
        it++;
        for (int i = 0; i < nshift; i++) {
            if (active[i] && z[i] * z[i] * rr <= tol[i] * tol[i] * b2) {
                active[i] = 0;
                nactive--;
                if (iters_out) iters_out[i] = it;
            }
        }
    }
    for (int i = 0; i < nshift; i++) {
        if (active[i] && iters_out) iters_out[i] = it;
        if (true_resid_out)
            true_resid_out[i] = hisq_oracle_true_residual(x[i], b, fat, lng, dims, parity, mass, shifts[i]);
        if (zeta_out) zeta_out[i] = z[i];
    }
    if (r_out) memcpy(r_out, r, sizeof(cplx) * n);
    int bad = 0;
    if (true_resid_out)
        for (int i = 0; i < nshift; i++) bad |= !(true_resid_out[i] <= tol[i]);
    for (int i = 0; i < nshift; i++) free(p[i]);
    free(p); free(z); free(zp); free(active); free(r); free(ap); free(tmp);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* storage codecs                                                            */
/* ------------------------------------------------------------------------ */

static uint32_t f32_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float f32_from_bits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* two's-complement B-bit field -> signed integer */
static int64_t sign_extend(uint64_t u, int bits)
{
    uint64_t m = (1ull << bits) - 1, sb = 1ull << (bits - 1);
    return (int64_t)((u & m) ^ sb) - (int64_t)sb;
}

/* QUDA half spinor (Sec. 2, Listing 1): six int16 and the site max |component|.
 * q = round-to-nearest-even(v * (32767/max)); decode v = q * (max/32767), the
 * quotient max/32767 rounded to FP32 once per site, then one FP32 product per
 * component.  A site whose max is zero, or whose 32767/max overflows FP32,
 * stores zeros with max 0.  Inputs are FP32 (the format's compute precision). */
void hisq_oracle_half16_encode(const float *v, int16_t *q, float *norm, long nsites)
{
    for (long s = 0; s < nsites; s++) {
        const float *a = v + 6 * s;
        float m = fabsf(a[0]);
        for (int k = 1; k < 6; k++) m = fmaxf(m, fabsf(a[k]));
        float c = 32767.0f / m;
        if (!(m > 0.0f) || !isfinite(c)) {
            norm[s] = 0.0f;
            for (int k = 0; k < 6; k++) q[6 * s + k] = 0;
            continue;
        }
        norm[s] = m;
        for (int k = 0; k < 6; k++) q[6 * s + k] = (int16_t)lrintf(a[k] * c);
    }
}

void hisq_oracle_half16_decode(const int16_t *q, const float *norm, float *v, long nsites)
{
    for (long s = 0; s < nsites; s++) {
        float d = norm[s] / 32767.0f;
        for (int k = 0; k < 6; k++) v[6 * s + k] = (float)q[6 * s + k] * d;
    }
}

/* 20-bit shared-exponent spinor (Sec. 4 Listing 2; packing of Appendix A).
 * max M over the six |components| (FP32); t = M/(2^19-1) in FP32; the stored
 * exponent E is t's biased FP32 exponent plus one (mantissa dropped, i.e. t
 * rounded up to a power of two), clamped to [1,254]; q_k = rint(v_k * 2^(127-E));
 * decode v_k = q_k * 2^(E-127).  Four 32-bit words, fields filled from the
 * least significant bit; a field split across words keeps its high bits at
 * the top of the earlier word:
 *   w0: a_re[19:0] | a_im[19:8]<<20      w1: a_im[7:0] | b_re<<8 | b_im[19:16]<<28
 *   w2: b_im[15:0] | c_re[19:4]<<16      w3: c_re[3:0] | c_im<<4 | E<<24          */
void hisq_oracle_int20_encode(const float *v, uint32_t *w, long nsites)
{
    for (long s = 0; s < nsites; s++) {
        const float *a = v + 6 * s;
        float m = fabsf(a[0]);
        for (int k = 1; k < 6; k++) m = fmaxf(m, fabsf(a[k]));
        float t = m / 524287.0f;
        uint32_t e = ((f32_bits(t) >> 23) & 0xffu) + 1u;
        if (e > 254u) e = 254u;
        float inv = f32_from_bits((254u - e) << 23);  /* 2^(127-E) */
        uint32_t u[6];
        for (int k = 0; k < 6; k++) u[k] = (uint32_t)(int32_t)lrintf(a[k] * inv) & 0xfffffu;
        uint32_t *o = w + 4 * s;
        o[0] = u[0] | ((u[1] >> 8) << 20);
        o[1] = (u[1] & 0xffu) | (u[2] << 8) | ((u[3] >> 16) << 28);
        o[2] = (u[3] & 0xffffu) | ((u[4] >> 4) << 16);
        o[3] = (u[4] & 0xfu) | (u[5] << 4) | (e << 24);
    }
}

void hisq_oracle_int20_decode(const uint32_t *w, float *v, long nsites)
{
    for (long s = 0; s < nsites; s++) {
        const uint32_t *o = w + 4 * s;
        uint32_t u[6];
        u[0] = o[0] & 0xfffffu;
        u[1] = ((o[0] >> 20) << 8) | (o[1] & 0xffu);
        u[2] = (o[1] >> 8) & 0xfffffu;
        u[3] = ((o[1] >> 28) << 16) | (o[2] & 0xffffu);
        u[4] = ((o[2] >> 16) << 4) | (o[3] & 0xfu);
        u[5] = (o[3] >> 4) & 0xfffffu;
        uint32_t e = o[3] >> 24;
        float sc = f32_from_bits(e << 23);  /* 2^(E-127) */
        for (int k = 0; k < 6; k++) v[6 * s + k] = (float)sign_extend(u[k], 20) * sc;
    }
}

/* 30-bit shared-exponent spinor (Sec. 4 Listing 3), same rule as the 20-bit
 * format with scale 2^29-1, in FP64 (the format is paired with FP64 compute,
 * Sec. 5.2): t = M/(2^29-1); E = (unbiased exponent of t) + 1 + 127, clamped
 * to [1,254] (E = 1 for t = 0); q_k = rint(v_k * 2^(127-E)).  Six words:
 *   w0: a_re | a_im[29:28]<<30   w1: a_im[27:0] | b_re[29:26]<<28
 *   w2: b_re[25:0] | b_im[29:24]<<26   w3: b_im[23:0] | c_re[29:22]<<24
 *   w4: c_re[21:0] | c_im[29:20]<<22   w5: c_im[19:0] | E<<20 (bits 28-31 zero) */
void hisq_oracle_int30_encode(const double *v, uint32_t *w, long nsites)
{
    for (long s = 0; s < nsites; s++) {
        const double *a = v + 6 * s;
        double m = fabs(a[0]);
        for (int k = 1; k < 6; k++) m = fmax(m, fabs(a[k]));
        double t = m / 536870911.0;
        int e = 1;
        if (t > 0.0) {
            int ex;
            (void)frexp(t, &ex);          /* t = f * 2^ex, f in [0.5,1) */
            e = (ex - 1) + 1 + 127;        /* unbiased exponent of t is ex-1 */
            if (e < 1) e = 1;
            if (e > 254) e = 254;
        }
        double inv = ldexp(1.0, 127 - e);
        uint32_t u[6];
        for (int k = 0; k < 6; k++) u[k] = (uint32_t)(int64_t)llrint(a[k] * inv) & 0x3fffffffu;
        uint32_t *o = w + 6 * s;
        o[0] = u[0] | ((u[1] >> 28) << 30);
        o[1] = (u[1] & 0x0fffffffu) | ((u[2] >> 26) << 28);
        o[2] = (u[2] & 0x03ffffffu) | ((u[3] >> 24) << 26);
        o[3] = (u[3] & 0x00ffffffu) | ((u[4] >> 22) << 24);
        o[4] = (u[4] & 0x003fffffu) | ((u[5] >> 20) << 22);
        o[5] = (u[5] & 0x000fffffu) | ((uint32_t)e << 20);
    }
}

void hisq_oracle_int30_decode(const uint32_t *w, double *v, long nsites)
{
    for (long s = 0; s < nsites; s++) {
        const uint32_t *o = w + 6 * s;
        uint32_t u[6];
        u[0] = o[0] & 0x3fffffffu;
        u[1] = ((o[0] >> 30) << 28) | (o[1] & 0x0fffffffu);
        u[2] = ((o[1] >> 28) << 26) | (o[2] & 0x03ffffffu);
        u[3] = ((o[2] >> 26) << 24) | (o[3] & 0x00ffffffu);
        u[4] = ((o[3] >> 24) << 22) | (o[4] & 0x003fffffu);
        u[5] = ((o[4] >> 22) << 20) | (o[5] & 0x000fffffu);
        int e = (int)((o[5] >> 20) & 0xffu);
        double sc = ldexp(1.0, e - 127);
        for (int k = 0; k < 6; k++) v[6 * s + k] = (double)sign_extend(u[k], 30) * sc;
    }
}

/* Fixed-point gauge (Sec. 2 footnote: smeared links are scaled by the global
 * max field element; Sec. 4: 16-bit with the 20-bit spinor, 32-bit with the
 * 30-bit spinor).  q = rint(u * (Q/absmax)) in FP64 with Q = 2^15-1 or 2^31-1.
 * Decode q * (absmax/Q) in the compute precision (32: both factors rounded to
 * FP32 first; 64: FP64).  absmax = 0 encodes zeros. */
void hisq_oracle_fix16_encode(const double *u, int16_t *q, long n, double absmax)
{
    double c = absmax > 0.0 ? 32767.0 / absmax : 0.0;
    for (long k = 0; k < n; k++) q[k] = (int16_t)llrint(u[k] * c);
}

void hisq_oracle_fix32_encode(const double *u, int32_t *q, long n, double absmax)
{
    double c = absmax > 0.0 ? 2147483647.0 / absmax : 0.0;
    for (long k = 0; k < n; k++) q[k] = (int32_t)llrint(u[k] * c);
}

void hisq_oracle_fix16_decode(const int16_t *q, double *u, long n, double absmax, int compute_bits)
{
    double g = absmax / 32767.0;
    float g32 = (float)g;
    for (long k = 0; k < n; k++)
        u[k] = compute_bits == 32 ? (double)((float)q[k] * g32) : (double)q[k] * g;
}

void hisq_oracle_fix32_decode(const int32_t *q, double *u, long n, double absmax, int compute_bits)
{
    double g = absmax / 2147483647.0;
    float g32 = (float)g;
    for (long k = 0; k < n; k++)
        u[k] = compute_bits == 32 ? (double)((float)q[k] * g32) : (double)q[k] * g;
}
