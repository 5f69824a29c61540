/*
 * CPU model of FP32 arithmetic forms of the Lax-Wendroff step of
 * Eqs. (3)-(4), for studying where single-precision rounding enters.
 *
 * TEST INFRASTRUCTURE.  Loaded only by the test suite and its precision
 * study script.  It takes the FP64 coefficient planes and the source's
 * space factor from the oracle (the caller copies them in) and re-runs the
 * scheme with the rounding of selected quantities switched on:
 *
 *   FM_ARITH32    the stencil arithmetic is FP32: every sum, difference and
 *                 product is rounded to FP32 (emulated: computed in double,
 *                 rounded after each operation), coefficients included.
 *   FM_STORE32    the state is stored as an FP32 value f plus a bf16 Kahan
 *                 term c; Eq. (4)'s update is added to (f, c) with an exact
 *                 two-sum and c is rounded to bf16 (a sum in double where
 *                 the source is non-zero).  Without it the state is double.
 *   FM_DIFF_RAD   the radial difference u_{i+1} - u_i is formed from f and c
 *                 as (f1 - f0) + (c1 - c0); without it from f alone.
 *   FM_DIFF_ANG   the angular operator is applied as differences first,
 *                 d+ = X_{j+1} - X_j and d- = X_j - X_{j-1} from f and c,
 *                 then d2 = d+ - d-, d1 = d+ + d- times their coefficients;
 *                 without it, as one weighted sum of the three rows' values
 *                 (weights of size c_thth / dtheta^2) from f alone.
 *   FM_HALF_PAIR  the radial averages and the half-step values of Eq. (3)
 *                 carry an FP32 compensation term (a value is s + e); without
 *                 it they are single FP32 numbers.
 *   FM_COEF64     the coefficients keep their FP64 values (each product with
 *                 a coefficient is rounded once); without it they are
 *                 rounded to FP32 first.
 *
 * With FM_ARITH32 off, the arithmetic is double on the stored value f + c,
 * so FM_STORE32 alone isolates the storage format.  With every flag off the
 * model is the FP64 scheme itself (the test suite checks it against the
 * oracle).  Boundary conditions are those of Section 2.2 (Dirichlet at both
 * radial ends, or the outflow extrapolation at null infinity when the grid
 * ends in a hyperboloidal layer; pole rows by the parity of m + s), formed in
 * double from the stored values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { FM_ARITH32 = 1, FM_STORE32 = 2, FM_DIFF_RAD = 4, FM_DIFF_ANG = 8, FM_HALF_PAIR = 16, FM_COEF64 = 32 };

/* Must match the ctypes Structure in tests/fp32c_model.py */
typedef struct {
    int nr, nth;
    double h, dth, dt;
    int pole_even; /* m + s even: (4 X1 - X2) / 3 at the poles; else 0 */
    int layer;     /* the last node is null infinity (outflow) */
    int i_obs, extract_every;
    double m, Omega, t0, ramp; /* source time factor exp(-i m Omega (t + t0)) s(t / ramp) */
    int flags;
} fm_desc;

typedef struct {
    fm_desc d;
    /* coefficient planes [j][q] (FP64 values, premultiplied by the grid
     * constants they appear with): b/h, bi/h, d/h, ct, c0, and the angular
     * weights A2 = cthth / dtheta^2, A1 = cth / (2 dtheta) */
    double *bh, *bih, *dhr, *dhi, *ctr, *cti, *c0r, *c0i, *A2, *A1;
    double *gr, *gi; /* source space factor (fw A g_r g_theta e^{-i m phase0}), [j][q] */
    /* state: 4 components (Phi.re, Phi.im, Pi.re, Pi.im), value f (+ c), [k][j][i] */
    double *f, *c, *nf, *nc;
    /* half-step values s (+ e), [k][j][i] with i <-> i + 1/2 */
    double *hs, *he;
    long step;
    double *wave;
    long n_wave, cap_wave;
} fm_grid;

#define PIDX(g, k, j, i) (((size_t)(k) * (size_t)(g)->d.nth + (size_t)(j)) * (size_t)(g)->d.nr + (size_t)(i))
#define QJ(g, q, j) ((size_t)(j) * (2 * (size_t)(g)->d.nr - 1) + (size_t)(q))

/* ---- rounding ---------------------------------------------------- */

static inline double r32(double x) { return (double)(float)x; }

/* x (an FP32 value) rounded to the nearest bf16, ties to even */
static inline double bf16(double x)
{
    float v = (float)x;
    uint32_t u;
    memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u)
        return x;
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&v, &u, 4);
    return (double)v;
}

typedef struct {
    int a32; /* round every operation to FP32 */
} ar;

static inline double rd(const ar *A, double x) { return A->a32 ? r32(x) : x; }
static inline double add(const ar *A, double x, double y) { return rd(A, x + y); }
static inline double sub(const ar *A, double x, double y) { return rd(A, x - y); }
static inline double mul(const ar *A, double x, double y) { return rd(A, x * y); }

typedef struct {
    double s, e;
} pr; /* value s + e */

/* exact sum a + b = s + e in the arithmetic (two-sum) */
static inline pr two_sum(const ar *A, double a, double b)
{
    pr o;
    o.s = add(A, a, b);
    double bb = sub(A, o.s, a);
    o.e = add(A, sub(A, a, sub(A, o.s, bb)), sub(A, b, bb));
    return o;
}

/* ---- setup -------------------------------------------------------- */

void fm_free(void *hd)
{
    fm_grid *g = (fm_grid *)hd;
    if (!g)
        return;
    double *ps[] = {g->bh, g->bih, g->dhr, g->dhi, g->ctr, g->cti, g->c0r, g->c0i, g->A2, g->A1,
                    g->gr, g->gi, g->f, g->c, g->nf, g->nc, g->hs, g->he, g->wave};
    for (size_t k = 0; k < sizeof(ps) / sizeof(ps[0]); ++k)
        free(ps[k]);
    free(g);
}

/* coef: [2 nr - 1][nth][12] as the oracle exports a coefficient column
 * (b, cthth, cth, ct.re, ct.im, c0.re, c0.im, d.re, d.im, bi, fw, 0);
 * src: [2 nr - 1][nth][2] the source's space factor without fw (may be NULL). */
void *fm_new(const fm_desc *d, const double *coef, const double *src)
{
    fm_grid *g = (fm_grid *)calloc(1, sizeof(fm_grid));
    if (!g)
        return NULL;
    g->d = *d;
    size_t nq = 2 * (size_t)d->nr - 1, nqp = nq * (size_t)d->nth, np4 = 4 * (size_t)d->nr * (size_t)d->nth;
    double **planes[] = {&g->bh, &g->bih, &g->dhr, &g->dhi, &g->ctr, &g->cti, &g->c0r, &g->c0i, &g->A2, &g->A1,
                         &g->gr, &g->gi};
    for (size_t k = 0; k < sizeof(planes) / sizeof(planes[0]); ++k)
        if (!(*planes[k] = (double *)calloc(nqp, sizeof(double)))) {
            fm_free(g);
            return NULL;
        }
    double **st[] = {&g->f, &g->c, &g->nf, &g->nc, &g->hs, &g->he};
    for (size_t k = 0; k < sizeof(st) / sizeof(st[0]); ++k)
        if (!(*st[k] = (double *)calloc(np4, sizeof(double)))) {
            fm_free(g);
            return NULL;
        }
    for (size_t q = 0; q < nq; ++q)
        for (int j = 0; j < d->nth; ++j) {
            const size_t i = q * (size_t)d->nth + (size_t)j, o = QJ(g, q, j);
            const double *cc = coef + 12 * i;
            g->bh[o] = cc[0] / d->h;
            g->A2[o] = cc[1] / (d->dth * d->dth);
            g->A1[o] = cc[2] / (2 * d->dth);
            g->ctr[o] = cc[3];
            g->cti[o] = cc[4];
            g->c0r[o] = cc[5];
            g->c0i[o] = cc[6];
            g->dhr[o] = cc[7] / d->h;
            g->dhi[o] = cc[8] / d->h;
            g->bih[o] = cc[9] / d->h;
            if (src) {
                g->gr[o] = cc[10] * src[2 * i];
                g->gi[o] = cc[10] * src[2 * i + 1];
            }
        }
    return g;
}

/* Host state arrays are [theta][r*][re, im] complex (as the oracle's). */
void fm_set_state(void *hd, const double *phi, const double *pi, long step)
{
    fm_grid *g = (fm_grid *)hd;
    const int store32 = (g->d.flags & FM_STORE32) != 0;
    for (int j = 0; j < g->d.nth; ++j)
        for (int i = 0; i < g->d.nr; ++i) {
            size_t p = (size_t)j * g->d.nr + i;
            double v[4] = {phi[2 * p], phi[2 * p + 1], pi[2 * p], pi[2 * p + 1]};
            for (int k = 0; k < 4; ++k) {
                double f = store32 ? r32(v[k]) : v[k];
                g->f[PIDX(g, k, j, i)] = f;
                g->c[PIDX(g, k, j, i)] = store32 ? bf16(v[k] - f) : 0.0;
            }
        }
    g->step = step;
    g->n_wave = 0;
}

void fm_get_state(void *hd, double *phi, double *pi)
{
    fm_grid *g = (fm_grid *)hd;
    for (int j = 0; j < g->d.nth; ++j)
        for (int i = 0; i < g->d.nr; ++i) {
            size_t p = (size_t)j * g->d.nr + i;
            double v[4];
            for (int k = 0; k < 4; ++k)
                v[k] = g->f[PIDX(g, k, j, i)] + g->c[PIDX(g, k, j, i)];
            phi[2 * p] = v[0];
            phi[2 * p + 1] = v[1];
            pi[2 * p] = v[2];
            pi[2 * p + 1] = v[3];
        }
}

/* ---- the step ------------------------------------------------------ */

/* Source time factor at time t since step 0: exp(-i m Omega (t + t0)) s(t/ramp) */
static void time_factor(const fm_desc *d, double t, double *er, double *ei)
{
    double w = 1.0;
    if (d->ramp > 0) {
        double x = t / d->ramp;
        if (x <= 0)
            w = 0;
        else if (x < 1) {
            double a = exp(-1 / x), b = exp(-1 / (1 - x));
            w = a / (a + b);
        }
    }
    double ph = -d->m * d->Omega * (t + d->t0);
    *er = w * cos(ph);
    *ei = w * sin(ph);
}

/* The value at (k, j, i) of a plane pair as a pair. */
static inline pr at(const double *s, const double *e, size_t o) { return (pr){s[o], e[o]}; }

typedef struct {
    const ar *A;
    int diff_rad, diff_ang, pairs, coef64;
} form;

/* Difference a - b of two pairs: from s and e (a difference of values), or
 * from s alone. */
static inline double pdiff(const form *F, pr a, pr b, int use_e)
{
    const ar *A = F->A;
    if (!A->a32)
        return (a.s + a.e) - (b.s + b.e);
    if (!use_e)
        return sub(A, a.s, b.s);
    return add(A, sub(A, a.s, b.s), sub(A, a.e, b.e));
}

/* a + du / 2, as a pair (s + e) when keep is set */
static inline pr pmid(const form *F, pr a, double du, int keep)
{
    const ar *A = F->A;
    if (!A->a32)
        return (pr){(a.s + a.e) + 0.5 * du, 0.0};
    if (!keep)
        return (pr){add(A, a.s, mul(A, 0.5, du)), 0.0};
    pr t = two_sum(A, a.s, mul(A, 0.5, du));
    t.e = add(A, t.e, a.e);
    return t;
}

/* base - fac * br as a pair */
static inline pr pupdate(const form *F, pr base, double fac, double br)
{
    const ar *A = F->A;
    if (!A->a32)
        return (pr){(base.s + base.e) - fac * br, 0.0};
    double inc = mul(A, fac, br);
    if (!F->pairs)
        return (pr){sub(A, base.s, inc), 0.0};
    return two_sum(A, base.s, sub(A, base.e, inc));
}

/* The bracket D du / h - S at one point (q, j): u = averaged (Phi, Pi) on
 * row j, Phi also on rows j -+ 1 (ph[0], ph[2]); du = radial differences.
 * S_Pi = ct Pi + c0 Phi + cthth (d2 Phi + cot d1 Phi); in the weighted-sum
 * form the angular part is (A2 + A1) Phi_{j+1} + (A2 - A1) Phi_{j-1} with
 * -2 A2 folded into c0 (A2 = cthth / dtheta^2, A1 = cth / (2 dtheta)). */
static void bracket(const fm_grid *g, const form *F, size_t c, const pr ph[3][2], const pr pi[2], const double du[4],
                    double br[4])
{
    const ar *A = F->A;
    const int wsum = A->a32 && !F->diff_ang;
    const ar C = {A->a32 && !F->coef64}; /* rounding of the coefficients themselves */
    const double bh = rd(&C, g->bh[c]), bih = rd(&C, g->bih[c]);
    const double dhr = rd(&C, g->dhr[c]), dhi = rd(&C, g->dhi[c]);
    const double ctr = rd(&C, g->ctr[c]), cti = rd(&C, g->cti[c]);
    const double A2 = g->A2[c], A1 = g->A1[c];
    const double c0r = rd(&C, wsum ? g->c0r[c] - 2 * A2 : g->c0r[c]), c0i = rd(&C, g->c0i[c]);
    double ang[2];
    for (int k = 0; k < 2; ++k) {
        if (wsum) {
            ang[k] = add(A, mul(A, rd(&C, A2 + A1), ph[2][k].s), mul(A, rd(&C, A2 - A1), ph[0][k].s));
        } else {
            double dp = pdiff(F, ph[2][k], ph[1][k], 1);
            double dm = pdiff(F, ph[1][k], ph[0][k], 1);
            ang[k] = add(A, mul(A, rd(&C, A2), sub(A, dp, dm)), mul(A, rd(&C, A1), add(A, dp, dm)));
        }
    }
    const double p0r = A->a32 ? pi[0].s : pi[0].s + pi[0].e, p0i = A->a32 ? pi[1].s : pi[1].s + pi[1].e;
    const double f0r = A->a32 ? ph[1][0].s : ph[1][0].s + ph[1][0].e;
    const double f0i = A->a32 ? ph[1][1].s : ph[1][1].s + ph[1][1].e;
    const double s_re =
        add(A, add(A, sub(A, mul(A, ctr, p0r), mul(A, cti, p0i)), sub(A, mul(A, c0r, f0r), mul(A, c0i, f0i))), ang[0]);
    const double s_im =
        add(A, add(A, add(A, mul(A, ctr, p0i), mul(A, cti, p0r)), add(A, mul(A, c0r, f0i), mul(A, c0i, f0r))), ang[1]);
    br[0] = sub(A, mul(A, bh, du[0]), p0r);
    br[1] = sub(A, mul(A, bh, du[1]), p0i);
    br[2] = sub(A, sub(A, sub(A, mul(A, dhr, du[0]), mul(A, dhi, du[1])), mul(A, bih, du[2])), s_re);
    br[3] = sub(A, sub(A, add(A, mul(A, dhr, du[1]), mul(A, dhi, du[0])), mul(A, bih, du[3])), s_im);
}

static double pole_v(const fm_grid *g, double x1, double x2) { return g->d.pole_even ? (4 * x1 - x2) / 3 : 0.0; }

/* store value v at (k, j, i) of the new state */
static inline void put_new(fm_grid *g, int k, int j, int i, double v)
{
    size_t o = PIDX(g, k, j, i);
    if (g->d.flags & FM_STORE32) {
        double f = r32(v);
        g->nf[o] = f;
        g->nc[o] = bf16(v - f);
    } else {
        g->nf[o] = v;
        g->nc[o] = 0.0;
    }
}

static void fm_step1(fm_grid *g)
{
    const fm_desc *d = &g->d;
    const int nr = d->nr, nth = d->nth;
    const int flags = d->flags;
    ar A = {(flags & FM_ARITH32) != 0};
    form F = {&A, (flags & FM_DIFF_RAD) != 0, (flags & FM_DIFF_ANG) != 0, (flags & FM_HALF_PAIR) != 0,
              (flags & FM_COEF64) != 0};
    const double dt = d->dt, tn = (double)g->step * dt;
    double ehr, ehi, efr, efi;
    time_factor(d, tn, &ehr, &ehi);
    time_factor(d, tn + 0.5 * dt, &efr, &efi);
    const double *f = g->f, *cc = g->c;

    /* Eq. (3): half node i + 1/2, rows 1 .. nth - 2 */
#pragma omp parallel for schedule(static)
    for (int j = 1; j < nth - 1; ++j) {
        for (int i = 0; i < nr - 1; ++i) {
            size_t c = QJ(g, 2 * i + 1, j);
            double du[4];
            pr ph[3][2], pi[2];
            for (int k = 0; k < 4; ++k) {
                pr a0 = at(f, cc, PIDX(g, k, j, i)), a1 = at(f, cc, PIDX(g, k, j, i + 1));
                du[k] = pdiff(&F, a1, a0, F.diff_rad);
                const int keep = F.pairs || (k < 2 && F.diff_ang);
                pr m = pmid(&F, a0, keep ? pdiff(&F, a1, a0, 1) : du[k], keep);
                if (k < 2)
                    ph[1][k] = m;
                else
                    pi[k - 2] = m;
            }
            for (int s = -1; s <= 1; s += 2)
                for (int k = 0; k < 2; ++k) {
                    pr a0 = at(f, cc, PIDX(g, k, j + s, i)), a1 = at(f, cc, PIDX(g, k, j + s, i + 1));
                    const int keep = F.pairs || F.diff_ang;
                    ph[1 + s][k] = pmid(&F, a0, pdiff(&F, a1, a0, keep), keep);
                }
            double br[4];
            bracket(g, &F, c, (const pr(*)[2])ph, pi, du, br);
            pr base[4] = {ph[1][0], ph[1][1], pi[0], pi[1]};
            for (int k = 0; k < 4; ++k) {
                pr hv = pupdate(&F, base[k], 0.5 * dt, br[k]);
                if (k >= 2 && (g->gr[c] != 0.0 || g->gi[c] != 0.0)) {
                    /* FP64 source increment (dt / 2) F */
                    double Fr = g->gr[c] * ehr - g->gi[c] * ehi, Fi = g->gr[c] * ehi + g->gi[c] * ehr;
                    double v = hv.s + hv.e + 0.5 * dt * (k == 2 ? Fr : Fi);
                    hv.s = A.a32 ? r32(v) : v;
                    hv.e = A.a32 && F.pairs ? r32(v - hv.s) : 0.0;
                }
                g->hs[PIDX(g, k, j, i)] = hv.s;
                g->he[PIDX(g, k, j, i)] = hv.e;
            }
        }
    }
    /* pole rows of the half array, in double from the pairs */
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < nr - 1; ++i) {
            int rows[2][3] = {{0, 1, 2}, {nth - 1, nth - 2, nth - 3}};
            for (int p = 0; p < 2; ++p) {
                size_t o1 = PIDX(g, k, rows[p][1], i), o2 = PIDX(g, k, rows[p][2], i), o0 = PIDX(g, k, rows[p][0], i);
                double v = pole_v(g, g->hs[o1] + g->he[o1], g->hs[o2] + g->he[o2]);
                double s = A.a32 ? r32(v) : v;
                g->hs[o0] = s;
                g->he[o0] = A.a32 && F.pairs ? r32(v - s) : 0.0;
            }
        }

    /* Eq. (4): node i, rows 1 .. nth - 2 */
#pragma omp parallel for schedule(static)
    for (int j = 1; j < nth - 1; ++j) {
        for (int i = 1; i < nr - 1; ++i) {
            size_t c = QJ(g, 2 * i, j);
            double du[4];
            pr ph[3][2], pi[2];
            for (int k = 0; k < 4; ++k) {
                pr a0 = at(g->hs, g->he, PIDX(g, k, j, i - 1)), a1 = at(g->hs, g->he, PIDX(g, k, j, i));
                du[k] = pdiff(&F, a1, a0, F.diff_rad);
                const int keep = F.pairs || (k < 2 && F.diff_ang);
                pr m = pmid(&F, a0, keep ? pdiff(&F, a1, a0, 1) : du[k], keep);
                if (k < 2)
                    ph[1][k] = m;
                else
                    pi[k - 2] = m;
            }
            for (int s = -1; s <= 1; s += 2)
                for (int k = 0; k < 2; ++k) {
                    pr a0 = at(g->hs, g->he, PIDX(g, k, j + s, i - 1)), a1 = at(g->hs, g->he, PIDX(g, k, j + s, i));
                    const int keep = F.pairs || F.diff_ang;
                    ph[1 + s][k] = pmid(&F, a0, pdiff(&F, a1, a0, keep), keep);
                }
            double br[4];
            bracket(g, &F, c, (const pr(*)[2])ph, pi, du, br);
            const int src = g->gr[c] != 0.0 || g->gi[c] != 0.0;
            const double Fr = g->gr[c] * efr - g->gi[c] * efi, Fi = g->gr[c] * efi + g->gi[c] * efr;
            for (int k = 0; k < 4; ++k) {
                size_t o = PIDX(g, k, j, i);
                double fv = f[o], cv = cc[o];
                if (!(flags & FM_STORE32)) {
                    double v = fv - (A.a32 ? mul(&A, dt, br[k]) : dt * br[k]);
                    if (k >= 2 && src)
                        v += dt * (k == 2 ? Fr : Fi);
                    g->nf[o] = v;
                    g->nc[o] = 0.0;
                } else if (src && k >= 2) {
                    double v = (fv + cv) + (A.a32 ? -mul(&A, dt, br[k]) : -dt * br[k]) + dt * (k == 2 ? Fr : Fi);
                    double nfv = r32(v);
                    g->nf[o] = nfv;
                    g->nc[o] = bf16(v - nfv);
                } else if (A.a32) {
                    pr t = two_sum(&A, fv, sub(&A, cv, mul(&A, dt, br[k])));
                    g->nf[o] = t.s;
                    g->nc[o] = bf16(t.e);
                } else {
                    double v = (fv + cv) - dt * br[k];
                    double nfv = r32(v);
                    g->nf[o] = nfv;
                    g->nc[o] = bf16(v - nfv);
                }
            }
        }
    }
    /* radial boundaries, then the pole rows, in double */
    for (int k = 0; k < 4; ++k)
        for (int j = 1; j < nth - 1; ++j) {
            put_new(g, k, j, 0, 0.0);
            if (d->layer) {
                size_t o2 = PIDX(g, k, j, nr - 2), o3 = PIDX(g, k, j, nr - 3);
                put_new(g, k, j, nr - 1, 2 * (g->nf[o2] + g->nc[o2]) - (g->nf[o3] + g->nc[o3]));
            } else {
                put_new(g, k, j, nr - 1, 0.0);
            }
        }
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < nr; ++i) {
            int rows[2][3] = {{0, 1, 2}, {nth - 1, nth - 2, nth - 3}};
            for (int p = 0; p < 2; ++p) {
                size_t o1 = PIDX(g, k, rows[p][1], i), o2 = PIDX(g, k, rows[p][2], i);
                put_new(g, k, rows[p][0], i, pole_v(g, g->nf[o1] + g->nc[o1], g->nf[o2] + g->nc[o2]));
            }
        }
    double *t = g->f;
    g->f = g->nf;
    g->nf = t;
    t = g->c;
    g->c = g->nc;
    g->nc = t;
    g->step += 1;

    if (d->extract_every > 0 && g->step % d->extract_every == 0) {
        if (g->n_wave == g->cap_wave) {
            long nc = g->cap_wave ? 2 * g->cap_wave : 256;
            double *w = (double *)realloc(g->wave, (size_t)nc * (size_t)nth * 2 * sizeof(double));
            if (!w)
                return;
            g->wave = w;
            g->cap_wave = nc;
        }
        double *dst = g->wave + (size_t)g->n_wave * (size_t)nth * 2;
        for (int j = 0; j < nth; ++j) {
            dst[2 * j] = g->f[PIDX(g, 0, j, d->i_obs)] + g->c[PIDX(g, 0, j, d->i_obs)];
            dst[2 * j + 1] = g->f[PIDX(g, 1, j, d->i_obs)] + g->c[PIDX(g, 1, j, d->i_obs)];
        }
        g->n_wave += 1;
    }
}

/* Subnormal values (the far tails of a spreading front) are flushed to zero
 * on every worker thread: they carry nothing at this study's accuracy and
 * make x86 arithmetic on them about a hundred times slower. */
static void flush_subnormals(void)
{
#pragma omp parallel
    _mm_setcsr(_mm_getcsr() | 0x8040);
}

long fm_run(void *hd, long n)
{
    fm_grid *g = (fm_grid *)hd;
    flush_subnormals();
    for (long s = 0; s < n; ++s)
        fm_step1(g);
    return g->n_wave;
}

long fm_get_wave(void *hd, double *out, long max_samples)
{
    fm_grid *g = (fm_grid *)hd;
    long n = g->n_wave < max_samples ? g->n_wave : max_samples;
    memcpy(out, g->wave, (size_t)n * (size_t)g->d.nth * 2 * sizeof(double));
    return n;
}

void fm_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
