/*
 * Plain reference implementation ("oracle") of the time-domain Teukolsky
 * m-mode evolution: the two-step Lax-Wendroff scheme of Eqs. (3)-(4),
 * applied to the first-order (Phi, Pi) form of the Teukolsky master
 * equation, Eq. (1), after the azimuthal decomposition of Eq. (2).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product (the HIP
 * library) never calls it and shares no code with it.
 *
 * Written for a reader who checks it against the paper by eye: coefficient
 * planes are built once per grid, then each step is two plain loops over the
 * grid, in the order of Eqs. (3) and (4), followed by the boundary
 * conditions of Section 2.2.  No blocking, fusion or reordering.
 *
 * Compiled twice from this one file:
 *   OR_REAL=double       -> liboracle_f64.so   (the parity reference)
 *   OR_REAL=long double  -> liboracle_ld.so    (x87 80-bit, rounding check)
 * with -ffp-contract=off so every product/sum is rounded as written.
 * All inputs and outputs at the ABI are double; the long-double build
 * converts on entry and exit.
 *
 * Readings of points the paper leaves open (each is stated where it is used):
 *  - Pi is the auxiliary momentum Pi = d_t Phi + b d_{r*} Phi of the
 *    first-order method the paper cites for the scheme (Krivan et al. 1997);
 *    it is the choice that makes the principal part u_t + D u_{r*} with the
 *    2x2 advection matrix D of Eqs. (3)-(4).
 *  - The azimuth in Eq. (2) is the Kerr azimuth phi~ with
 *    d phi~ = d phi + (a/Delta) dr (same cited method); for a = 0 it is phi.
 *  - The radial coordinate is the tortoise coordinate r* with
 *    d(r*)/dr = (r^2+a^2)/Delta and the integration constant fixed below.
 *  - theta grid: theta_j = j*pi/(N_theta-1), poles included.
 *  - S at half points/times is S evaluated on the averaged fields with the
 *    exact coefficients at the half node; the source is taken at t^n in the
 *    first step and at t^n + dt/2 in the second.
 *  - Pole conditions of Section 2.2: where m + s is even (for the s = -2
 *    field of the paper: even |m|) d_theta X = 0 is imposed to second order,
 *    X_0 = (4X_1 - X_2)/3 (same at theta = pi); where m + s is odd, X = 0.
 *    A spin-weighted mode behaves like sin^{|m+s|} at the poles, so the
 *    parity of m + s decides.  Applied to Phi and Pi on the half-step array
 *    and on u^{n+1}.
 *  - The point particle is the smeared Gaussian of Section 2.3 item 1:
 *    F = A exp(-i m (Omega t + phi0)) g_r(r* - r*_p) g_theta(theta - pi/2),
 *    g(xi) = exp(-xi^2 / (2 sigma^2)) / (sigma sqrt(2 pi)) for
 *    |xi| <= window*sigma and 0 outside; Omega is the prograde circular
 *    equatorial Kerr orbital frequency sqrt(M) / (r0^{3/2} + a sqrt(M)).
 *    F enters the Pi equation additively.  In place of g_r and g_theta the
 *    source may take the discrete delta functions that item 1 describes as
 *    the finite-difference derivative of a step function on the grid (kinds
 *    2 and 3 below).
 *  - Hyperboloidal layer (Section 2.3, item 2): beyond rho = R the grid
 *    coordinate rho is compactified, r* = rho / Omega(rho), so that the last
 *    node rho = S is future null infinity, and the time is tau = t - h(r*)
 *    with h' = 1 - d rho / d r*.  The evolved pair there is (Phi, Pi~) with
 *    Pi~ = Pi / (1 - h' b); the last node is an outflow boundary, filled by
 *    linear extrapolation.  The transformed system is derived below.
 */
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include <float.h>
#ifdef OR_LONG_DOUBLE
#define OR_REAL long double
#define OR_EPS LDBL_EPSILON
#else
#define OR_REAL double
#define OR_EPS DBL_EPSILON
#endif
typedef OR_REAL real;
typedef OR_REAL _Complex cplx;

#define PI_R ((real)3.14159265358979323846264338327950288L)
#define IU ((cplx)_Complex_I)

/* ------------------------------------------------------------------ */
/* Kerr background                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    real M, a, rp, rm, Ap, Am; /* horizons r+/-; tortoise weights */
} kerr_bg;

static kerr_bg make_bg(real M, real a)
{
    kerr_bg k;
    real q = sqrt(M * M - a * a);
    k.M = M;
    k.a = a;
    k.rp = M + q;
    k.rm = M - q;
    /* d(r*)/dr = (r^2+a^2)/Delta = 1 + Ap/(r-r+) - Am/(r-r-) */
    k.Ap = 2 * M * k.rp / (k.rp - k.rm);
    k.Am = 2 * M * k.rm / (k.rp - k.rm);
    return k;
}

/* Tortoise coordinate as a function of x = r - r+ (x > 0):
 * r* = r + Ap ln((r - r+)/2M) - Am ln((r - r-)/2M).
 * For a = 0 this is r + 2M ln(r/2M - 1). */
static real tortoise_x(const kerr_bg *k, real x)
{
    real r = k->rp + x;
    real val = r + k->Ap * log(x / (2 * k->M));
    if (k->Am != 0)
        val -= k->Am * log((x + k->rp - k->rm) / (2 * k->M));
    return val;
}

/* d r* / d ln x = x * d(r*)/dr */
static real dtortoise_dlnx(const kerr_bg *k, real x)
{
    return x + k->Ap - k->Am * x / (x + k->rp - k->rm);
}

/* Invert r*(x) for x = r - r+.  Newton in y = ln x, safeguarded by
 * bisection on a bracket; r*(y) is strictly increasing.  Near the horizon
 * the root is only defined to about ulp(r*)/Ap relative, by conditioning. */
static real x_of_rstar(const kerr_bg *k, real rstar)
{
    real lo = -700, hi = 40, y;
    while (tortoise_x(k, exp(lo)) > rstar && lo > -11000)
        lo *= 2;
    while (tortoise_x(k, exp(hi)) < rstar)
        hi *= 2;
    y = (lo + hi) / 2;
    int settled = 0;
    for (int it = 0; it < 400 && settled < 2; ++it) {
        real x = exp(y);
        real f = tortoise_x(k, x) - rstar;
        if (f == 0)
            break;
        if (f > 0)
            hi = y;
        else
            lo = y;
        real yn = y - f / dtortoise_dlnx(k, x);
        if (!(yn >= lo && yn <= hi))
            yn = (lo + hi) / 2;
        if (fabs(yn - y) <= 2 * OR_EPS * (fabs(y) > 1 ? fabs(y) : 1))
            settled++;
        y = yn;
    }
    return exp(y);
}

/* ------------------------------------------------------------------ */
/* Coefficients of the first-order system  u_t + D u_{r*} = S          */
/* ------------------------------------------------------------------ */

/* Dividing Eq. (1) (with Psi = exp(i m phi~) r^3 Phi) by the coefficient
 * of d_tt gives
 *   Phi_tt = b^2 Phi_{r*r*} + c1 Phi_{r*} + cthth (Phi_thth + cot Phi_th)
 *            + ct Phi_t + c0 Phi + F,
 * with  Delta = r^2 - 2Mr + a^2, rho = r^2 + a^2,
 *       Sh2 = rho^2 - a^2 Delta sin^2(theta)   ("Sigma-hat squared"):
 *   b     = rho / sqrt(Sh2)
 *   cthth = Delta / Sh2
 *   ct    = -[4 i M a m r + 2 s (r Delta - M (r^2 - a^2) + i a Delta cos)] / Sh2
 *   c1    =  [6 rho Delta / r + 2 s (r - M) rho + 2 r Delta + 2 i m a rho] / Sh2
 *   c0    =  [6 Delta^2/r^2 + 6 (1+s) Delta (r-M)/r + 6 i m a Delta / r
 *             + 4 i m s a (r - M) - Delta ((m + s cos)^2 / sin^2 - s)] / Sh2
 * With Pi = Phi_t + b Phi_{r*}:
 *   Phi_t + b Phi_{r*} = Pi
 *   Pi_t - b Pi_{r*} + d Phi_{r*} = ct Pi + cthth (Phi_thth + cot Phi_th)
 *                                   + c0 Phi + F
 *   d = -(c1 - b b' - b ct),   b' = d b / d r*
 *     = (Delta/rho) a^2 sin^2 [rho (r - M) - 2 r Delta] / Sh2^{3/2}.
 * So D = [[b, 0], [d, -b]] acting on (Phi, Pi) and
 *    S = (Pi, ct Pi + cthth (Phi_thth + cot Phi_th) + c0 Phi + F).
 * Delta is formed from x = r - r+ as x (x + r+ - r-) so that it keeps full
 * relative precision next to the horizon. */
typedef struct {
    real b, bp, cthth, cth; /* cth = cthth * cot(theta) */
    cplx ct, c1, c0, d;
} coeffs;

static coeffs point_coeffs(const kerr_bg *k, int s, int m, real x, real th)
{
    coeffs c;
    real M = k->M, a = k->a;
    real r = k->rp + x;
    real Delta = x * (x + k->rp - k->rm);
    real rho = r * r + a * a;
    real sn = sin(th), cs = cos(th);
    real sn2 = sn * sn;
    real Sh2 = rho * rho - a * a * Delta * sn2;
    real Sh = sqrt(Sh2);
    real Vth = (m + s * cs) * (m + s * cs) / sn2 - s;

    c.b = rho / Sh;
    c.bp = (Delta / rho) * a * a * sn2 * (rho * (r - M) - 2 * r * Delta) / (Sh2 * Sh);
    c.cthth = Delta / Sh2;
    c.cth = c.cthth * cs / sn;
    c.ct = -(4 * IU * M * a * m * r + 2 * s * (r * Delta - M * (r * r - a * a) + IU * a * Delta * cs)) / Sh2;
    c.c1 = (6 * rho * Delta / r + 2 * s * (r - M) * rho + 2 * r * Delta + 2 * IU * m * a * rho) / Sh2;
    c.c0 = (6 * Delta * Delta / (r * r) + 6 * (1 + s) * Delta * (r - M) / r + 6 * IU * m * a * Delta / r +
            4 * IU * m * s * a * (r - M) - Delta * Vth) /
           Sh2;
    c.d = -(c.c1 - c.b * c.bp - c.b * c.ct);
    return c;
}

/* ------------------------------------------------------------------ */
/* Hyperboloidal layer                                                  */
/* ------------------------------------------------------------------ */

/* Compactifying layer on rho in [R, S] (0 < R < S):
 *   r*(rho) = rho / Omega(rho),  Omega = 1 - ((rho - R)/(S - R))^4,
 * equal to rho for rho <= R, so r* runs to infinity as rho -> S.  With
 *   rho' = d rho / d r* = Omega^2 / (Omega - rho Omega'),
 *   H    = d h / d r*   = 1 - rho'        (tau = t - h(r*)),
 *   rho'' = d rho' / d rho,
 * outgoing rays keep unit speed in rho.  out = r*, rho', H, rho''. */
typedef struct {
    real rstar, rhop, H, rhopp;
} layer_map;

static layer_map layer_map_at(real R, real S, real rho)
{
    layer_map L;
    if (rho <= R) {
        L.rstar = rho;
        L.rhop = 1;
        L.H = 0;
        L.rhopp = 0;
        return L;
    }
    real L4 = S - R, xi = (rho - R) / L4;
    real Om = 1 - xi * xi * xi * xi;
    real Om1 = -4 * xi * xi * xi / L4;
    real Om2 = -12 * xi * xi / (L4 * L4);
    real q = Om - rho * Om1; /* d q / d rho = -rho Om2 */
    L.rstar = rho / Om;
    L.rhop = Om * Om / q;
    L.H = 1 - L.rhop;
    L.rhopp = (2 * Om * Om1 * q + Om * Om * rho * Om2) / (q * q);
    return L;
}

/* Coefficients of the first-order system in the layer.  Changing to
 * (tau, rho) turns d_t into d_tau and d_{r*} into -H d_tau + rho' d_rho.
 * With w = 1 - H b, v = 1 + H b, the Phi equation Phi_t + b Phi_{r*} = Pi
 * becomes w Phi_tau + b rho' Phi_rho = Pi, and the Pi equation
 * (1 + H b) Pi_tau - b rho' Pi_rho - d H Phi_tau + d rho' Phi_rho = S_Pi.
 * Eliminating Phi_tau (H b + w = 1) and writing Pi = w Pi~:
 *   Phi_tau + (b rho'/w) Phi_rho = Pi~
 *   Pi~_tau - (b rho'/v) Pi~_rho + (d rho'/(w^2 v)) Phi_rho
 *       = [ct w + d H + b rho' w_rho] Pi~ / (w v)
 *         + [cthth (Phi_thth + cot Phi_th) + c0 Phi + F] / (w v),
 * with b rho' w_rho = b^2 rho' rho'' - b H b'.  So the layer has separate
 * outgoing and ingoing speeds bo = b rho'/w and bi = b rho'/v, and
 * d~ = d rho'/(w^2 v), ct~ = (ct w + d H + b^2 rho' rho'' - b H b')/(w v),
 * and cthth, cth, c0 and F scaled by fw = 1/(w v).  For the spin s = -2
 * field every one of them stays finite as rho -> S: w ~ rho' there and
 * c1 - ct, d, c0, cthth all fall off like 1/r^2.  Near S, 1 - b is far
 * below rounding of b, so w is formed as rho' b + (1 - b) with
 * 1 - b = -a^2 Delta sin^2 / (Sh (Sh + rho)). */
typedef struct {
    real bo, bi, cthth, cth, fw;
    cplx ct, c0, d;
} lcoeffs;

static lcoeffs layer_coeffs(const kerr_bg *k, int s, int m, real x, real th, const layer_map *L)
{
    coeffs c = point_coeffs(k, s, m, x, th);
    lcoeffs o;
    if (L->H == 0 && L->rhop == 1) {
        o.bo = o.bi = c.b;
        o.cthth = c.cthth;
        o.cth = c.cth;
        o.fw = 1;
        o.ct = c.ct;
        o.c0 = c.c0;
        o.d = c.d;
        return o;
    }
    real a = k->a;
    real r = k->rp + x;
    real Delta = x * (x + k->rp - k->rm);
    real rho = r * r + a * a;
    real sn = sin(th);
    real Sh = sqrt(rho * rho - a * a * Delta * sn * sn);
    real one_minus_b = -a * a * Delta * sn * sn / (Sh * (Sh + rho));
    real w = L->rhop * c.b + one_minus_b;
    real v = 1 + L->H * c.b;
    real wv = w * v;
    o.bo = c.b * L->rhop / w;
    o.bi = c.b * L->rhop / v;
    o.d = c.d * L->rhop / (w * wv);
    o.ct = (c.ct * w + c.d * L->H + c.b * c.b * L->rhop * L->rhopp - c.b * L->H * c.bp) / wv;
    o.fw = 1 / wv;
    o.cthth = c.cthth / wv;
    o.cth = c.cth / wv;
    o.c0 = c.c0 / wv;
    return o;
}

/* ------------------------------------------------------------------ */
/* Grid, state, source                                                  */
/* ------------------------------------------------------------------ */

/* Must match the ctypes Structure in oracle/__init__.py */
typedef struct {
    double M, a;
    int s, m;
    int n_r, n_theta;
    double rstar_min, rstar_max, dt;
    int i_obs;         /* extraction column (r* index) */
    int extract_every; /* steps between waveform samples; 0 = none */
    /* synthetic particle source; kind 0 = none, 1 = Gaussian circular orbit,
       2 / 3 = the step / linear discrete delta */
    int src_kind;
    double src_r0, src_amp, src_phase0;
    double src_sigma_r_cells, src_sigma_th_cells, src_window_sigmas;
    double src_t0;   /* time along the orbit at step 0 (a segment's start) */
    double src_ramp; /* switch-on time of the source (0 = none) */
    /* hyperboloidal layer: 0 = none; else the layer starts at rho = layer_R
       and rstar_max is the grid position S of future null infinity */
    double layer_R;
} or_desc;

typedef struct {
    or_desc desc;
    kerr_bg k;
    int nr, nth;
    real h, dth, dt;
    /* radial positions: index q = 2i (node i) or 2i+1 (half node i+1/2) */
    real *rstar, *x; /* [2*nr-1] */
    /* coefficient planes [q][j]; b is the outgoing speed (Phi row) and bi
       the ingoing one (Pi row), equal outside a hyperboloidal layer; fw
       scales the source (1 outside a layer) */
    real *b, *bi, *fw, *cthth, *cth;
    cplx *d, *ct, *c0;
    int layer; /* hyperboloidal layer on: the last node is future null infinity */
    /* state u^n = (Phi, Pi), [j][i]; half-step array [j][i] (i <-> i+1/2) */
    cplx *phi, *pi, *hphi, *hpi, *nphi, *npi;
    long step;
    /* source */
    real src_rstar_p, src_Omega;
    /* waveform ring (grows on demand): samples of Phi(i_obs, j) */
    double *wave;
    long n_wave, cap_wave;
} or_grid;

#define IDX(g, j, i) ((size_t)(j) * (size_t)(g)->nr + (size_t)(i))
#define QIDX(g, q, j) ((size_t)(q) * (size_t)(g)->nth + (size_t)(j))

static void free_grid(or_grid *g)
{
    if (!g)
        return;
    free(g->rstar);
    free(g->x);
    free(g->b);
    free(g->bi);
    free(g->fw);
    free(g->cthth);
    free(g->cth);
    free(g->d);
    free(g->ct);
    free(g->c0);
    free(g->phi);
    free(g->pi);
    free(g->hphi);
    free(g->hpi);
    free(g->nphi);
    free(g->npi);
    free(g->wave);
    free(g);
}

/* Normalised Gaussian of standard deviation sig, cut at |xi| > win*sig. */
static real gauss_window(real xi, real sig, real win)
{
    if (fabs(xi) > win * sig)
        return 0;
    return exp(-xi * xi / (2 * sig * sig)) / (sig * sqrt(2 * PI_R));
}

/* Discrete delta functions (Section 2.3, item 1): a step function laid on
 * the grid, differenced.  Kind 2 takes the sharp Heaviside step H, with the
 * value 1/2 at the jump (a point within 1e-9 of a cell of it counts as on
 * it), and its centred difference over the neighbours x +- dx.  Kind 3 takes
 * the step that rises linearly over the cell below xp and its difference
 * over one cell. */
static real heaviside(real y, real dx)
{
    if (y > (real)1e-9 * dx)
        return 1;
    if (y < -(real)1e-9 * dx)
        return 0;
    return (real)0.5;
}

static real ramp_step(real y, real dx)
{
    real v = y / dx + 1;
    return v <= 0 ? 0 : (v >= 1 ? 1 : v);
}

static real discrete_delta(int kind, real x, real xp, real dx)
{
    if (kind == 2)
        return (heaviside(x + dx - xp, dx) - heaviside(x - dx - xp, dx)) / (2 * dx);
    return (ramp_step(x - xp, dx) - ramp_step(x - dx - xp, dx)) / dx;
}

/* Smooth switch-on of the source (the remedy for the junk of a run that
 * starts with the source at full strength, Section 4): the step
 *   s(x) = f(x) / (f(x) + f(1 - x)),  f(x) = exp(-1/x) for x > 0, 0 else,
 * which is 0 for x <= 0, 1 for x >= 1 and has every derivative zero at both
 * ends. */
static real bump_tail(real x) { return x > 0 ? exp(-1 / x) : 0; }

static real switch_on(real x)
{
    real a = bump_tail(x), b = bump_tail(1 - x);
    return a / (a + b);
}

/* Synthetic particle source F(t, r*, theta), t the time since step 0. */
static cplx source_at(const or_grid *g, real t, real rstar, real th)
{
    const or_desc *d = &g->desc;
    real gr, gt;
    if (d->src_kind == 1) {
        gr = gauss_window(rstar - g->src_rstar_p, (real)d->src_sigma_r_cells * g->h, (real)d->src_window_sigmas);
        gt = gauss_window(th - PI_R / 2, (real)d->src_sigma_th_cells * g->dth, (real)d->src_window_sigmas);
    } else if (d->src_kind == 2 || d->src_kind == 3) {
        gr = discrete_delta(d->src_kind, rstar, g->src_rstar_p, g->h);
        gt = discrete_delta(d->src_kind, th, PI_R / 2, g->dth);
    } else {
        return 0;
    }
    if (gr == 0 || gt == 0)
        return 0;
    real phase = -(real)d->m * (g->src_Omega * (t + (real)d->src_t0) + (real)d->src_phase0);
    real w = d->src_ramp > 0 ? switch_on(t / (real)d->src_ramp) : 1;
    return (real)d->src_amp * w * gr * gt * (cos(phase) + IU * sin(phase));
}

/* ------------------------------------------------------------------ */
/* The operator S (right-hand side apart from the advection term)      */
/* ------------------------------------------------------------------ */

/* Second component of S at radial position q, row j (1 <= j <= nth-2), on
 * the (averaged) fields f_phi/f_pi given as three theta rows j-1, j, j+1:
 *   ct Pi + cthth (d2 Phi + cot d1 Phi) + c0 Phi + F
 * with the second-order centred differences of Section 2.2:
 *   d2 X_j = (X_{j+1} - 2 X_j + X_{j-1}) / dth^2
 *   d1 X_j = (X_{j+1} - X_{j-1}) / (2 dth). */
static cplx S_pi(const or_grid *g, int q, int j, cplx phim, cplx phi0, cplx phip, cplx pi0, cplx F)
{
    size_t c = QIDX(g, q, j);
    cplx d2 = (phip - 2 * phi0 + phim) / (g->dth * g->dth);
    cplx d1 = (phip - phim) / (2 * g->dth);
    return g->ct[c] * pi0 + g->cthth[c] * d2 + g->cth[c] * d1 + g->c0[c] * phi0 + g->fw[c] * F;
}

/* Pole value from the two next interior rows (Section 2.2): for even m + s
 * d_theta X = 0 to second order, X_pole = (4 X_1 - X_2) / 3; for odd m + s
 * X_pole = 0.  Used by the stepper and by or_rhs_column alike. */
static cplx pole_value(const or_grid *g, cplx x1, cplx x2)
{
    if (abs(g->desc.m + g->desc.s) % 2 == 0)
        return (4 * x1 - x2) / 3;
    return 0;
}

static void pole_bc_rows(const or_grid *g, cplx *X, int ncols)
{
    int n = g->nth;
    for (int i = 0; i < ncols; ++i) {
        X[IDX(g, 0, i)] = pole_value(g, X[IDX(g, 1, i)], X[IDX(g, 2, i)]);
        X[IDX(g, n - 1, i)] = pole_value(g, X[IDX(g, n - 2, i)], X[IDX(g, n - 3, i)]);
    }
}

/* One full Lax-Wendroff step u^n -> u^{n+1}.  F_half / F_node are optional
 * externally supplied forcing planes (complex, [j][i], with i the half node
 * i+1/2 for F_half); when NULL the configured synthetic source is used. */
static void lw_step(or_grid *g, const double *F_half, const double *F_node)
{
    const int nr = g->nr, nth = g->nth;
    const real h = g->h, dt = g->dt;
    const real tn = (real)g->step * dt;
    const real th_half = tn + dt / 2;

    /* Eq. (3): u^{n+1/2}_{i+1/2} = (u_{i+1} + u_i)/2
     *          - dt/2 [ D_{i+1/2} (u_{i+1} - u_i)/h - S_{i+1/2} ] */
#pragma omp parallel for schedule(static)
    for (int j = 1; j < nth - 1; ++j) {
        real th = j * g->dth;
        for (int i = 0; i < nr - 1; ++i) {
            int q = 2 * i + 1;
            size_t c = QIDX(g, q, j);
            cplx phb[3], pib;
            for (int jj = -1; jj <= 1; ++jj)
                phb[jj + 1] = (g->phi[IDX(g, j + jj, i + 1)] + g->phi[IDX(g, j + jj, i)]) / 2;
            pib = (g->pi[IDX(g, j, i + 1)] + g->pi[IDX(g, j, i)]) / 2;
            cplx dphi = g->phi[IDX(g, j, i + 1)] - g->phi[IDX(g, j, i)];
            cplx dpi = g->pi[IDX(g, j, i + 1)] - g->pi[IDX(g, j, i)];
            cplx F;
            if (F_half)
                F = F_half[2 * IDX(g, j, i)] + IU * F_half[2 * IDX(g, j, i) + 1];
            else
                F = source_at(g, tn, g->rstar[q], th);
            cplx s_phi = pib;
            cplx s_pi = S_pi(g, q, j, phb[0], phb[1], phb[2], pib, F);
            cplx adv_phi = g->b[c] * dphi / h;
            cplx adv_pi = (g->d[c] * dphi - g->bi[c] * dpi) / h;
            g->hphi[IDX(g, j, i)] = phb[1] - dt / 2 * (adv_phi - s_phi);
            g->hpi[IDX(g, j, i)] = pib - dt / 2 * (adv_pi - s_pi);
        }
    }
    pole_bc_rows(g, g->hphi, nr - 1);
    pole_bc_rows(g, g->hpi, nr - 1);

    /* Eq. (4): u^{n+1}_i = u^n_i
     *          - dt [ D_i (u^{n+1/2}_{i+1/2} - u^{n+1/2}_{i-1/2})/h - S^{n+1/2}_i ] */
#pragma omp parallel for schedule(static)
    for (int j = 1; j < nth - 1; ++j) {
        real th = j * g->dth;
        for (int i = 1; i < nr - 1; ++i) {
            int q = 2 * i;
            size_t c = QIDX(g, q, j);
            cplx pht[3], pit;
            for (int jj = -1; jj <= 1; ++jj)
                pht[jj + 1] = (g->hphi[IDX(g, j + jj, i)] + g->hphi[IDX(g, j + jj, i - 1)]) / 2;
            pit = (g->hpi[IDX(g, j, i)] + g->hpi[IDX(g, j, i - 1)]) / 2;
            cplx dphi = g->hphi[IDX(g, j, i)] - g->hphi[IDX(g, j, i - 1)];
            cplx dpi = g->hpi[IDX(g, j, i)] - g->hpi[IDX(g, j, i - 1)];
            cplx F;
            if (F_node)
                F = F_node[2 * IDX(g, j, i)] + IU * F_node[2 * IDX(g, j, i) + 1];
            else
                F = source_at(g, th_half, g->rstar[q], th);
            cplx s_phi = pit;
            cplx s_pi = S_pi(g, q, j, pht[0], pht[1], pht[2], pit, F);
            cplx adv_phi = g->b[c] * dphi / h;
            cplx adv_pi = (g->d[c] * dphi - g->bi[c] * dpi) / h;
            g->nphi[IDX(g, j, i)] = g->phi[IDX(g, j, i)] - dt * (adv_phi - s_phi);
            g->npi[IDX(g, j, i)] = g->pi[IDX(g, j, i)] - dt * (adv_pi - s_pi);
        }
    }
    /* Radial boundaries: Phi = Pi = 0 at i = 0 and i = nr-1.  With a
     * hyperboloidal layer the last node is future null infinity, where no
     * characteristic enters: it takes the linear extrapolation
     * X_{nr-1} = 2 X_{nr-2} - X_{nr-3} of the new interior values. */
    for (int j = 0; j < nth; ++j) {
        g->nphi[IDX(g, j, 0)] = 0;
        g->npi[IDX(g, j, 0)] = 0;
        if (g->layer) {
            g->nphi[IDX(g, j, nr - 1)] = 2 * g->nphi[IDX(g, j, nr - 2)] - g->nphi[IDX(g, j, nr - 3)];
            g->npi[IDX(g, j, nr - 1)] = 2 * g->npi[IDX(g, j, nr - 2)] - g->npi[IDX(g, j, nr - 3)];
        } else {
            g->nphi[IDX(g, j, nr - 1)] = 0;
            g->npi[IDX(g, j, nr - 1)] = 0;
        }
    }
    pole_bc_rows(g, g->nphi, nr);
    pole_bc_rows(g, g->npi, nr);

    cplx *t;
    t = g->phi;
    g->phi = g->nphi;
    g->nphi = t;
    t = g->pi;
    g->pi = g->npi;
    g->npi = t;
    g->step += 1;

    /* Waveform: Phi at the extraction column, all theta rows, at the new
     * time, every extract_every steps. */
    if (g->desc.extract_every > 0 && g->step % g->desc.extract_every == 0) {
        if (g->n_wave == g->cap_wave) {
            long nc = g->cap_wave ? 2 * g->cap_wave : 64;
            double *w = (double *)realloc(g->wave, (size_t)nc * (size_t)nth * 2 * sizeof(double));
            if (!w)
                return;
            g->wave = w;
            g->cap_wave = nc;
        }
        double *dst = g->wave + (size_t)g->n_wave * (size_t)nth * 2;
        for (int j = 0; j < nth; ++j) {
            cplx v = g->phi[IDX(g, j, g->desc.i_obs)];
            dst[2 * j] = (double)creal(v);
            dst[2 * j + 1] = (double)cimag(v);
        }
        g->n_wave += 1;
    }
}

/* ------------------------------------------------------------------ */
/* Exported API (ctypes)                                                */
/* ------------------------------------------------------------------ */

double or_tortoise(double M, double a, double x)
{
    kerr_bg k = make_bg(M, a);
    return (double)tortoise_x(&k, x);
}

double or_x_of_rstar(double M, double a, double rstar)
{
    kerr_bg k = make_bg(M, a);
    return (double)x_of_rstar(&k, rstar);
}

/* out[14] = b, b', cthth, cth, ct.re, ct.im, c1.re, c1.im, c0.re, c0.im,
 *           d.re, d.im, r, Delta   at (x = r - r+, theta). */
void or_coeffs(double M, double a, int s, int m, double x, double th, double *out)
{
    kerr_bg k = make_bg(M, a);
    coeffs c = point_coeffs(&k, s, m, x, th);
    real r = k.rp + (real)x;
    out[0] = (double)c.b;
    out[1] = (double)c.bp;
    out[2] = (double)c.cthth;
    out[3] = (double)c.cth;
    out[4] = (double)creal(c.ct);
    out[5] = (double)cimag(c.ct);
    out[6] = (double)creal(c.c1);
    out[7] = (double)cimag(c.c1);
    out[8] = (double)creal(c.c0);
    out[9] = (double)cimag(c.c0);
    out[10] = (double)creal(c.d);
    out[11] = (double)cimag(c.d);
    out[12] = (double)r;
    out[13] = (double)((real)x * ((real)x + k.rp - k.rm));
}

/* Circular equatorial prograde orbital frequency (Kerr). */
double or_orbit_omega(double M, double a, double r0)
{
    real sm = sqrt((real)M);
    return (double)(sm / (pow((real)r0, (real)1.5) + (real)a * sm));
}

void *or_grid_new(const or_desc *d)
{
    if (!d || d->n_r < 5 || d->n_theta < 5 || !(d->M > 0) || !(fabs(d->a) < d->M) || !(d->rstar_max > d->rstar_min) ||
        !(d->dt > 0) || d->i_obs < 0 || d->i_obs >= d->n_r)
        return NULL;
    if (d->layer_R != 0 && !(d->layer_R > 0 && d->layer_R > d->rstar_min && d->layer_R < d->rstar_max && d->s == -2))
        return NULL;
    or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
    if (!g)
        return NULL;
    g->desc = *d;
    g->k = make_bg(d->M, d->a);
    g->nr = d->n_r;
    g->nth = d->n_theta;
    g->h = ((real)d->rstar_max - (real)d->rstar_min) / (g->nr - 1);
    g->dth = PI_R / (g->nth - 1);
    g->dt = d->dt;
    size_t nq = 2 * (size_t)g->nr - 1;
    size_t npt = (size_t)g->nr * g->nth;
    size_t nqp = nq * g->nth;
    g->rstar = (real *)malloc(nq * sizeof(real));
    g->x = (real *)malloc(nq * sizeof(real));
    g->b = (real *)calloc(nqp, sizeof(real));
    g->bi = (real *)calloc(nqp, sizeof(real));
    g->fw = (real *)calloc(nqp, sizeof(real));
    g->cthth = (real *)calloc(nqp, sizeof(real));
    g->cth = (real *)calloc(nqp, sizeof(real));
    g->d = (cplx *)calloc(nqp, sizeof(cplx));
    g->ct = (cplx *)calloc(nqp, sizeof(cplx));
    g->c0 = (cplx *)calloc(nqp, sizeof(cplx));
    g->phi = (cplx *)calloc(npt, sizeof(cplx));
    g->pi = (cplx *)calloc(npt, sizeof(cplx));
    g->hphi = (cplx *)calloc(npt, sizeof(cplx));
    g->hpi = (cplx *)calloc(npt, sizeof(cplx));
    g->nphi = (cplx *)calloc(npt, sizeof(cplx));
    g->npi = (cplx *)calloc(npt, sizeof(cplx));
    if (!g->rstar || !g->x || !g->b || !g->bi || !g->fw || !g->cthth || !g->cth || !g->d || !g->ct || !g->c0 || !g->phi || !g->pi ||
        !g->hphi || !g->hpi || !g->nphi || !g->npi) {
        free_grid(g);
        return NULL;
    }
    /* Nodes r*_i = r*_min + i h, half nodes r*_min + (i + 1/2) h.  With a
     * layer these are the grid positions rho, and r* = rho / Omega(rho)
     * beyond R; the last node is future null infinity (r* infinite), where
     * no coefficient is used. */
    g->layer = d->layer_R != 0;
    size_t nq_used = g->layer ? nq - 1 : nq;
    for (size_t q = 0; q < nq; ++q) {
        real rho = (real)d->rstar_min + (real)q * g->h / 2;
        if (q >= nq_used) {
            g->rstar[q] = INFINITY;
            g->x[q] = INFINITY;
            continue;
        }
        g->rstar[q] = g->layer ? layer_map_at((real)d->layer_R, (real)d->rstar_max, rho).rstar : rho;
        g->x[q] = x_of_rstar(&g->k, g->rstar[q]);
    }
    /* Coefficients at every interior theta row (never on the poles). */
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < nq_used; ++q) {
        real rho = (real)d->rstar_min + (real)q * g->h / 2;
        layer_map L = layer_map_at(g->layer ? (real)d->layer_R : INFINITY, (real)d->rstar_max, rho);
        for (int j = 1; j < g->nth - 1; ++j) {
            lcoeffs c = layer_coeffs(&g->k, d->s, d->m, g->x[q], j * g->dth, &L);
            size_t o = QIDX(g, q, j);
            g->b[o] = c.bo;
            g->bi[o] = c.bi;
            g->fw[o] = c.fw;
            g->cthth[o] = c.cthth;
            g->cth[o] = c.cth;
            g->d[o] = c.d;
            g->ct[o] = c.ct;
            g->c0[o] = c.c0;
        }
    }
    if (d->src_kind >= 1 && d->src_kind <= 3) {
        g->src_rstar_p = tortoise_x(&g->k, (real)d->src_r0 - g->k.rp);
        real sm = sqrt((real)d->M);
        g->src_Omega = sm / (pow((real)d->src_r0, (real)1.5) + (real)d->a * sm);
    }
    return g;
}

void or_grid_free(void *h) { free_grid((or_grid *)h); }

/* Host arrays are [theta_j][r*_i][re, im]. */
void or_set_state(void *hd, const double *phi, const double *pi, long step)
{
    or_grid *g = (or_grid *)hd;
    size_t npt = (size_t)g->nr * g->nth;
    for (size_t p = 0; p < npt; ++p) {
        g->phi[p] = (real)phi[2 * p] + IU * (real)phi[2 * p + 1];
        g->pi[p] = (real)pi[2 * p] + IU * (real)pi[2 * p + 1];
    }
    g->step = step;
    g->n_wave = 0;
}

void or_get_state(void *hd, double *phi, double *pi)
{
    or_grid *g = (or_grid *)hd;
    size_t npt = (size_t)g->nr * g->nth;
    for (size_t p = 0; p < npt; ++p) {
        phi[2 * p] = (double)creal(g->phi[p]);
        phi[2 * p + 1] = (double)cimag(g->phi[p]);
        pi[2 * p] = (double)creal(g->pi[p]);
        pi[2 * p + 1] = (double)cimag(g->pi[p]);
    }
}

long or_get_step(void *hd) { return ((or_grid *)hd)->step; }

/* One step with optional external forcing planes (see lw_step). */
void or_step(void *hd, const double *F_half, const double *F_node) { lw_step((or_grid *)hd, F_half, F_node); }

/* n steps with the configured source.  Returns the number of waveform
 * samples held (samples are taken after every extract_every steps). */
long or_run(void *hd, long n_steps)
{
    or_grid *g = (or_grid *)hd;
    for (long n = 0; n < n_steps; ++n)
        lw_step(g, NULL, NULL);
    return g->n_wave;
}

/* Copy up to max_samples waveform samples ([sample][theta][re, im]). */
long or_get_wave(void *hd, double *out, long max_samples)
{
    or_grid *g = (or_grid *)hd;
    long n = g->n_wave < max_samples ? g->n_wave : max_samples;
    memcpy(out, g->wave, (size_t)n * (size_t)g->nth * 2 * sizeof(double));
    return n;
}

/* Radial positions r*_q and x_q = r - r+ for q = 0 .. 2 n_r - 2. */
void or_get_radial(void *hd, double *rstar, double *x)
{
    or_grid *g = (or_grid *)hd;
    for (int q = 0; q < 2 * g->nr - 1; ++q) {
        rstar[q] = (double)g->rstar[q];
        x[q] = (double)g->x[q];
    }
}

/* The Pi-component of S at radial position q (q even: node q/2; odd: half
 * node) for a whole theta column of fields, after imposing the pole rows on
 * the input.  Used to inspect the discrete angular operator.  phi_col and
 * pi_col are [theta][re, im]; out is [theta][re, im] with pole rows 0. */
void or_rhs_column(void *hd, int q, const double *phi_col, const double *pi_col, double *out)
{
    or_grid *g = (or_grid *)hd;
    int n = g->nth;
    cplx *ph = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *pp = (cplx *)malloc((size_t)n * sizeof(cplx));
    for (int j = 0; j < n; ++j) {
        ph[j] = (real)phi_col[2 * j] + IU * (real)phi_col[2 * j + 1];
        pp[j] = (real)pi_col[2 * j] + IU * (real)pi_col[2 * j + 1];
    }
    ph[0] = pole_value(g, ph[1], ph[2]);
    ph[n - 1] = pole_value(g, ph[n - 2], ph[n - 3]);
    pp[0] = pole_value(g, pp[1], pp[2]);
    pp[n - 1] = pole_value(g, pp[n - 2], pp[n - 3]);
    out[0] = out[1] = out[2 * (n - 1)] = out[2 * (n - 1) + 1] = 0;
    for (int j = 1; j < n - 1; ++j) {
        cplx v = S_pi(g, q, j, ph[j - 1], ph[j], ph[j + 1], pp[j], 0);
        out[2 * j] = (double)creal(v);
        out[2 * j + 1] = (double)cimag(v);
    }
    free(ph);
    free(pp);
}

/* Coefficient planes at radial position q for all theta rows:
 * out[nth][12] = b, cthth, cth, ct.re, ct.im, c0.re, c0.im, d.re, d.im,
 *                bi, fw, 0 */
void or_get_coeff_column(void *hd, int q, double *out)
{
    or_grid *g = (or_grid *)hd;
    for (int j = 0; j < g->nth; ++j) {
        size_t c = QIDX(g, q, j);
        double *o = out + 12 * j;
        o[0] = (double)g->b[c];
        o[1] = (double)g->cthth[c];
        o[2] = (double)g->cth[c];
        o[3] = (double)creal(g->ct[c]);
        o[4] = (double)cimag(g->ct[c]);
        o[5] = (double)creal(g->c0[c]);
        o[6] = (double)cimag(g->c0[c]);
        o[7] = (double)creal(g->d[c]);
        o[8] = (double)cimag(g->d[c]);
        o[9] = (double)g->bi[c];
        o[10] = (double)g->fw[c];
        o[11] = 0;
    }
}

/* Layer map at grid position rho: out = r*, rho', H, rho''. */
void or_layer_map(double R, double S, double rho, double *out)
{
    layer_map L = layer_map_at(R, S, rho);
    out[0] = (double)L.rstar;
    out[1] = (double)L.rhop;
    out[2] = (double)L.H;
    out[3] = (double)L.rhopp;
}

/* Layer coefficients at grid position rho (R < rho < S) and theta:
 * out[13] = bo, bi, cthth, cth, fw, ct.re, ct.im, c0.re, c0.im, d.re, d.im,
 *           r, Delta.  Outside the layer they are the plain coefficients. */
void or_layer_coeffs(double M, double a, int s, int m, double R, double S, double rho, double th, double *out)
{
    kerr_bg k = make_bg(M, a);
    layer_map L = layer_map_at(R, S, rho);
    real x = x_of_rstar(&k, L.rstar);
    lcoeffs c = layer_coeffs(&k, s, m, x, th, &L);
    out[0] = (double)c.bo;
    out[1] = (double)c.bi;
    out[2] = (double)c.cthth;
    out[3] = (double)c.cth;
    out[4] = (double)c.fw;
    out[5] = (double)creal(c.ct);
    out[6] = (double)cimag(c.ct);
    out[7] = (double)creal(c.c0);
    out[8] = (double)cimag(c.c0);
    out[9] = (double)creal(c.d);
    out[10] = (double)cimag(c.d);
    out[11] = (double)(k.rp + x);
    out[12] = (double)(x * (x + k.rp - k.rm));
}

/* Synthetic source value at (t, r*, theta) (for tests of the source). */
void or_source_value(void *hd, double t, double rstar, double th, double *out)
{
    cplx v = source_at((or_grid *)hd, t, rstar, th);
    out[0] = (double)creal(v);
    out[1] = (double)cimag(v);
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_real_bytes(void) { return (int)sizeof(real); }
