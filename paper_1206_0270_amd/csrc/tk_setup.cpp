// Host-side, once-per-instance setup: tortoise coordinate inversion, radial
// and angular coefficient tables, and the time-step stability bound.
//
// The evolved system is Eq. (1) after the m-mode decomposition of Eq. (2)
// (Kerr azimuth, d phi~ = d phi + a/Delta dr, and tortoise r* with
// d r*/dr = (r^2 + a^2)/Delta), divided by the coefficient of Psi_tt and
// written in first-order form with Pi = Phi_t + b Phi_{r*} so that
// u = (Phi, Pi) obeys u_t + D u_{r*} = S as in Eqs. (3)-(4).
#include <cmath>
#include <limits>

#include "tk_internal.h"
#include "tk_layer.h"

namespace tk {

namespace {

struct Kerr {
    double M, a, rp, rm, wp, wm;  // horizons; wp = 2M r+/(r+ - r-), wm = 2M r-/(r+ - r-)
};

Kerr kerr(double M, double a)
{
    Kerr k;
    double q = std::sqrt((M - a) * (M + a));
    k.M = M;
    k.a = a;
    k.rp = M + q;
    k.rm = M - q;
    k.wp = 2.0 * M * k.rp / (2.0 * q);
    k.wm = 2.0 * M * k.rm / (2.0 * q);
    return k;
}

// r*(x), x = r - r+ > 0:  r + wp ln(x/2M) - wm ln((r - r-)/2M)
double rstar_x(const Kerr &k, double x)
{
    double v = k.rp + x + k.wp * std::log(x / (2.0 * k.M));
    if (k.wm != 0.0) v -= k.wm * std::log((x + (k.rp - k.rm)) / (2.0 * k.M));
    return v;
}

}  // namespace

double tortoise_of_x(double M, double a, double x) { return rstar_x(kerr(M, a), x); }

// Inverse tortoise coordinate.  The unknown is u = ln x, in which r* is
// increasing, asymptotically linear towards the horizon (slope wp) and
// exponential outwards.  Newton steps use d r*/du = x + wp - wm x/(x + r+ - r-)
// (no 0 * inf at tiny x) and fall back to bisection of a bracket that
// shrinks with every evaluation.
double x_of_tortoise(double M, double a, double rstar)
{
    Kerr k = kerr(M, a);
    double lo = -700.0, hi = 8.0;
    while (rstar_x(k, std::exp(lo)) > rstar && lo > -740.0) lo -= 8.0;
    while (rstar_x(k, std::exp(hi)) < rstar && hi < 700.0) hi += 8.0;
    double u = rstar > k.rp + 4.0 ? std::log(rstar) : std::log(2.0 * k.M) + (rstar - k.rp) / k.wp;
    if (!(u > lo && u < hi)) u = 0.5 * (lo + hi);
    const double eps = std::numeric_limits<double>::epsilon();
    for (int it = 0; it < 400; ++it) {
        const double x = std::exp(u);
        const double f = rstar_x(k, x) - rstar;
        if (f == 0.0) break;
        if (f < 0.0)
            lo = u;
        else
            hi = u;
        const double g = x + k.wp - k.wm * x / (x + (k.rp - k.rm));
        double un = u - f / g;
        if (!(un > lo && un < hi)) un = 0.5 * (lo + hi);
        const bool done = std::fabs(un - u) <= eps * std::fmax(1.0, std::fabs(u));
        u = un;
        if (done || hi - lo <= eps * std::fmax(1.0, std::fabs(u))) break;
    }
    return std::exp(u);
}

double orbit_frequency(double M, double a, double r0)
{
    double sm = std::sqrt(M);
    return sm / (std::pow(r0, 1.5) + a * sm);
}

// Hyperboloidal layer map (Section 2.3, item 2) on [R, S]: with
// xi = (rho - R)/(S - R) and Omega = 1 - xi^4, r* = rho / Omega; rho' =
// d rho / d r* = Omega^2 / q with q = Omega - rho Omega' (so that
// d q / d rho = -rho Omega''), H = 1 - rho', and rho'' = d rho' / d rho =
// (2 Omega Omega' q + Omega^2 rho Omega'') / q^2.
void layer_map(double R, double S, double rho, double *rstar, double *rhop, double *H, double *rhopp)
{
    if (!(rho > R)) {
        *rstar = rho;
        *rhop = 1.0;
        *H = 0.0;
        *rhopp = 0.0;
        return;
    }
    const double L = S - R, xi = (rho - R) / L, xi2 = xi * xi;
    const double Om = 1.0 - xi2 * xi2;
    const double dOm = -4.0 * xi2 * xi / L, d2Om = -12.0 * xi2 / (L * L);
    const double q = Om - rho * dOm;
    *rstar = rho / Om;
    *rhop = Om * Om / q;
    *H = 1.0 - *rhop;
    *rhopp = (2.0 * Om * dOm * q + Om * Om * rho * d2Om) / (q * q);
}

void fill_layer(const HostInst &hi, LayerTab *tab)
{
    const tk_instance_desc &d = hi.desc;
    const int nq = 2 * d.n_r - 1;
    for (int q = 0; q < nq; ++q) {
        LayerTab &T = tab[q];
        T.pad = 0.0;
        if (q == nq - 1) {  // null infinity: never read (the node is extrapolated)
            T.rhop = T.H = T.rhopp = 0.0;
            continue;
        }
        double rs;
        layer_map(d.layer_start, d.rstar_max, d.rstar_min + (double)q * hi.h / 2.0, &rs, &T.rhop, &T.H, &T.rhopp);
    }
}

void fill_radial(const HostInst &hi, Radial *rad)
{
    const tk_instance_desc &d = hi.desc;
    const double M = d.M, a = d.a, s = d.s, m = d.m;
    const int nq = 2 * d.n_r - 1;
    const bool layer = d.layer_start != 0.0;
    for (int q = 0; q < nq; ++q) {
        double rs = d.rstar_min + (double)q * hi.h / 2.0;
        if (layer && q == nq - 1) {  // null infinity: no coefficient is read there
            rad[q] = Radial{};
            rad[q].rstar = INFINITY;
            continue;
        }
        if (layer) {
            double rhop, H, rhopp;
            layer_map(d.layer_start, d.rstar_max, rs, &rs, &rhop, &H, &rhopp);
        }
        double x = x_of_tortoise(M, a, rs);
        double r = hi.rp + x;
        double Dl = x * (x + (hi.rp - hi.rm));  // Delta = (r - r+)(r - r-)
        double rho = r * r + a * a;
        Radial &R = rad[q];
        R.rho2 = rho * rho;
        R.a2D = a * a * Dl;
        R.rho = rho;
        R.Dl = Dl;
        // ct = -[4 i M a m r + 2 s (r Delta - M (r^2 - a^2) + i a Delta cos)] / Sh2
        R.ct_re = -2.0 * s * (r * Dl - M * (r * r - a * a));
        R.ct_im0 = -4.0 * M * a * m * r;
        R.ct_imc = -2.0 * s * a * Dl;
        // b' = (Delta/rho) a^2 sin^2 [rho (r - M) - 2 r Delta] / Sh2^{3/2}
        R.K = (Dl / rho) * a * a * (rho * (r - M) - 2.0 * r * Dl);
        // c1 = [6 rho Delta / r + 2 s (r - M) rho + 2 r Delta + 2 i m a rho] / Sh2
        R.c1_re = 6.0 * rho * Dl / r + 2.0 * s * (r - M) * rho + 2.0 * r * Dl;
        R.c1_im = 2.0 * m * a * rho;
        // c0 = [6 Delta^2/r^2 + 6(1+s) Delta (r-M)/r + 6 i m a Delta/r
        //       + 4 i m s a (r - M) - Delta V(theta)] / Sh2
        R.c0_re = 6.0 * Dl * Dl / (r * r) + 6.0 * (1.0 + s) * Dl * (r - M) / r;
        R.c0_im = 6.0 * m * a * Dl / r + 4.0 * m * s * a * (r - M);
        R.rstar = rs;
        R.srcg = R.pad1 = R.pad2 = 0.0;
    }
}

void fill_angular(const HostInst &hi, Angular *ang)
{
    const tk_instance_desc &d = hi.desc;
    for (int j = 0; j < d.n_theta; ++j) {
        Angular &A = ang[j];
        double th = j * hi.dth;
        A.theta = th;
        A.srcg = A.cot_h = A.sa = A.kcs = A.V2 = A.pad1 = A.pad2 = 0.0;
        if (j == 0 || j == d.n_theta - 1) {  // coefficients never used on the poles
            A.sn2 = A.cs = A.cot = A.V = 0.0;
            continue;
        }
        double sn = std::sin(th), cs = std::cos(th);
        A.sn2 = sn * sn;
        A.cs = cs;
        A.cot = cs / sn;
        A.cot_h = A.cot * hi.dth * 0.5;
        const double q = 2.0 * hi.dth * hi.dth;  // 1 / (Delta-factor scale)
        double w = d.m + d.s * cs;
        A.V = w * w / A.sn2 - d.s;
        A.sa = q * d.a * d.a * A.sn2;
        A.kcs = q * (-2.0 * d.s * d.a) * cs;
        A.V2 = q * A.V;
    }
}

namespace {
double gauss_cut(double xi, double sig, double win)
{
    if (std::fabs(xi) > win * sig) return 0.0;
    return std::exp(-xi * xi / (2.0 * sig * sig)) / (sig * std::sqrt(2.0 * M_PI));
}
}  // namespace

// Discrete delta of spacing dx around xp at a grid point x (the two forms of
// tk_source_kind): with u = |x - xp| / dx, the linear form is the hat
// (1 - u)/dx on u < 1; the step form is 1/(2dx) inside one cell of xp and
// 1/(4dx) at exactly one cell (the step's midpoint value), a point within
// 1e-9 of a cell boundary counting as on it.
static double discrete_delta(int kind, double x, double xp, double dx)
{
    constexpr double tol = 1e-9;
    const double u = std::fabs(x - xp) / dx;
    if (kind == TK_SRC_CIRCULAR_LINEAR_DELTA) return u < 1.0 ? (1.0 - u) / dx : 0.0;
    if (u < 1.0 - tol) return 0.5 / dx;
    if (u <= 1.0 + tol) return 0.25 / dx;
    return 0.0;
}

void fill_source(const HostInst &hi, Radial *rad, Angular *ang)
{
    const tk_instance_desc &d = hi.desc;
    const int kind = hi.src.kind;
    const double A = hi.src.amplitude;
    if (kind == TK_SRC_CIRCULAR_GAUSSIAN) {
        const double sig_r = hi.src.sigma_r_cells * hi.h, sig_t = hi.src.sigma_th_cells * hi.dth;
        for (int q = 0; q < 2 * d.n_r - 1; ++q)
            rad[q].srcg = A * gauss_cut(rad[q].rstar - hi.src_rstar_p, sig_r, hi.src.window_sigmas);
        for (int j = 0; j < d.n_theta; ++j) ang[j].srcg = gauss_cut(ang[j].theta - M_PI / 2, sig_t, hi.src.window_sigmas);
    } else if (kind == TK_SRC_CIRCULAR_STEP_DELTA || kind == TK_SRC_CIRCULAR_LINEAR_DELTA) {
        for (int q = 0; q < 2 * d.n_r - 1; ++q) rad[q].srcg = A * discrete_delta(kind, rad[q].rstar, hi.src_rstar_p, hi.h);
        for (int j = 0; j < d.n_theta; ++j) ang[j].srcg = discrete_delta(kind, ang[j].theta, M_PI / 2, hi.dth);
    } else {
        for (int q = 0; q < 2 * d.n_r - 1; ++q) rad[q].srcg = 0.0;
        for (int j = 0; j < d.n_theta; ++j) ang[j].srcg = 0.0;
    }
}

// Time-step bound.  With the angular terms inside S, one Lax-Wendroff step
// acts on an oscillatory angular mode of frequency w (frozen coefficients,
// smooth in r*) as the explicit midpoint polynomial, |G|^2 = 1 + (w dt)^4/4,
// a spurious growth of about w^4 dt^3 / 8 per unit time.  It is held to
// 0.01/M with w_max^2 = kappa (2 + (|m| + |s|)^2) / dtheta^2, kappa =
// max_r Delta/(rho^2 - a^2 Delta) (the equatorial angular speed factor),
// together with the radial CFL limit dt <= h / max b.
double stable_dt_bound(const tk_instance_desc &d)
{
    Kerr k = kerr(d.M, d.a);
    const double a2 = d.a * d.a;
    double kap = 0.0, bmax = 1.0;
    // log-spaced scan in x = r - r+, then a local refinement
    double best_lx = 0.0;
    for (int i = 0; i <= 4000; ++i) {
        double lx = -12.0 + i * (20.0 / 4000.0);
        double x = std::exp(lx), r = k.rp + x;
        double Dl = x * (x + (k.rp - k.rm)), rho = r * r + a2;
        double v = Dl / (rho * rho - a2 * Dl);
        if (v > kap) {
            kap = v;
            best_lx = lx;
        }
        bmax = std::fmax(bmax, rho / std::sqrt(rho * rho - a2 * Dl));
    }
    for (int i = -200; i <= 200; ++i) {
        double lx = best_lx + i * (20.0 / 4000.0) / 100.0;
        double x = std::exp(lx), r = k.rp + x;
        double Dl = x * (x + (k.rp - k.rm)), rho = r * r + a2;
        kap = std::fmax(kap, Dl / (rho * rho - a2 * Dl));
    }
    const double dth = M_PI / (d.n_theta - 1);
    const double ms = std::abs(d.m) + std::abs(d.s);
    const double w2 = kap * (2.0 + ms * ms) / (dth * dth);
    const double dt_th = std::cbrt(8.0 * 0.01 / (w2 * w2));
    const double h = (d.rstar_max - d.rstar_min) / (d.n_r - 1);
    return std::fmin(h / bmax, dt_th);
}

}  // namespace tk
