// Device-side helpers shared by the HIP kernels: complex arithmetic, the
// pointwise coefficients of the first-order system, the Lax-Wendroff update
// of Eqs. (3)-(4) at one point, and the smeared particle source.
#pragma once

#include <hip/hip_runtime.h>

#include "tk_internal.h"

namespace tk {

struct cd {  // complex double
    double re, im;
};
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// (Phi, Pi) at one point
struct P4 {
    cd phi, pi;
};
__device__ __forceinline__ P4 operator+(P4 a, P4 b) { return P4{a.phi + b.phi, a.pi + b.pi}; }
__device__ __forceinline__ P4 operator-(P4 a, P4 b) { return P4{a.phi - b.phi, a.pi - b.pi}; }
__device__ __forceinline__ P4 half_sum(P4 a, P4 b)
{
    return P4{mk((a.phi.re + b.phi.re) * 0.5, (a.phi.im + b.phi.im) * 0.5),
              mk((a.pi.re + b.pi.re) * 0.5, (a.pi.im + b.pi.im) * 0.5)};
}
// Second-order one-sided Neumann value at a pole: (4 X1 - X2) / 3
__device__ __forceinline__ double pole_x(double x1, double x2) { return (4.0 * x1 - x2) / 3.0; }
__device__ __forceinline__ P4 pole_bc(P4 a1, P4 a2)
{
    return P4{mk(pole_x(a1.phi.re, a2.phi.re), pole_x(a1.phi.im, a2.phi.im)),
              mk(pole_x(a1.pi.re, a2.pi.re), pole_x(a1.pi.im, a2.pi.im))};
}
__device__ __forceinline__ P4 zero4() { return P4{mk(0, 0), mk(0, 0)}; }

__device__ __forceinline__ P4 ld_p4(const double4 *p)
{
    double4 v = *p;
    return P4{mk(v.x, v.y), mk(v.z, v.w)};
}
__device__ __forceinline__ void st_p4(double4 *p, P4 v) { *p = make_double4(v.phi.re, v.phi.im, v.pi.re, v.pi.im); }

// Coefficients of u_t + D u_{r*} = S at one (radial position, theta row).
struct Coef {
    double b, cthth, cth;
    cd ct, c0, d;
};

__device__ __forceinline__ Coef coef_at(const Radial &R, const Angular &A)
{
    Coef c;
    const double Sh2 = R.rho2 - R.a2D * A.sn2;
    const double W = 1.0 / Sh2;
    const double sig = sqrt(W);
    c.b = R.rho * sig;
    c.cthth = R.Dl * W;
    c.cth = c.cthth * A.cot;
    c.ct = mk(W * R.ct_re, W * (R.ct_im0 + R.ct_imc * A.cs));
    const cd c1 = mk(W * R.c1_re, W * R.c1_im);
    c.c0 = mk(W * (R.c0_re - R.Dl * A.V), W * R.c0_im);
    const double bp = R.K * A.sn2 * W * sig;
    // d = -(c1 - b b' - b ct)
    c.d = mk(c.b * bp + c.b * c.ct.re - c1.re, c.b * c.ct.im - c1.im);
    return c;
}

// One Lax-Wendroff update at a point (Eq. (3) with base = averaged fields and
// fac = dt/2, or Eq. (4) with base = u^n and fac = dt):
//   out = base - fac [ D du / h - S ],
//   S = (Pi_a, ct Pi_a + cthth (d2 Phi_a + cot d1 Phi_a) + c0 Phi_a + F)
// where Phi_a / Pi_a are the averaged fields (rows j-1, j, j+1 for Phi) and
// du the difference across the radial stencil.
__device__ __forceinline__ P4 lw_point(const Coef &c, const P4 &base, cd phm, cd ph0, cd php, cd pi0, const P4 &du,
                                       double fac, double inv_h, double inv_dth2, double inv_2dth, cd F)
{
    const cd d2 = inv_dth2 * (php - 2.0 * ph0 + phm);
    const cd d1 = inv_2dth * (php - phm);
    const cd spi = cmul(c.ct, pi0) + c.cthth * d2 + c.cth * d1 + cmul(c.c0, ph0) + F;
    const cd adv_phi = inv_h * (c.b * du.phi);
    const cd adv_pi = inv_h * (cmul(c.d, du.phi) - c.b * du.pi);
    P4 o;
    o.phi = base.phi - fac * (adv_phi - pi0);
    o.pi = base.pi - fac * (adv_pi - spi);
    return o;
}

// Time factor of the smeared particle source, exp(-i m (Omega t + phase0)).
__device__ __forceinline__ cd source_phase(const DevInst &I, double t)
{
    const double ph = -(double)I.m * (I.src_Omega * t + I.src_phase0);
    return mk(cos(ph), sin(ph));
}

// F(t, r*_q, theta_j) = [A g_r(q)] g_theta(j) exp(-i m (Omega t + phase0));
// the bracket and g_theta are tabulated (zero off the source window).
__device__ __forceinline__ cd source_value(double gq, double gj, cd e)
{
    const double s = gq * gj;
    return mk(s * e.re, s * e.im);
}

}  // namespace tk
