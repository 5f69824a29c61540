// Device-side helpers shared by the HIP kernels: complex arithmetic, the
// pointwise coefficients of the first-order system, the Lax-Wendroff update
// of Eqs. (3)-(4) at one point, and the smeared particle source.  Templated
// on the arithmetic type (double for the FP64 path, float for the
// FP32-compensated path).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_internal.h"

namespace tk {

// Pointers read out of device-side descriptors are generic to the compiler,
// which then emits FLAT memory instructions; those are counted against the
// LDS wait counter as well, so every LDS wait would also drain the loads in
// flight.  These casts state that the memory is global.
#define TK_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const TK_GLOBAL T *gload_ptr(const T *p)
{
    return (const TK_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ TK_GLOBAL T *gstore_ptr(T *p)
{
    return (TK_GLOBAL T *)p;
}
// Tables that no kernel writes (coefficients): through the constant address
// space a wave-uniform index becomes a scalar load, which does not queue
// behind the vector loads in flight.
#define TK_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const TK_CONST T *cload_ptr(const T *p)
{
    return (const TK_CONST T *)p;
}

// Copy of a table entry (a struct of doubles) through a qualified pointer:
// the implicit copy constructor cannot bind to an address-space lvalue, so
// the fields are read one by one (unused ones are dropped by the compiler).
template <typename S>
__device__ __forceinline__ S load_entry(const TK_GLOBAL S *p)
{
    static_assert(sizeof(S) % sizeof(double) == 0, "table entries are arrays of doubles");
    S s;
    double *d = reinterpret_cast<double *>(&s);
    const TK_GLOBAL double *q = reinterpret_cast<const TK_GLOBAL double *>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / sizeof(double)); ++k) d[k] = q[k];
    return s;
}
template <typename S>
__device__ __forceinline__ S load_entry(const TK_CONST S *p)
{
    static_assert(sizeof(S) % sizeof(double) == 0, "table entries are arrays of doubles");
    S s;
    double *d = reinterpret_cast<double *>(&s);
    const TK_CONST double *q = reinterpret_cast<const TK_CONST double *>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / sizeof(double)); ++k) d[k] = q[k];
    return s;
}

template <typename T>
struct cx {
    T re, im;
};
using cd = cx<double>;

template <typename T>
__device__ __forceinline__ cx<T> mkc(T r, T i)
{
    return cx<T>{r, i};
}
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b)
{
    return cx<T>{a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b)
{
    return cx<T>{a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a)
{
    return cx<T>{s * a.re, s * a.im};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> avg(cx<T> a, cx<T> b)
{
    return cx<T>{(a.re + b.re) * T(0.5), (a.im + b.im) * T(0.5)};
}

// (Phi, Pi) at one point
template <typename T>
struct Q4 {
    cx<T> phi, pi;
};
using P4 = Q4<double>;
template <typename T>
__device__ __forceinline__ Q4<T> operator+(Q4<T> a, Q4<T> b)
{
    return Q4<T>{a.phi + b.phi, a.pi + b.pi};
}
template <typename T>
__device__ __forceinline__ Q4<T> operator-(Q4<T> a, Q4<T> b)
{
    return Q4<T>{a.phi - b.phi, a.pi - b.pi};
}
template <typename T>
__device__ __forceinline__ Q4<T> half_sum(Q4<T> a, Q4<T> b)
{
    return Q4<T>{avg(a.phi, b.phi), avg(a.pi, b.pi)};
}
// Second-order one-sided Neumann value at a pole: (4 X1 - X2) / 3
template <typename T>
__device__ __forceinline__ T pole_x(T x1, T x2)
{
    return (T(4) * x1 - x2) / T(3);
}
template <typename T>
__device__ __forceinline__ Q4<T> pole_bc(Q4<T> a1, Q4<T> a2)
{
    return Q4<T>{mkc(pole_x(a1.phi.re, a2.phi.re), pole_x(a1.phi.im, a2.phi.im)),
                 mkc(pole_x(a1.pi.re, a2.pi.re), pole_x(a1.pi.im, a2.pi.im))};
}
template <typename T>
__device__ __forceinline__ Q4<T> zero_q4()
{
    return Q4<T>{mkc(T(0), T(0)), mkc(T(0), T(0))};
}
__device__ __forceinline__ P4 zero4() { return zero_q4<double>(); }

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef unsigned short hvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ P4 ld_p4(const double4 *p)
{
    const dvec4 v = *gload_ptr((const dvec4 *)p);
    return P4{mk(v.x, v.y), mk(v.z, v.w)};
}
__device__ __forceinline__ void st_p4(double4 *p, P4 v)
{
    const dvec4 x = {v.phi.re, v.phi.im, v.pi.re, v.pi.im};
    *gstore_ptr((dvec4 *)p) = x;
}

// Coefficients of u_t + D u_{r*} = S at one (radial position, theta row).
template <typename T>
struct Coef {
    T b, cthth, cth;
    cx<T> ct, c0, d;
};

// From the full tables (two-pass kernel).
__device__ __forceinline__ Coef<double> coef_at(const Radial &R, const Angular &A)
{
    Coef<double> c;
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

// 1/sqrt(x) for x > 0: hardware estimate refined by Newton steps
// y <- y (3 - x y^2) / 2 (two for double, one for float).
__device__ __forceinline__ double inv_sqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = fma(y, fma(-hx * y, y, 0.5), y);
    y = fma(y, fma(-hx * y, y, 0.5), y);
    return y;
}
// 1/x from the hardware estimate and two Newton steps y <- y + y (1 - x y)
// (each squares the relative error): within an ulp or two of the rounded
// quotient, for x finite and away from zero and the denormal range.
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}
__device__ __forceinline__ float inv_sqrt(float x)
{
    float y = __builtin_amdgcn_rsqf(x);
    const float hx = 0.5f * x;
    return fmaf(y, fmaf(-hx * y, y, 0.5f), y);
}

// ---------------------------------------------------------------------------
// Fused-kernel form of the same arithmetic, arranged as chains of fused
// multiply-adds.  The angular part of S_Pi,
//   cthth (Phi_thth + cot Phi_th) ~ A2f (P+ - 2 P0 + P-) + A1f (P+ - P-),
//   A2f = cthth / dtheta^2, A1f = cthth cot / (2 dtheta),
// becomes a weight per row: (A2f + A1f) on row j+1, (A2f - A1f) on row j-1
// and -2 A2f on row j (folded into c0).  The averages on rows j+-1 are
// half the sum of two values; the 1/2 goes into the weights (Ap, Am), and
// 1/h into b and d.
// ---------------------------------------------------------------------------

// Radial factors of one node or half node, premultiplied by the grid
// constants they appear with: rho^2, rho/h, Re ct, Im ct at cos = 0, K
// (b' = K sin^2 W sig), c1/h, D2h = Delta/(2 dtheta^2), c0 (all before the
// 1/Sigma-hat^2 factor W).  Every other Delta-dependent term is D2h times a
// row factor.
template <typename T>
struct RadF {
    T rho2, rho_h, ct_re, ct_im0, K, c1h_re, c1h_im, D2h, c0_re, c0_im;
};
constexpr int kRadF = 10;  // read as 5 pairs

// Uniform factors of a row: sa, kcs, V2 (a^2 Delta sin^2, kct Delta cos,
// Delta V divided by D2h), sin^2, and cot dtheta / 2.
template <typename T>
struct AngF {
    T sa, sn2, kcs, V2, kc;
};

// Coefficients of the fused bracket at one point: bh = b/h (the Phi row's
// speed; bih the Pi row's, the same value outside a hyperboloidal layer),
// dh = d/h, ct, c0a = c0 - 2 A2f, and the row weights Ap, Am = (A2f +-
// A1f)/2; with Sh2 = Sigma-hat^2 and sig = 1/Sigma-hat for the layer's
// transformation.
template <typename T>
struct CoefF {
    T bh, bih, Ap, Am;
    cx<T> ct, c0a, dh;
    T Sh2, sig;
};

// The same from a given sig = 1/Sigma-hat (the two-step kernel hands level
// 1's value to level 2, which needs the same points), and from scratch.
template <typename T>
__device__ __forceinline__ CoefF<T> coef_fused_sig(const RadF<T> &R, const AngF<T> &A, T sig)
{
    CoefF<T> c;
    const T Sh2 = fma(-R.D2h, A.sa, R.rho2);
    const T W = sig * sig;
    c.Sh2 = Sh2;
    c.sig = sig;
    c.bh = R.rho_h * sig;
    c.bih = c.bh;
    const T A2 = R.D2h * W;  // A2f / 2
    const T A1 = A2 * A.kc;  // A1f / 2
    c.Ap = A2 + A1;
    c.Am = A2 - A1;
    const T cti = fma(R.D2h, A.kcs, R.ct_im0);
    c.ct = mkc(W * R.ct_re, W * cti);
    c.c0a = mkc(fma(T(-4), A2, W * fma(-R.D2h, A.V2, R.c0_re)), W * R.c0_im);
    // d/h = (b (b' + ct) - c1) / h; b' + Re ct = W (K sin^2 sig + ct_re)
    const T t = fma(R.K * A.sn2, sig, R.ct_re);
    c.dh = mkc(W * fma(c.bh, t, -R.c1h_re), W * fma(c.bh, cti, -R.c1h_im));
    return c;
}
template <typename T>
__device__ __forceinline__ CoefF<T> coef_fused(const RadF<T> &R, const AngF<T> &A)
{
    return coef_fused_sig(R, A, inv_sqrt(fma(-R.D2h, A.sa, R.rho2)));
}

// The same coefficients with the metric factor W = 1/Sigma-hat^2 left out:
// every term of S_Pi and of d du carries it, so the plain (layer-free) form
// sums the Pi row from these W-free factors and multiplies by W once.
// P, M = Ap / W, Am / W = D2h (1 +- kc); ct, c0 = ct / W, c0a / W; d = (d/h) / W.
template <typename T>
struct CoefW {
    T W, bh, P, M;
    cx<T> ct, c0, d;
};
template <typename T>
__device__ __forceinline__ CoefW<T> coef_w_sig(const RadF<T> &R, const AngF<T> &A, T sig)
{
    CoefW<T> c;
    c.W = sig * sig;
    c.bh = R.rho_h * sig;
    c.P = fma(R.D2h, A.kc, R.D2h);
    c.M = fma(-R.D2h, A.kc, R.D2h);
    const T cti = fma(R.D2h, A.kcs, R.ct_im0);
    c.ct = mkc(R.ct_re, cti);
    c.c0 = mkc(fma(T(-4), R.D2h, fma(-R.D2h, A.V2, R.c0_re)), R.c0_im);
    const T t = fma(R.K * A.sn2, sig, R.ct_re);
    c.d = mkc(fma(c.bh, t, -R.c1h_re), fma(c.bh, cti, -R.c1h_im));
    return c;
}

// Bracket D du / h - S from the W-free factors (arguments as bracket_fused's
// below, no source term: the fused path adds it afterwards):
//   Pi row = W (d' du_Phi - S'_Pi) - b du_Pi, S'_Pi = S_Pi / W.
template <typename T>
__device__ __forceinline__ Q4<T> bracket_w(const CoefW<T> &c, cx<T> pm, cx<T> pp, cx<T> ph0, cx<T> pi0,
                                           const Q4<T> &du)
{
    const T sre = fma(c.ct.re, pi0.re,
                      fma(-c.ct.im, pi0.im, fma(c.c0.re, ph0.re, fma(-c.c0.im, ph0.im, fma(c.P, pp.re, c.M * pm.re)))));
    const T sim = fma(c.ct.re, pi0.im,
                      fma(c.ct.im, pi0.re, fma(c.c0.re, ph0.im, fma(c.c0.im, ph0.re, fma(c.P, pp.im, c.M * pm.im)))));
    const T xre = fma(c.d.re, du.phi.re, fma(-c.d.im, du.phi.im, -sre));
    const T xim = fma(c.d.re, du.phi.im, fma(c.d.im, du.phi.re, -sim));
    Q4<T> br;
    br.phi = mkc(fma(c.bh, du.phi.re, -pi0.re), fma(c.bh, du.phi.im, -pi0.im));
    br.pi = mkc(fma(c.W, xre, -(c.bh * du.pi.re)), fma(c.W, xim, -(c.bh * du.pi.im)));
    return br;
}

// Bracket D du / h - S at a point: pm, pp = the two values whose average is
// Phi on rows j-1, j+1; ph0, pi0 = averaged fields on row j; du = the
// difference across the cell; F = source (zero off its window).
template <typename T>
__device__ __forceinline__ Q4<T> bracket_fused(const CoefF<T> &c, cx<T> pm, cx<T> pp, cx<T> ph0, cx<T> pi0,
                                               const Q4<T> &du, cx<T> F)
{
    // S_Pi = ct pi0 + c0a ph0 + Ap pp + Am pm + F
    const T sre = fma(c.ct.re, pi0.re,
                      fma(-c.ct.im, pi0.im,
                          fma(c.c0a.re, ph0.re, fma(-c.c0a.im, ph0.im, fma(c.Ap, pp.re, fma(c.Am, pm.re, F.re))))));
    const T sim = fma(c.ct.re, pi0.im,
                      fma(c.ct.im, pi0.re,
                          fma(c.c0a.re, ph0.im, fma(c.c0a.im, ph0.re, fma(c.Ap, pp.im, fma(c.Am, pm.im, F.im))))));
    Q4<T> br;
    br.phi = mkc(fma(c.bh, du.phi.re, -pi0.re), fma(c.bh, du.phi.im, -pi0.im));
    br.pi = mkc(fma(c.dh.re, du.phi.re, fma(-c.dh.im, du.phi.im, fma(-c.bih, du.pi.re, -sre))),
                fma(c.dh.re, du.phi.im, fma(c.dh.im, du.phi.re, fma(-c.bih, du.pi.im, -sim))));
    return br;
}

// ---------------------------------------------------------------------------
// Differences form of the same bracket (the FP32-compensated kernels).  The
// angular part of S_Pi is applied to undivided differences down the theta
// columns, d2 = X_{j+1} - 2 X_j + X_{j-1} and d1 = X_{j+1} - X_{j-1}, formed
// from the compensated values before any product and summed over the two
// columns whose average Eqs. (3)-(4) take:
//   cthth (d2 Phi_a / dtheta^2 + cot d1 Phi_a / (2 dtheta)) = A2 D2 + A1 D1,
//   A2 = cthth / (2 dtheta^2), A1 = cthth cot / (4 dtheta),
// with D2, D1 the sums over the two columns.  In a weighted sum of values
// the weights are of size cthth / dtheta^2 and the values' rounding enters
// multiplied by them; here it enters relative to the differences.
// ---------------------------------------------------------------------------

// bh: the Phi row's speed over h, bih the Pi row's (the same value outside a
// hyperboloidal layer); Sh2 = Sigma-hat^2 and sig = 1/Sigma-hat for the
// layer's transformation.
template <typename T>
struct CoefD {
    T bh, bih, A2, A1;
    cx<T> ct, c0, dh;
    T Sh2, sig;
};

template <typename T>
__device__ __forceinline__ CoefD<T> coef_diff_sig(const RadF<T> &R, const AngF<T> &A, T sig)
{
    CoefD<T> c;
    const T Sh2 = fma(-R.D2h, A.sa, R.rho2);
    const T W = sig * sig;
    c.Sh2 = Sh2;
    c.sig = sig;
    c.bh = R.rho_h * sig;
    c.bih = c.bh;
    c.A2 = R.D2h * W;
    c.A1 = c.A2 * A.kc;
    const T cti = fma(R.D2h, A.kcs, R.ct_im0);
    c.ct = mkc(W * R.ct_re, W * cti);
    c.c0 = mkc(W * fma(-R.D2h, A.V2, R.c0_re), W * R.c0_im);
    // d/h = (b (b' + ct) - c1) / h; b' + Re ct = W (K sin^2 sig + ct_re)
    const T t = fma(R.K * A.sn2, sig, R.ct_re);
    c.dh = mkc(W * fma(c.bh, t, -R.c1h_re), W * fma(c.bh, cti, -R.c1h_im));
    return c;
}
template <typename T>
__device__ __forceinline__ CoefD<T> coef_diff(const RadF<T> &R, const AngF<T> &A)
{
    return coef_diff_sig(R, A, inv_sqrt(fma(-R.D2h, A.sa, R.rho2)));
}

// Bracket D du / h - S with S_Pi = ct pi0 + c0 ph0 + A2 D2 + A1 D1.
template <typename T>
__device__ __forceinline__ Q4<T> bracket_diff(const CoefD<T> &c, cx<T> D2, cx<T> D1, cx<T> ph0, cx<T> pi0,
                                              const Q4<T> &du)
{
    const T sre = fma(c.ct.re, pi0.re,
                      fma(-c.ct.im, pi0.im, fma(c.c0.re, ph0.re, fma(-c.c0.im, ph0.im, fma(c.A2, D2.re, c.A1 * D1.re)))));
    const T sim = fma(c.ct.re, pi0.im,
                      fma(c.ct.im, pi0.re, fma(c.c0.re, ph0.im, fma(c.c0.im, ph0.re, fma(c.A2, D2.im, c.A1 * D1.im)))));
    Q4<T> br;
    br.phi = mkc(fma(c.bh, du.phi.re, -pi0.re), fma(c.bh, du.phi.im, -pi0.im));
    br.pi = mkc(fma(c.dh.re, du.phi.re, fma(-c.dh.im, du.phi.im, fma(-c.bih, du.pi.re, -sre))),
                fma(c.dh.re, du.phi.im, fma(c.dh.im, du.phi.re, fma(-c.bih, du.pi.im, -sim))));
    return br;
}

// base - fac * br
template <typename T>
__device__ __forceinline__ Q4<T> lw_update(const Q4<T> &base, T fac, const Q4<T> &br)
{
    return Q4<T>{mkc(fma(-fac, br.phi.re, base.phi.re), fma(-fac, br.phi.im, base.phi.im)),
                 mkc(fma(-fac, br.pi.re, base.pi.re), fma(-fac, br.pi.im, base.pi.im))};
}

// a + w (b - a) componentwise (the average of a and b for w = 1/2, given d = b - a)
template <typename T>
__device__ __forceinline__ Q4<T> mid_from(const Q4<T> &a, const Q4<T> &d)
{
    const T h = T(0.5);
    return Q4<T>{mkc(fma(h, d.phi.re, a.phi.re), fma(h, d.phi.im, a.phi.im)),
                 mkc(fma(h, d.pi.re, a.pi.re), fma(h, d.pi.im, a.pi.im))};
}

// The bracket of Eqs. (3)/(4) at a point: D du / h - S with
//   S = (Pi_a, ct Pi_a + cthth (d2 Phi_a + cot d1 Phi_a) + c0 Phi_a + F)
// where Phi_a / Pi_a are the averaged fields (rows j-1, j, j+1 for Phi) and
// du the difference across the radial stencil.
template <typename T>
__device__ __forceinline__ Q4<T> lw_bracket(const Coef<T> &c, cx<T> phm, cx<T> ph0, cx<T> php, cx<T> pi0,
                                            const Q4<T> &du, T inv_h, T inv_dth2, T inv_2dth, cx<T> F)
{
    const cx<T> d2 = inv_dth2 * (php - T(2) * ph0 + phm);
    const cx<T> d1 = inv_2dth * (php - phm);
    const cx<T> spi = cmul(c.ct, pi0) + c.cthth * d2 + c.cth * d1 + cmul(c.c0, ph0) + F;
    const cx<T> adv_phi = inv_h * (c.b * du.phi);
    const cx<T> adv_pi = inv_h * (cmul(c.d, du.phi) - c.b * du.pi);
    return Q4<T>{adv_phi - pi0, adv_pi - spi};
}

// One Lax-Wendroff update at a point (Eq. (3) with base = averaged fields and
// fac = dt/2, or Eq. (4) with base = u^n and fac = dt):
//   out = base - fac [ D du / h - S ].
template <typename T>
__device__ __forceinline__ Q4<T> lw_point(const Coef<T> &c, const Q4<T> &base, cx<T> phm, cx<T> ph0, cx<T> php,
                                          cx<T> pi0, const Q4<T> &du, T fac, T inv_h, T inv_dth2, T inv_2dth, cx<T> F)
{
    const Q4<T> br = lw_bracket(c, phm, ph0, php, pi0, du, inv_h, inv_dth2, inv_2dth, F);
    return Q4<T>{base.phi - fac * br.phi, base.pi - fac * br.pi};
}

// Smooth switch-on s(x): 0 for x <= 0, 1 for x >= 1, and
// e^{-1/x} / (e^{-1/x} + e^{-1/(1-x)}) = 1 / (1 + e^{1/x - 1/(1-x)}) between.
__device__ __forceinline__ double switch_on(double x)
{
    if (x <= 0.0) return 0.0;
    if (x >= 1.0) return 1.0;
    return 1.0 / (1.0 + exp(1.0 / x - 1.0 / (1.0 - x)));
}

// Time factor of the particle source at time t since step 0:
// s(t / T_on) exp(-i m (Omega (t + t0) + phase0)).
__device__ __forceinline__ cd source_phase(const DevInst &I, double t)
{
    const double ph = -(double)I.m * (I.src_Omega * (t + I.src_t0) + I.src_phase0);
    const double w = I.src_ramp_inv > 0.0 ? switch_on(t * I.src_ramp_inv) : 1.0;
    return mk(w * cos(ph), w * sin(ph));
}

// F(t, r*_q, theta_j) = [A g_r(q)] g_theta(j) exp(-i m (Omega t + phase0));
// the bracket and g_theta are tabulated (zero off the source window).
__device__ __forceinline__ cd source_value(double gq, double gj, cd e)
{
    const double s = gq * gj;
    return mk(s * e.re, s * e.im);
}

}  // namespace tk
