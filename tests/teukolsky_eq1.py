"""The Teukolsky master equation, Eq. (1), typed directly from the paper, and
a method-of-manufactured-solutions forcing built from it.

Test helper.  It is independent of the oracle's derived first-order system:
it applies Eq. (1) to Psi = exp(i m phi~) r^3 Phi(t, r*, theta) (Eq. (2) with
the Kerr azimuth, d phi~ = d phi + a/Delta dr) using only the chain rule with
d r*/dr = (r^2 + a^2)/Delta, and returns the forcing F that makes a chosen
Phi an exact solution of Phi_tt = (...) + F, where the Phi_tt coefficient is
normalised to one:
    F = -(Delta / Sh2) * exp(-i m phi~) r^-3 * L[Psi],
    Sh2 = (r^2 + a^2)^2 - a^2 Delta sin^2(theta)
(L[Psi] is the left-hand side of Eq. (1); -Sh2/Delta is the coefficient of
Psi_tt in it).
"""
import functools

import numpy as np
import sympy as sp


@functools.lru_cache(maxsize=None)
def operator_coefficients(M, a, s, m):
    """Numeric functions c_k(r, Delta, theta) such that the forcing is
    F = sum_k c_k * D_k with D_k in
      (f_xx Th, f_x Th, f_tt Th, f_t Th, f Th'', f Th', f Th)
    for Phi = f(t, r*) Th(theta)."""
    r, th, t, ph = sp.symbols("r theta t phi", real=True)
    Dl = sp.Symbol("Delta", positive=True)
    Ms, As = sp.nsimplify(M), sp.nsimplify(a)
    I = sp.I
    delta_r = r ** 2 - 2 * Ms * r + As ** 2
    rho = r ** 2 + As ** 2
    G = sp.Function("G")(t, r, th)
    h = sp.Function("h")(r)
    Psi = sp.exp(I * m * (ph + h)) * r ** 3 * G
    sn, cs = sp.sin(th), sp.cos(th)
    # Eq. (1), left-hand side
    L = (-(rho ** 2 / delta_r - As ** 2 * sn ** 2) * sp.diff(Psi, t, 2)
         - 4 * Ms * As * r / delta_r * sp.diff(Psi, t, ph)
         - 2 * s * (r - Ms * (r ** 2 - As ** 2) / delta_r + I * As * cs) * sp.diff(Psi, t)
         + delta_r ** (-s) * sp.diff(delta_r ** (s + 1) * sp.diff(Psi, r), r)
         + 1 / sn * sp.diff(sn * sp.diff(Psi, th), th)
         + (1 / sn ** 2 - As ** 2 / delta_r) * sp.diff(Psi, ph, 2)
         + 2 * s * (As * (r - Ms) / delta_r + I * cs / sn ** 2) * sp.diff(Psi, ph)
         - (s ** 2 * sp.cot(th) ** 2 - s) * Psi)
    # d phi~/dr = a / Delta
    L = L.subs(sp.Derivative(h, (r, 2)), sp.diff(As / delta_r, r)).subs(sp.Derivative(h, r), As / delta_r)
    L = sp.expand(L * sp.exp(-I * m * (ph + h)) / r ** 3)
    fxx, fx, ftt, ft, f0 = sp.symbols("fxx fx ftt ft f0")
    T0, T1, T2 = sp.symbols("T0 T1 T2")
    rs_r = rho / delta_r  # d r*/dr
    L = L.subs(sp.Derivative(G, (r, 2)), rs_r ** 2 * fxx * T0 + sp.diff(rs_r, r) * fx * T0)
    L = L.subs({sp.Derivative(G, r): rs_r * fx * T0,
                sp.Derivative(G, (t, 2)): ftt * T0,
                sp.Derivative(G, t): ft * T0,
                sp.Derivative(G, (th, 2)): f0 * T2,
                sp.Derivative(G, th): f0 * T1})
    L = sp.expand(L.subs(G, f0 * T0))
    sh2 = rho ** 2 - As ** 2 * Dl * sn ** 2
    out = []
    for mono in (fxx * T0, fx * T0, ftt * T0, ft * T0, f0 * T2, f0 * T1, f0 * T0):
        c = L.coeff(fxx if mono.has(fxx) else fx if mono.has(fx) else
                    ftt if mono.has(ftt) else ft if mono.has(ft) else f0)
        sym_T = T0 if mono.has(T0) else T1 if mono.has(T1) else T2
        c = sp.expand(c).coeff(sym_T)
        # Delta written as the symbol so that it can be supplied accurately
        c = sp.together(c.subs(r ** 2 - 2 * Ms * r + As ** 2, Dl))
        c = c.subs(delta_r, Dl)
        expr = -(Dl / sh2) * c
        out.append(sp.lambdify((r, Dl, th), expr, "numpy"))
    return tuple(out)


def forcing(M, a, s, m, r, Delta, theta, D):
    """F on arrays r, Delta, theta (broadcast) given the seven products D_k."""
    cs = operator_coefficients(M, a, s, m)
    F = 0
    for c, d in zip(cs, D):
        F = F + c(r, Delta, theta) * d
    return F


def b_speed(M, a, r, Delta, theta):
    """Characteristic speed b: b^2 is minus the ratio of the Psi_{r* r*} and
    Psi_tt coefficients of Eq. (1), i.e. rho^2/Delta over Sh2/Delta."""
    rho = r * r + a * a
    return rho / np.sqrt(rho * rho - a * a * Delta * np.sin(theta) ** 2)
