"""Pins of the oracle's hyperboloidal layer (Section 2.3, item 2): a layer on
rho in [R, S] in which r* = rho / Omega(rho), Omega = 1 - ((rho-R)/(S-R))^4,
with the time tau = t - h(r*), h' = 1 - d rho / d r*, so that the last grid
node is future null infinity and the waveform can be read there.

What fixes the oracle's layer, independently of it:
  * the map: rho' and rho'' against finite differences of r*(rho);
  * the transformed equations: for any smooth Phi(tau, rho, theta), with
    Pi~ = Phi_tau + bo Phi_rho (the layer's Phi equation), the residual of
    the layer's Pi~ equation equals the residual of Eq. (1) itself (from
    tests/teukolsky_eq1.py, typed from the paper with the chain rule only)
    divided by 1 - H^2 b^2;
  * regularity: every coefficient has a finite limit at future null infinity
    (the source factor fw aside: the source is never there);
  * dynamics: inside rho < R a layered run agrees with a run on a domain so
    large that nothing returns from its outer boundary, the difference
    falling at second order with the grid spacing, and a layered run stays
    bounded and decays once the pulse has left;
  * physics at null infinity: the Schwarzschild l = 2 ringdown read there has
    the published quasinormal frequency.
"""
import numpy as np
import pytest

import oracle
import teukolsky_eq1 as EQ

R, S = 30.0, 50.0


MAP_POINTS = (26.0, 30.0, 31.0, 36.0, 40.0, 45.0, 49.0, 49.9)


def map_check(rho, kind="f64"):
    lm = lambda x: oracle.layer_map(R, S, x, kind=kind)
    rs, rp, H, rpp = lm(rho)
    e = 1e-5
    fd_rp = 2 * e / (lm(rho + e)[0] - lm(rho - e)[0])
    fd_rpp = (lm(rho + e)[1] - lm(rho - e)[1]) / (2 * e)
    assert H == pytest.approx(1 - rp, abs=1e-15)
    if rho <= R:
        assert (rs, rp, H, rpp) == (rho, 1.0, 0.0, 0.0)
        return
    assert rs > rho
    assert rp == pytest.approx(fd_rp, rel=1e-7)
    assert rpp == pytest.approx(fd_rpp, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("rho", MAP_POINTS)
def test_layer_map_derivatives(rho):
    map_check(rho)


def test_layer_map_reaches_infinity():
    rs = [oracle.layer_map(R, S, S - d)[0] for d in (1.0, 1e-1, 1e-2, 1e-3)]
    assert all(b > 5 * a for a, b in zip(rs, rs[1:]))  # r* ~ 1/Omega ~ 1/(S - rho)


def _f(tau, rho, c0=38.0, w0=4.0, k0=0.7):
    """f = exp(-(rho - c0 - tau)^2 / w0^2) exp(-i k0 tau) and its derivatives."""
    z = rho - c0 - tau
    g = np.exp(-z * z / w0 ** 2)
    e = np.exp(-1j * k0 * tau)
    gz = -2 * z / w0 ** 2 * g
    gzz = (-2 / w0 ** 2 + 4 * z * z / w0 ** 4) * g
    return dict(f=g * e, r=gz * e, rr=gzz * e, t=-gz * e - 1j * k0 * g * e,
                tt=gzz * e + 2j * k0 * gz * e - k0 * k0 * g * e, tr=-gzz * e - 1j * k0 * gz * e)


def _Th(th):
    c, s = np.cos(th), np.sin(th)
    return (1 + c) ** 2, -2 * (1 + c) * s, 2 * s * s - 2 * (1 + c) * c


def eq1_check(a, m, kind="f64"):
    M, s = 1.0, -2
    lc = lambda x, th: oracle.layer_coeffs(M, a, s, m, R, S, x, th, kind=kind)
    worst = 0.0
    for rho in (25.0, 31.0, 36.0, 42.0, 47.0, 49.5):
        for th in (0.4, 1.3, 2.5):
            tau = 1.3
            rs, rp, H, rpp = oracle.layer_map(R, S, rho, kind=kind)
            d = _f(tau, rho)
            T0, T1, T2 = _Th(th)
            # the same function in (t, r*): d_t = d_tau, d_{r*} = -H d_tau + rho' d_rho
            fx = -H * d["t"] + rp * d["r"]
            fxx = H * H * d["tt"] - 2 * H * rp * d["tr"] + rp * rp * d["rr"] + rp * rpp * (d["r"] + d["t"])
            c = lc(rho, th)
            r, Dl = c["r"], c["Delta"]
            E = EQ.forcing(M, a, s, m, r, Dl, th,
                           (fxx * T0, fx * T0, d["tt"] * T0, d["t"] * T0, d["f"] * T2, d["f"] * T1, d["f"] * T0))
            b = EQ.b_speed(M, a, r, Dl, th)
            e = 1e-4
            bo_p = lc(rho + e, th)["bo"]
            bo_m = lc(rho - e, th)["bo"]
            bo_rho = (bo_p - bo_m) / (2 * e)
            pt = d["t"] * T0 + c["bo"] * d["r"] * T0
            pt_tau = d["tt"] * T0 + c["bo"] * d["tr"] * T0
            pt_rho = d["tr"] * T0 + bo_rho * d["r"] * T0 + c["bo"] * d["rr"] * T0
            s_pi = c["ct"] * pt + c["cthth"] * d["f"] * T2 + c["cth"] * d["f"] * T1 + c["c0"] * d["f"] * T0
            res = pt_tau - c["bi"] * pt_rho + c["d"] * d["r"] * T0 - s_pi
            want = E / (1 - H * H * b * b)
            worst = max(worst, abs(res - want) / max(abs(want), 1e-12))
    assert worst < 1e-8, worst


@pytest.mark.parametrize("a,m", [(0.0, 2), (0.5, 1), (0.9, 2), (0.9, -3)])
def test_layer_equations_follow_from_eq1(a, m):
    eq1_check(a, m)


@pytest.mark.parametrize("a,m", [(0.5, 2), (0.9, 3)])
def test_layer_coefficients_regular_at_scri(a, m):
    names = ("bo", "bi", "cthth", "cth", "ct", "c0", "d")
    cs = [oracle.layer_coeffs(1.0, a, -2, m, R, S, S - e, 1.1) for e in (1e-2, 1e-3, 1e-4)]
    for k in names:
        v = [c[k] for c in cs]
        assert all(np.isfinite(x) for x in v)
        # settling: the change from 1e-3 to 1e-4 is under half that from 1e-2 to 1e-3
        assert abs(v[2] - v[1]) <= 0.5 * abs(v[1] - v[0]) + 1e-12, (k, v)
    assert cs[2]["bi"] < 1e-6 and 0.99 < cs[2]["bo"] < 1.01  # ingoing speed -> 0, outgoing -> ~1


def _pulse(n_r, n_th, rmin, h):
    rho = rmin + h * np.arange(n_r)
    th = np.arange(n_th) * np.pi / (n_th - 1)
    phi = np.exp(-rho ** 2 / 32.0)[None, :] * ((1 + np.cos(th)) ** 2)[:, None] * (1 + 0.3j)
    return phi.astype(np.complex128), np.zeros_like(phi, dtype=np.complex128)


def _run(h, T, a, m, big, n_th=17, rmin=-50.0, dt=0.025, kind="f64"):
    rmax, layer = (160.0, 0.0) if big else (S, R)
    n_r = int(round((rmax - rmin) / h)) + 1
    g = oracle.Grid(a=a, m=m, n_r=n_r, n_theta=n_th, rstar_min=rmin, rstar_max=rmax, dt=dt, layer_R=layer,
                    i_obs=n_r - 1, kind=kind)
    g.set_state(*_pulse(n_r, n_th, rmin, h))
    g.run(int(round(T / dt)))
    return g.get_state()[0]


def interior_check(a, m, kind="f64"):
    """Inside rho < R the layered run is the solution on an unbounded domain
    (here 160M, whose reflection cannot return by T = 100M) up to the
    scheme's O(h^2) error in the layer."""
    diffs = []
    for h in (0.25, 0.125):
        pl = _run(h, 100.0, a, m, big=False, kind=kind)
        pb = _run(h, 100.0, a, m, big=True)
        n_in = int(round((R + 50.0) / h)) + 1
        peak = np.abs(pb[:, :n_in]).max()
        diffs.append(np.abs(pl[:, :n_in] - pb[:, :n_in]).max())
        assert peak > 1e-2
    assert diffs[0] / diffs[1] > 3.5, diffs     # second order
    assert diffs[1] < 5e-3, diffs               # of a pulse of amplitude ~1 at t = 0


@pytest.mark.parametrize("a,m", [(0.0, 2), (0.5, 2)])
def test_layer_interior_matches_unbounded_domain(a, m):
    interior_check(a, m)


def decay_check(kind="f64"):
    """With the outflow node at null infinity nothing is reflected back: the
    field decays by many orders once the pulse has left (no growth from the
    layer or its boundary)."""
    h, dt, n_th = 0.25, 0.025, 17
    n_r = int(round((S + 100.0) / h)) + 1
    g = oracle.Grid(a=0.5, m=2, n_r=n_r, n_theta=n_th, rstar_min=-100.0, rstar_max=S, dt=dt, layer_R=R,
                    i_obs=n_r - 1, extract_every=40, kind=kind)
    g.set_state(*_pulse(n_r, n_th, -100.0, h))
    g.run(int(round(500.0 / dt)))
    phi, pit = g.get_state()
    assert np.abs(phi).max() < 1e-6 and np.abs(pit).max() < 1e-6
    w = g.waveform()  # Phi at null infinity, every 1M
    amp = np.abs(w).max(axis=1)
    assert amp.max() > 0.1 and amp[-1] < 1e-6 * amp.max()


def test_layer_run_decays():
    decay_check()


def test_layer_rejects_bad_descriptions():
    with pytest.raises(ValueError):
        oracle.Grid(n_r=101, rstar_min=-50.0, rstar_max=50.0, layer_R=60.0)   # R beyond S
    with pytest.raises(ValueError):
        oracle.Grid(n_r=101, rstar_min=-50.0, rstar_max=50.0, layer_R=30.0, s=0)  # s = -2 only


def test_ringdown_at_null_infinity_is_the_schwarzschild_qnm():
    """Read at null infinity, the l = 2 ringdown of a Schwarzschild pulse has
    the fundamental quasinormal frequency (tests/golden/schwarzschild_qnm_l2.json,
    the same bar as the plain domain's pin at r* = 30M).  The fit starts 20M
    after the peak, when the overtones have died away, and runs for 50M, before
    the power-law tail (which decays more slowly at null infinity than at a
    finite radius) takes over."""
    import json
    import os

    import test_oracle_pins as PINS
    from paper_1206_0270_amd import workloads as W

    with open(os.path.join(PINS.GOLDEN, "schwarzschild_qnm_l2.json")) as f:
        want = complex(*json.load(f)["M_omega"])
    h, nth, dt, every = 0.125, 33, 0.025, 4
    n_r = int(round((60.0 + 100.0) / h)) + 1
    g = oracle.Grid(a=0.0, m=2, n_r=n_r, n_theta=nth, rstar_min=-100.0, rstar_max=60.0, dt=dt, layer_R=40.0,
                    i_obs=n_r - 1, extract_every=every)
    th = np.arange(nth) * np.pi / (nth - 1)
    Y = W.swsh_profile(-2, 2, 2, th)
    rho = -100.0 + h * np.arange(n_r)
    phi = (np.exp(-rho ** 2 / 32.0)[None, :] * Y[:, None]).astype(np.complex128)
    g.set_state(phi, np.zeros_like(phi))
    g.run(int(round(160.0 / dt)))
    c = oracle.project(g.waveform(), Y[None, :], np.pi / (nth - 1))[:, 0]
    t = (np.arange(len(c)) + 1) * every * dt
    assert np.max(np.abs(c.imag)) < 1e-14 * np.max(np.abs(c.real))  # real data stay real at a = 0
    t_peak = t[np.argmax(np.abs(c))]
    sel = (t >= t_peak + 20.0) & (t <= t_peak + 70.0)
    om = PINS._matrix_pencil(c[sel].real, every * dt, 2)
    om = om[np.argmax(om.real)]
    assert abs(om.real - want.real) < 0.005 * abs(want.real), om
    assert abs(om.imag - want.imag) < 0.02 * abs(want.imag), om
