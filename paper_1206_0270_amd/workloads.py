"""Seeded synthetic workloads for the Teukolsky m-mode stepper.

This module only generates inputs: grid descriptions, time steps, initial
data and source parameters.  It holds none of the scheme's arithmetic and is
shared, as an input generator, by the HIP path's tests and benchmark and by
the CPU oracle's tests.

The paper (Section 5) evolves trajectory-driven inspirals on (r*, theta)
grids of about 10^4 x 10^2 points (32000 x 304 for its timing study); the
trajectories, the full Teukolsky source and its figure data are not
available, so these synthetic inputs stand in with the same grid shapes:
Gaussian pulses times spin-weighted angular profiles, and smeared-Gaussian
point particles on circular equatorial orbits.

Seeds: workload k (1-based) draws from numpy PCG64(12060270 + k).
"""
import math

import numpy as np
from scipy.special import eval_jacobi, gammaln

SEED_BASE = 12060270


def rng_for(k):
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


# ---------------------------------------------------------------------------
# Angular profiles (initial data and projection basis)
# ---------------------------------------------------------------------------

def swsh_profile(s, m, l, theta):
    """Spin-weighted spherical harmonic theta-profile _sY_lm(theta) (phi part
    dropped), up to sign, normalised to 2 pi int |Y|^2 sin(theta) dtheta = 1.

    Jacobi form: (1-x)^{|m+s|/2} (1+x)^{|m-s|/2} P_n^{(|m+s|, |m-s|)}(x),
    x = cos(theta), n = l - max(|m|, |s|).  These are the eigenfunctions of
    d2/dtheta2 + cot d/dtheta - ((m + s cos)^2 / sin^2 - s) with eigenvalue
    -(l - s)(l + s + 1)."""
    al, be = abs(m + s), abs(m - s)
    n = l - max(abs(m), abs(s))
    if n < 0:
        raise ValueError("l must be >= max(|m|, |s|)")
    x = np.cos(np.asarray(theta, dtype=np.float64))
    # (1-x)^{al/2}(1+x)^{be/2} written with half angles for accuracy at poles
    st2 = np.sin(np.asarray(theta) / 2.0)
    ct2 = np.cos(np.asarray(theta) / 2.0)
    w = (np.sqrt(2.0) * st2) ** al * (np.sqrt(2.0) * ct2) ** be
    p = eval_jacobi(n, al, be, x)
    # int_{-1}^{1} (1-x)^al (1+x)^be P_n^2 dx  (closed form)
    lognorm = ((al + be + 1) * math.log(2.0) - math.log(2 * n + al + be + 1)
               + gammaln(n + al + 1) + gammaln(n + be + 1)
               - gammaln(n + al + be + 1) - gammaln(n + 1))
    return w * p / math.sqrt(2 * math.pi * math.exp(lognorm))


# ---------------------------------------------------------------------------
# Time step
# ---------------------------------------------------------------------------

def kappa(a, M=1.0):
    """max over r > r_+ of Delta / (rho^2 - a^2 Delta): the largest angular
    wave speed factor (attained on the equator)."""
    rp = M + math.sqrt(M * M - a * a)
    x = np.logspace(-6, 3, 200001)
    r = rp + x
    delta = r * r - 2 * M * r + a * a
    rho = r * r + a * a
    return float(np.max(delta / (rho * rho - a * a * delta)))


def stable_dt(a, m, s, h, n_theta, growth=0.01, M=1.0):
    """Time step rule for the two-step scheme with the angular terms in S.

    A frozen-coefficient analysis of Eqs. (3)-(4) gives |G|^2 = 1 + z^4/4 for
    an oscillatory angular mode of frequency w (z = w dt), i.e. a spurious
    growth rate of about w^4 dt^3 / 8.  Bounding it by `growth` (per M) with
    w_max^2 = kappa(a) (2 + (|m| + |s|)^2) / dtheta^2 gives
    dt_theta = (8 growth / w_max^4)^{1/3}; the step is min(h/2, dt_theta),
    rounded down to 1/k M."""
    dth = math.pi / (n_theta - 1)
    w2 = kappa(a, M) * (2 + (abs(m) + abs(s)) ** 2) / dth ** 2
    dt_th = (8 * growth / (w2 * w2)) ** (1.0 / 3.0)
    dt = min(0.5 * h, dt_th)
    return 1.0 / math.ceil(1.0 / dt - 1e-9)


# ---------------------------------------------------------------------------
# Instances
# ---------------------------------------------------------------------------

def instance(M=1.0, a=0.0, s=-2, m=2, n_r=801, n_theta=33, rstar_min=-100.0,
             rstar_max=100.0, dt=None, rstar_obs=None, extract_every=None,
             source=None, init=None, name="", layer_start=0.0):
    """Plain dict describing one (a, s, m) mode on one grid.  With
    layer_start = R > 0 the grid ends in a hyperboloidal layer on
    [R, rstar_max] whose last node is future null infinity (rstar_obs
    defaults to that node)."""
    h = (rstar_max - rstar_min) / (n_r - 1)
    if dt is None:
        dt = stable_dt(a, m, s, h, n_theta, M=M)
    if rstar_obs is None:
        rstar_obs = rstar_max if layer_start else rstar_max - 10.0
    if extract_every is None:
        extract_every = max(1, int(round(1.0 / dt)))
    return dict(M=M, a=a, s=s, m=m, n_r=n_r, n_theta=n_theta,
                rstar_min=rstar_min, rstar_max=rstar_max, dt=dt,
                rstar_obs=rstar_obs, extract_every=extract_every,
                i_obs=int(math.floor((rstar_obs - rstar_min) / h + 0.5)),
                source=source, init=init, name=name, layer_start=layer_start)


def refine(inst, k, point_limit=False):
    """The same physical problem with the grid spacings h, dtheta and the
    time step divided by 2^k: n - 1 intervals become 2^k (n - 1), the waveform
    is sampled at the same times, and the source keeps its physical widths
    (its widths are given in cells).  Coarse nodes stay nodes of the refined
    grid, so results compare at the coarse points.  With point_limit the
    Gaussian keeps its width in cells instead, so that refinement tends to the
    point particle (the discrete deltas are one cell wide at every level)."""
    f = 2 ** k
    out = dict(inst)
    out["n_r"] = (inst["n_r"] - 1) * f + 1
    out["n_theta"] = (inst["n_theta"] - 1) * f + 1
    out["dt"] = inst["dt"] / f
    out["extract_every"] = inst["extract_every"] * f
    h = (inst["rstar_max"] - inst["rstar_min"]) / (out["n_r"] - 1)
    out["i_obs"] = int(math.floor((inst["rstar_obs"] - inst["rstar_min"]) / h + 0.5))
    if inst.get("source") and not point_limit:
        src = dict(inst["source"])
        src["sigma_r_cells"] = src.get("sigma_r_cells", 2.0) * f
        src["sigma_th_cells"] = src.get("sigma_th_cells", 2.0) * f
        out["source"] = src
    out["name"] = f"{inst.get('name', '')}/r{f}"
    return out


def richardson_family(inst, levels=3, point_limit=False):
    """refine(inst, k) for k = 0 .. levels-1, with the base time step lowered
    (if needed) so that every level satisfies its own step rule: the
    angular part of the rule scales like dtheta^(4/3), faster than the
    halving of dt.  The base step is 1/N M, so the halvings are exact."""
    h = (inst["rstar_max"] - inst["rstar_min"]) / (inst["n_r"] - 1)
    dt = inst["dt"]
    for k in range(levels):
        f = 2 ** k
        dt = min(dt, f * stable_dt(inst["a"], inst["m"], inst["s"], h / f, (inst["n_theta"] - 1) * f + 1,
                                   M=inst["M"]))
    base = dict(inst)
    base["dt"] = 1.0 / math.ceil(1.0 / dt - 1e-9)
    base["extract_every"] = max(1, int(round(inst["extract_every"] * inst["dt"] / base["dt"])))
    return [refine(base, k, point_limit) for k in range(levels)]


def initial_data(inst):
    """(phi, pi) complex arrays of shape (n_theta, n_r) for an instance.

    init = None: zero fields.  init = {"center", "width", "amps": {l: A}}:
    Phi = sum_l A_l exp(-(r* - c)^2 / (2 w^2)) Y_l(theta), Pi = 0
    (width is a standard deviation)."""
    n_r, n_th = inst["n_r"], inst["n_theta"]
    phi = np.zeros((n_th, n_r), np.complex128)
    pi = np.zeros((n_th, n_r), np.complex128)
    init = inst.get("init")
    if not init:
        return phi, pi
    rs = inst["rstar_min"] + np.arange(n_r) * (
        (inst["rstar_max"] - inst["rstar_min"]) / (n_r - 1))
    th = np.arange(n_th) * (math.pi / (n_th - 1))
    g = np.exp(-(rs - init["center"]) ** 2 / (2.0 * init["width"] ** 2))
    for l, A in init["amps"].items():
        phi += complex(A) * np.outer(swsh_profile(inst["s"], inst["m"], int(l), th), g)
    # Dirichlet radial boundaries
    phi[:, 0] = 0
    phi[:, -1] = 0
    return phi, pi


def _rand_amp(rng):
    return complex(rng.standard_normal(), rng.standard_normal()) / math.sqrt(2.0)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def schwarzschild_801x33():
    """Schwarzschild a=0, s=-2, m=2, source-free; r* in [-100, 100] with 801
    points, theta with 33 points; Gaussian pulse (center 10M, sd 4M) times the
    l=2 profile, Pi = 0; waveform at r* = 90M; T = 100M."""
    inst = instance(a=0.0, m=2, n_r=801, n_theta=33, rstar_min=-100.0,
                    rstar_max=100.0, dt=1.0 / 40, rstar_obs=90.0,
                    init=dict(center=10.0, width=4.0, amps={2: 1.0}), name="C1")
    return dict(instances=[inst], steps=4000, T=100.0)


def kerr_8001x129():
    """Kerr a=0.9, s=-2, m=2, source-free; 8001 x 129 on [-300, 300]M;
    Gaussian (center 20M, sd 6M) times A_2 Y_2 + A_3 Y_3, A_l complex normal;
    T = 1000M."""
    rng = rng_for(2)
    amps = {2: _rand_amp(rng), 3: _rand_amp(rng)}
    inst = instance(a=0.9, m=2, n_r=8001, n_theta=129, rstar_min=-300.0,
                    rstar_max=300.0, dt=1.0 / 300,
                    init=dict(center=20.0, width=6.0, amps=amps), name="C2")
    return dict(instances=[inst], steps=300000, T=1000.0)


def kerr_sourced_16001x257():
    """Kerr a=0.9, m=2, particle on a prograde circular equatorial orbit at
    r0 = 10M, Gaussian 2 cells wide in r* and theta, seeded phase; 16001 x 257
    on [-300, 300]M; zero initial data; waveform at r* = 290M every 1M;
    T = 5000M."""
    rng = rng_for(3)
    src = dict(r0=10.0, amplitude=1.0, phase0=float(rng.uniform(0, 2 * math.pi)),
               sigma_r_cells=2.0, sigma_th_cells=2.0, window_sigmas=6.0)
    inst = instance(a=0.9, m=2, n_r=16001, n_theta=257, rstar_min=-300.0,
                    rstar_max=300.0, dt=1.0 / 700, source=src, name="C3")
    return dict(instances=[inst], steps=3500000, T=5000.0)


def batched_40_uneven():
    """Batched, uneven sizes: m = 1..8 x a in {0, 0.3, 0.6, 0.9, 0.99}
    (40 instances).  Per instance: N_r uniform in 4001..16001, N_theta odd
    uniform in 33..257, r* in [-300, 300]M; half Gaussian initial data (the
    8001 x 129 workload's form), half circular-orbit sources with r0 in
    [6, 15]M; per-instance stable time step."""
    rng = rng_for(4)
    insts = []
    for m in range(1, 9):
        for a in (0.0, 0.3, 0.6, 0.9, 0.99):
            n_r = int(rng.integers(4001, 16002))
            n_th = 2 * int(rng.integers(16, 129)) + 1
            if rng.uniform() < 0.5:
                l0 = max(abs(m), 2)
                init = dict(center=20.0, width=6.0,
                            amps={l0: _rand_amp(rng), l0 + 1: _rand_amp(rng)})
                src = None
            else:
                init = None
                src = dict(r0=float(rng.uniform(6.0, 15.0)), amplitude=1.0,
                           phase0=float(rng.uniform(0, 2 * math.pi)),
                           sigma_r_cells=2.0, sigma_th_cells=2.0, window_sigmas=6.0)
            insts.append(instance(a=a, m=m, n_r=n_r, n_theta=n_th,
                                  rstar_min=-300.0, rstar_max=300.0,
                                  source=src, init=init, name=f"C4.m{m}.a{a}"))
    return dict(instances=insts, steps=1000, T=None)


def six_modes_16001x129():
    """Precision study: m = 2, 3, 4 x a in {0.5, 0.9}; circular orbits at
    r0 = 8M; 16001 x 129 on [-300, 300]M; dt = 1/500; T = 20000M."""
    rng = rng_for(5)
    insts = []
    for m in (2, 3, 4):
        for a in (0.5, 0.9):
            src = dict(r0=8.0, amplitude=1.0, phase0=float(rng.uniform(0, 2 * math.pi)),
                       sigma_r_cells=2.0, sigma_th_cells=2.0, window_sigmas=6.0)
            insts.append(instance(a=a, m=m, n_r=16001, n_theta=129,
                                  rstar_min=-300.0, rstar_max=300.0,
                                  dt=1.0 / 500, source=src, name=f"C5.m{m}.a{a}"))
    return dict(instances=insts, steps=10000000, T=20000.0)


WORKLOADS = {f.__name__: f for f in (schwarzschild_801x33, kerr_8001x129, kerr_sourced_16001x257,
                                        batched_40_uneven, six_modes_16001x129)}


def points(insts):
    return sum(i["n_r"] * i["n_theta"] for i in insts)
