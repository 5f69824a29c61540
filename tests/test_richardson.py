"""Richardson extrapolation (Section 2.3, item 3) and its two-extrapolant
error estimate (Section 5.1, footnote): the oracle's version pinned on exact
data and on manufactured solutions of Eq. (1), and the library's host
routine against it."""
import numpy as np
import pytest

import oracle.richardson as OR
from paper_1206_0270_amd import tk

import test_oracle_pins as PINS


def test_extrapolant_is_exact_for_a_pure_second_order_error():
    rng = np.random.default_rng(3)
    u = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    c = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    w = [u + c * h * h for h in (0.2, 0.1, 0.05)]
    ext, err = OR.richardson(*w)
    assert np.max(np.abs(ext - u)) < 1e-14 * np.max(np.abs(u)) + 1e-15
    assert np.max(err) < 1e-13


def test_extrapolant_leaves_the_next_order_and_estimates_it():
    # u(h) = u* + C h^2 + D h^3: the extrapolant's error is O(h^3) and the
    # two extrapolants differ by (1 - 1/8) times the coarse pair's error
    u, C, D = 1.0 + 0.5j, 2.0 - 1.0j, 3.0 + 0.25j
    hs = (0.1, 0.05, 0.025)
    w = [np.array([u + C * h ** 2 + D * h ** 3]) for h in hs]
    ext, err = OR.richardson(*w)
    e_fine_pair = abs(ext[0] - u)
    e_coarse_pair = abs(OR.extrapolant(w[0], w[1])[0] - u)
    assert e_coarse_pair / e_fine_pair == pytest.approx(8.0, rel=1e-6)   # third order
    assert err[0] * abs(ext[0]) == pytest.approx(e_coarse_pair - e_fine_pair, rel=1e-6)
    # p = 3 removes the cubic term when the quadratic one is absent
    w3 = [np.array([u + D * h ** 3]) for h in hs]
    assert abs(OR.richardson(*w3, order=3)[0][0] - u) < 1e-14


def test_extrapolation_of_manufactured_solutions_beats_the_finest_grid():
    # The same Eq. (1) solution at three resolutions (h, dtheta, dt halved
    # together): the extrapolant, compared at the coarse points with the
    # exact solution, must be far more accurate than the finest result, and
    # the two-extrapolant estimate must bound the coarse-pair error's size.
    levels = ((201, 17), (401, 33), (801, 65))
    phis, exact = [], None
    for k, (n_r, n_th) in enumerate(levels):
        steps = 64 * (n_r - 1) // 200
        phi, ex = PINS._mms_error(1.0, 0.7, -2, 2, n_r, n_th, steps, 4.0, fields=True)
        f = 2 ** k
        phis.append(phi[::f, ::f])
        if exact is None:
            exact = ex
    scale = np.max(np.abs(exact))
    e_raw = np.max(np.abs(phis[2] - exact)) / scale
    ext, est = OR.richardson(*phis)
    e_ext = np.max(np.abs(ext - exact)) / scale
    e_cp = np.max(np.abs(OR.extrapolant(phis[0], phis[1]) - exact)) / scale
    assert e_ext < e_raw / 8, (e_raw, e_ext)
    # the estimate (absolute form) is within a factor 3 of the coarse pair's true error
    est_abs = np.max(np.abs(ext - OR.extrapolant(phis[0], phis[1]))) / scale
    assert e_cp / 3 < est_abs < 3 * e_cp, (e_cp, est_abs)


def test_library_routine_matches_the_oracle():
    rng = np.random.default_rng(11)
    shp = (37, 9)
    w = [rng.standard_normal(shp) + 1j * rng.standard_normal(shp) for _ in range(3)]
    for order in (1, 2, 3):
        ext, err = tk.richardson(*w, order=order)
        oext, oerr = OR.richardson(*w, order=order)
        assert np.max(np.abs(ext - oext)) <= 4e-16 * np.max(np.abs(oext))
        assert np.max(np.abs(err - oerr)) <= 1e-14 * np.max(oerr)


def test_library_routine_errors():
    z = np.zeros(4, np.complex128)
    bad = z.copy()
    bad[2] = np.nan
    with pytest.raises(tk.TkError) as ei:
        tk.richardson(z, bad, z)
    assert ei.value.status == tk.TK_E_NONFINITE
    with pytest.raises(tk.TkError) as ei:
        tk.richardson(z, z, z, order=0)
    assert ei.value.status == tk.TK_E_INVALID
    with pytest.raises(ValueError):
        tk.richardson(z, z[:3], z)


def _projected(inst, wave):
    from paper_1206_0270_amd import workloads as W
    nt = inst["n_theta"]
    th = np.arange(nt) * np.pi / (nt - 1)
    Y = W.swsh_profile(inst["s"], inst["m"], max(abs(inst["m"]), 2), th)
    return wave @ (Y * 2 * np.pi * np.sin(th) * (np.pi / (nt - 1)))


@pytest.mark.gpu
def test_richardson_of_gpu_waveforms_matches_the_oracle_pipeline():
    # three resolutions of a sourced Kerr mode on the GPU; projected
    # waveforms extrapolated by the library, against the same pipeline on
    # the oracle
    from paper_1206_0270_amd import workloads as W
    import test_gpu_parity as GP
    base = W.instance(a=0.9, m=2, n_r=101, n_theta=9, rstar_min=-20.0, rstar_max=30.0, rstar_obs=25.0,
                      source=dict(r0=8.0, phase0=0.4), name="rich")
    fam = W.richardson_family(base)
    T = 30.0
    gw, ow = [], []
    for inst in fam:
        steps = int(round(T / inst["dt"]))
        (phi, pi, wave), = GP.gpu_run([inst], steps)
        gw.append(_projected(inst, wave))
        ow.append(_projected(inst, GP.oracle_run(inst, steps)[2]))
    assert all(len(w) == len(gw[0]) > 10 for w in gw + ow)
    gext, gerr = tk.richardson(*gw)
    oext, oerr = OR.richardson(*ow)
    rel = np.linalg.norm(gext - oext) / np.linalg.norm(oext)
    GP.say("extrapolated waveform rel L2 GPU vs oracle", f"{rel:.2e}",
           "estimate max", f"{np.max(oerr[np.abs(oext) > 1e-3 * np.abs(oext).max()]):.2e}")
    assert rel < 1e-11
    sel = np.abs(oext) > 1e-3 * np.abs(oext).max()
    assert np.max(np.abs(gerr[sel] - oerr[sel])) < 1e-8
