"""CPU checks of the library's host-side setup (tortoise inversion and the
coefficient tables the kernels read), compiled from the library's own source
with g++ and compared with closed forms and with the oracle's coefficients."""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1206_0270_amd", "csrc")
EXE = os.path.join(ROOT, "_build", "host_setup_check")


@pytest.fixture(scope="module")
def exe():
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + CSRC, os.path.join(os.path.dirname(__file__), "host_setup_check.cpp"),
                    os.path.join(CSRC, "tk_setup.cpp"), "-o", EXE], check=True)
    return EXE


def tables(exe, M, a, s, m, n_r, n_th, rmin, rmax):
    out = subprocess.run([exe, str(M), str(a), str(s), str(m), str(n_r), str(n_th), str(rmin), str(rmax)],
                         check=True, capture_output=True, text=True).stdout.split("\n")
    R = np.array([[float(v) for v in l.split()[2:]] for l in out if l.startswith("R ")])
    A = np.array([[float(v) for v in l.split()[2:]] for l in out if l.startswith("A ")])
    B = [float(l.split()[1]) for l in out if l.startswith("B ")][0]
    return R, A, B


def point_coeffs(R, A, j):
    """Recombine the library's factored tables into the coefficients."""
    rstar, rho2, a2D, rho, Dl, ct_re, ct_im0, ct_imc, K, c1_re, c1_im, c0_re, c0_im = R.T
    th, sn2, cs, cot, V = A[j]
    Sh2 = rho2 - a2D * sn2
    W = 1 / Sh2
    b = rho * np.sqrt(W)
    ct = W * (ct_re + 1j * (ct_im0 + ct_imc * cs))
    c1 = W * (c1_re + 1j * c1_im)
    c0 = W * (c0_re - Dl * V + 1j * c0_im)
    bp = K * sn2 * W * np.sqrt(W)
    d = -(c1 - b * bp - b * ct)
    return dict(b=b, cthth=Dl * W, ct=ct, c0=c0, d=d)


@pytest.mark.parametrize("a", [0.0, 0.3, 0.9, 0.99])
def test_inverse_tortoise_residual(exe, a):
    R, _, _ = tables(exe, 1.0, a, -2, 2, 2001, 9, -400.0, 400.0)
    rstar = R[:, 0]
    Dl = R[:, 4]
    rp = 1 + math.sqrt(1 - a * a)
    rm = 1 - math.sqrt(1 - a * a)
    # Delta = x (x + r+ - r-): the positive root, in cancellation-free form
    x = 2 * Dl / ((rp - rm) + np.sqrt((rp - rm) ** 2 + 4 * Dl))
    assert np.all(np.isfinite(R)) and np.all(x > 0)
    for xi, rs in zip(x[::37], rstar[::37]):
        back = oracle.tortoise(1.0, a, xi)
        assert abs(back - rs) <= 1e-11 * max(1.0, abs(rs)), (a, rs, back)


@pytest.mark.parametrize("a,m", [(0.9, 2), (0.0, 2), (0.6, -3), (0.99, 8)])
def test_tables_match_oracle_coefficients(exe, a, m):
    n_r, n_th = 201, 17
    R, A, _ = tables(exe, 1.0, a, -2, m, n_r, n_th, -60.0, 80.0)
    g = oracle.Grid(a=a, m=m, n_r=n_r, n_theta=n_th, rstar_min=-60.0, rstar_max=80.0, dt=0.01)
    assert np.allclose(A[:, 0], np.arange(n_th) * np.pi / (n_th - 1), rtol=0, atol=1e-15)
    for q in (1, 2, 57, 200, 201, 399, 400):
        oc = g.coeff_column(q)
        for j in (1, 3, n_th // 2, n_th - 2):
            lc = point_coeffs(R[q:q + 1], A, j)
            for key in ("b", "cthth", "ct", "c0", "d"):
                want = oc[key][j]
                got = lc[key][0]
                scale = max(abs(want), 1e-300)
                if key == "d":  # d = -(c1 - b b' - b ct) cancels to 0 at a = 0
                    scale = max(scale, abs(oc["b"][j] * oc["ct"][j]))
                assert abs(got - want) <= 1e-12 * scale + 1e-300, (q, j, key, got, want)


def test_stability_bound_values(exe):
    # the 801 x 33 workload's grid: 1/40 is admissible, the literal dr*/2 = 0.125 is not
    _, _, B = tables(exe, 1.0, 0.0, -2, 2, 801, 33, -100.0, 100.0)
    assert 1 / 40 <= B < 0.125
    assert abs(B - 0.02560) < 2e-4  # (8*0.01/w^4)^(1/3), w^2 = (2+16)/(27 dth^2)
