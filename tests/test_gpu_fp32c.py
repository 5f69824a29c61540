"""GPU checks of the FP32-compensated form against the FP64 path.

FP32 storage and stencil arithmetic with a bf16 Kahan term per value and
FP64 source increments.  Bar: field relative L2 <= 2e-5 after 150 steps on
small grids; set/get round trip keeps ~32 bits; waveform amplitude and phase
errors of the projected waveform well inside 1e-4 on a sourced run.
"""
import sys

import numpy as np
import pytest

from paper_1206_0270_amd import tk
from paper_1206_0270_amd import workloads as W

import test_gpu_parity as GP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(insts, steps, prec, rows=0):
    st = tk.Stepper(insts, precision=prec, force_dt=True)
    st.set_tuning(kernel=tk.TK_KERNEL_FUSED, rows_per_tile=rows)
    for k, inst in enumerate(insts):
        st.set_fields(k, *W.initial_data(inst))
    st.step(steps)
    out = [st.get_fields(k) + (st.extract(k),) for k in range(len(insts))]
    st.close()
    return out


def test_roundtrip_keeps_32_bits():
    inst = GP.small_instances()[1]
    rng = np.random.default_rng(5)
    shp = (inst["n_theta"], inst["n_r"])
    phi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    pi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    st = tk.Stepper([inst], precision=tk.TK_FP32_COMP)
    st.set_fields(0, phi, pi)
    p2, q2 = st.get_fields(0)
    st.close()
    assert GP.rel(p2, phi) < 3e-9 and GP.rel(q2, pi) < 3e-9


def test_small_grids_fp32c_vs_fp64():
    insts = GP.small_instances()
    a = run(insts, 150, tk.TK_FP64)
    b = run(insts, 150, tk.TK_FP32_COMP)
    for inst, x, y in zip(insts, a, b):
        e = (GP.rel(y[0], x[0]), GP.rel(y[1], x[1]), GP.rel(y[2], x[2]))
        say(inst["name"], e)
        assert max(e) < 2e-5, (inst["name"], e)


def test_fp32c_chunking_bitwise():
    insts = GP.small_instances()
    a = run(insts, 30, tk.TK_FP32_COMP, rows=0)
    b = run(insts, 30, tk.TK_FP32_COMP, rows=5)
    for x, y in zip(a, b):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def waveform_errors(inst, steps):
    """S18-style errors of the FP32-compensated waveform against FP64."""
    a = run([inst], steps, tk.TK_FP64)[0][2]
    b = run([inst], steps, tk.TK_FP32_COMP)[0][2]
    th = np.arange(inst["n_theta"]) * np.pi / (inst["n_theta"] - 1)
    Y = W.swsh_profile(-2, inst["m"], max(abs(inst["m"]), 2), th)
    wts = 2 * np.pi * np.sin(th) * (np.pi / (inst["n_theta"] - 1))
    wa = a @ (Y * wts)
    wb = b @ (Y * wts)
    sel = np.abs(wa) >= 1e-3 * np.abs(wa).max()
    amp = float(np.max(np.abs(np.abs(wb[sel]) - np.abs(wa[sel])) / np.abs(wa[sel])))
    ph = float(np.max(np.abs(np.angle(wb[sel] / wa[sel]))))
    return amp, ph


def test_sourced_waveform_error_fp32c_before_reflection():
    # Sourced Kerr run, compared with FP64 over the window before the wave
    # reflected at the outer (Dirichlet) boundary returns from the potential:
    # for s = -2 an ingoing perturbation grows like r^-4 on its way in, so
    # after that every rounding difference is amplified by ~(r_b/3M)^4 and
    # FP64 and FP32 storage diverge alike.  Inside the window the
    # compensated form must hold the paper's 1e-4 waveform target.
    out = {}
    for rmax in (100.0, 200.0):
        inst = W.instance(a=0.9, m=2, n_r=int((rmax + 40) / 0.25) + 1, n_theta=33, rstar_min=-40.0,
                          rstar_max=rmax, rstar_obs=rmax - 10.0, source=dict(r0=8.0, phase0=0.7))
        steps = int(round(150 / inst["dt"]))
        out[rmax] = waveform_errors(inst, steps)
        say("r*_max", rmax, "steps", steps, "amplitude / phase error vs FP64", out[rmax])
    for rmax, (amp, ph) in out.items():
        assert amp < 1e-4 and ph < 1e-4, out


def test_switch_on_run_after_the_reflection_stays_bounded():
    # After the outer-boundary reflection has returned (r*_max = 200M,
    # T = 400M), a source switched on smoothly over 100M keeps the FP32C
    # waveform within the level of the reflected steady wave (bound below).
    # The abrupt start on the same grid is printed as a measurement only: its
    # switch-on burst, ~2000x the steady signal, comes back amplified.
    errs = {}
    for ramp in (0.0, 100.0):
        inst = W.instance(a=0.9, m=2, n_r=int(240 / 0.25) + 1, n_theta=33, rstar_min=-40.0, rstar_max=200.0,
                          rstar_obs=190.0, source=dict(r0=8.0, phase0=0.7, ramp=ramp))
        errs[ramp] = waveform_errors(inst, int(round(400 / inst["dt"])))
        say("switch-on", ramp, "amplitude / phase error vs FP64 to T = 400M", errs[ramp])
    assert max(errs[100.0]) < 5e-3, errs
