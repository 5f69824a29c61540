"""CPU model of FP32 arithmetic forms of the scheme (tests/fp32c_model.c).

The model is first pinned to the oracle: with every FP32 switch off it is the
FP64 scheme of Eqs. (3)-(4), plain and with the hyperboloidal layer.  Then it
shows where single precision enters the compensated form's error: a weighted
sum of the three theta rows' values (weights of size cthth / dtheta^2, the
form the FP32 kernels first used) makes the error grow like 1/dtheta^2;
forming the angular differences first removes that growth, and keeping the
Kahan terms in every difference and a compensation term in the half-step
values brings the error down to a few times the storage format's own.
"""
import numpy as np
import pytest

import fp32c_model as FM
from paper_1206_0270_amd import workloads as W


def joint(a, b):
    return float(np.sqrt(np.linalg.norm(a[0] - b[0]) ** 2 + np.linalg.norm(a[1] - b[1]) ** 2)
                 / np.sqrt(np.linalg.norm(b[0]) ** 2 + np.linalg.norm(b[1]) ** 2))


def kerr_instance(n_theta, layer=0.0, n_r=401):
    return W.instance(a=0.9, m=2, n_r=n_r, n_theta=n_theta, rstar_min=-20.0, rstar_max=30.0, rstar_obs=20.0,
                      dt=1.0 / 500, extract_every=50, init=dict(center=5.0, width=3.0, amps={2: 1.0, 3: 0.5j}),
                      source=dict(r0=8.0, phase0=0.3), layer_start=layer)


def run(inst, form, steps, planes):
    m = FM.Model(inst, form, planes)
    m.set_state(*W.initial_data(inst))
    m.run(steps)
    return m.get_state(), m.waveform()


@pytest.mark.parametrize("layer", [0.0, 20.0])
def test_fp64_form_is_the_oracle(layer):
    inst = kerr_instance(33, layer)
    steps = 300
    (state, wave) = run(inst, "fp64", steps, FM.planes_of(inst))
    g = FM.oracle_grid(inst)
    g.set_state(*W.initial_data(inst))
    g.run(steps)
    ref = g.get_state()
    assert joint(state, ref) < 1e-13
    assert np.abs(wave - g.waveform()).max() <= 1e-13 * max(np.abs(g.waveform()).max(), 1e-300)


def test_storage_format_alone_keeps_about_32_bits():
    inst = kerr_instance(33)
    planes = FM.planes_of(inst)
    ref, _ = run(inst, "fp64", 300, planes)
    got, _ = run(inst, "store", 300, planes)
    e = joint(got, ref)
    assert 0 < e < 5e-9, e


def test_angular_weighted_sum_is_the_dtheta_squared_term():
    steps = 1000
    err = {}
    for nth in (33, 129):
        inst = kerr_instance(nth)
        planes = FM.planes_of(inst)
        ref, _ = run(inst, "fp64", steps, planes)
        for form in ("values", "values+ang", "differences", "store"):
            got, _ = run(inst, form, steps, planes)
            err[(form, nth)] = joint(got, ref)
    print({f"{k[0]}@{k[1]}": f"{v:.2e}" for k, v in err.items()})
    # the weighted sum of values grows with the theta resolution ...
    assert err[("values", 129)] > 4 * err[("values", 33)]
    # ... and at 129 rows most of it is the angular term
    assert err[("values+ang", 129)] < err[("values", 129)] / 4
    # every difference from compensated values: no growth with resolution,
    # far below the first form, a few times the storage format's own error
    assert err[("differences", 129)] < 1.5 * err[("differences", 33)]
    assert err[("differences", 129)] < err[("values", 129)] / 15
    assert err[("differences", 129)] < 20 * err[("store", 129)]
