"""The allocation-free autotuner (tk_autotune_static, save area in the
library's static scratch array) against tk_autotune (caller save area),
through the C ABI: both leave the simulation exactly as they found it, and
stepping on with the shape each one chose gives the same results (bitwise,
or within the FP64 parity bar when one of them chose the two-pass kernel,
which agrees with the fused ones up to rounding order).  Two calls in a row,
the second on a smaller workload; a workload larger than the static area is
refused with nothing changed."""
import numpy as np
import pytest

from paper_1206_0270_amd import tk
from paper_1206_0270_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)


def joint_rel(p1, q1, p0, q0):
    num = np.sqrt(np.linalg.norm(p1 - p0) ** 2 + np.linalg.norm(q1 - q0) ** 2)
    den = np.sqrt(np.linalg.norm(p0) ** 2 + np.linalg.norm(q0) ** 2)
    return float(num / den) if den > 0 else float(num)


def workload(big):
    rng = W.rng_for(77 if big else 78)
    shapes = [(4001, 129, 0.9, 2), (2999, 65, 0.5, 3), (1500, 33, 0.0, 1)] if big else [(777, 21, 0.6, 2)]
    out = []
    for k, (n_r, n_th, a, m) in enumerate(shapes):
        src = dict(r0=8.0, phase0=float(rng.uniform(0, 6.28))) if k % 2 == 0 else None
        init = None if src else dict(center=2.0, width=3.0, amps={max(m, 2): complex(rng.standard_normal(), 1.0)})
        out.append(W.instance(a=a, m=m, n_r=n_r, n_theta=n_th, rstar_min=-40.0, rstar_max=60.0, rstar_obs=50.0,
                              extract_every=4, source=src, init=init, name=f"na.{n_r}x{n_th}"))
    return out


def stepper(insts, precision):
    st = tk.Stepper(insts, precision=precision, wave_capacity=512)
    for k, inst in enumerate(insts):
        st.set_fields(k, *W.initial_data(inst))
    return st


def state(st, n):
    return [st.get_fields(k) for k in range(n)]


def run_pair(insts, precision):
    n = len(insts)
    a, b = stepper(insts, precision), stepper(insts, precision)
    a.step(9)
    b.step(9)
    before = state(b, n)
    step0 = b.step_index
    ms_a, tried_a = a.autotune(warmup=2, steps=4)
    ms_b, tried_b = b.autotune_static(warmup=2, steps=4)
    say(f"  autotune: {tried_a} shapes, best {ms_a:.4f} ms {a.get_tuning()}; "
        f"static: {tried_b} shapes, best {ms_b:.4f} ms {b.get_tuning()}")
    assert tried_a == tried_b > 0
    # the simulation is left as it was found, bit for bit
    assert b.step_index == step0 == a.step_index
    for (p0, q0), (p1, q1) in zip(before, state(b, n)):
        assert np.array_equal(p0, p1) and np.array_equal(q0, q1)
    for (p0, q0), (p1, q1) in zip(before, state(a, n)):
        assert np.array_equal(p0, p1) and np.array_equal(q0, q1)
    # stepping on with the chosen shapes: the same results
    a.step(21)
    b.step(21)
    two_pass = tk.TK_KERNEL_TWO_PASS in (a.get_tuning()["kernel"], b.get_tuning()["kernel"])
    worst = 0.0
    for k in range(n):
        (pa, qa), (pb, qb) = a.get_fields(k), b.get_fields(k)
        wa, wb = a.extract(k), b.extract(k)
        assert wa.shape == wb.shape == (30 // 4, insts[k]["n_theta"])
        if two_pass:
            e = joint_rel(pb, qb, pa, qa)
            worst = max(worst, e)
            assert e <= TOL, (k, e)
            assert np.linalg.norm(wb - wa) <= TOL * max(np.linalg.norm(wa), 1e-300)
        else:
            assert np.array_equal(pa, pb) and np.array_equal(qa, qb), k
            assert np.array_equal(wa, wb), k
    say(f"  stepping on: {'two-pass chosen, worst joint rel L2 %.2e' % worst if two_pass else 'bitwise equal'}")
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
def test_static_autotune_matches_autotune_twice_in_a_row(precision):
    for big in (True, False):
        insts = workload(big)
        say(f"no-alloc autotune, precision {precision}, {W.points(insts)} points")
        run_pair(insts, precision)


def test_static_autotune_refuses_a_state_above_its_area():
    inst = W.kerr_sourced_16001x257()["instances"][0]  # 16001 x 257 in FP64: about 132 MB of state
    st = stepper([inst], tk.TK_FP64)
    st.step(3)
    before = st.get_fields(0)
    with pytest.raises(tk.TkError) as e:
        st.autotune_static(warmup=2, steps=4)
    assert e.value.status == tk.TK_E_NOMEM
    assert "static scratch area" in str(e.value)
    assert st.step_index == 3
    after = st.get_fields(0)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    st.close()
