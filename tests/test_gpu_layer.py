"""GPU parity of the hyperboloidal layer (Section 2.3, item 2) against the
oracle's layer, through the C ABI.

Same bar as the other FP64 parity tests: the state (Phi, Pi~) jointly within
relative L2 1e-12, each field and the waveform read at null infinity within
max(1e-12, 4 e_ld) (e_ld: the FP64 oracle's distance to its long-double
build on the same run).  Contexts mix layered and plain instances, ragged
sizes, both pole rules, sourced and source-free runs.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1206_0270_amd import tk
from paper_1206_0270_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_run(inst, steps, kind="f64"):
    g = oracle.Grid(M=inst["M"], a=inst["a"], s=inst["s"], m=inst["m"], n_r=inst["n_r"],
                    n_theta=inst["n_theta"], rstar_min=inst["rstar_min"], rstar_max=inst["rstar_max"],
                    dt=inst["dt"], i_obs=inst["i_obs"], extract_every=inst["extract_every"],
                    source=inst.get("source"), layer_R=inst.get("layer_start", 0.0), kind=kind)
    g.set_state(*W.initial_data(inst))
    g.run(steps)
    phi, pi = g.get_state()
    return phi, pi, g.waveform()


def check(inst, steps, got, ref):
    phi, pi, wave = got
    ophi, opi, owave = ref
    num = np.sqrt(np.linalg.norm(phi - ophi) ** 2 + np.linalg.norm(pi - opi) ** 2)
    den = np.sqrt(np.linalg.norm(ophi) ** 2 + np.linalg.norm(opi) ** 2)
    e = dict(joint=num / den, phi=rel(phi, ophi), pi=rel(pi, opi), wave=rel(wave, owave))
    say(inst["name"], {k: f"{v:.2e}" for k, v in e.items()})
    assert wave.shape == owave.shape and owave.size > 0
    assert e["joint"] <= TOL, e
    if max(e["phi"], e["pi"], e["wave"]) > TOL:
        lphi, lpi, lwave = oracle_run(inst, steps, kind="ld")
        floor = dict(phi=rel(ophi, lphi), pi=rel(opi, lpi), wave=rel(owave, lwave))
        say("  oracle double vs long double:", {k: f"{v:.2e}" for k, v in floor.items()})
        for k in ("phi", "pi", "wave"):
            assert e[k] <= max(TOL, 4 * floor[k]), (k, e[k], floor[k])


def gpu_run(insts, steps, graph=0, chunks=None, rows=0, autotune=False, kernel=tk.TK_KERNEL_AUTO,
            precision=tk.TK_FP64, counters=None):
    st = tk.Stepper(insts, force_dt=False, precision=precision)
    st.set_tuning(kernel=kernel, graph_steps=graph, rows_per_tile=rows)
    for k, inst in enumerate(insts):
        st.set_fields(k, *W.initial_data(inst))
    if autotune:
        _, tried = st.autotune(warmup=2, steps=4)
        assert tried >= 4
    for n in (chunks or [steps]):
        st.step(n)
    out = [st.get_fields(k) + (st.extract(k),) for k in range(len(insts))]
    if counters is not None:
        counters.update(st.counters())
    st.close()
    return out


def layered_instances():
    rng = W.rng_for(1206)
    out = []
    for (n_r, n_th, a, m, src, R, S, lay) in [(201, 17, 0.5, 2, False, 30.0, 50.0, True),
                                              (163, 13, 0.9, 3, True, 25.0, 40.0, True),
                                              (150, 9, 0.0, 2, False, 20.0, 45.0, True),
                                              (130, 11, 0.7, -2, True, 0.0, 30.0, False),
                                              (97, 7, 0.3, 4, False, 10.0, 30.0, True)]:
        init = None if src else dict(center=2.0, width=3.0,
                                     amps={max(abs(m), 2): complex(rng.standard_normal(), rng.standard_normal())})
        source = dict(r0=6.0 + 3 * rng.uniform(), phase0=float(rng.uniform(0, 6.28)), sigma_r_cells=2.0,
                      sigma_th_cells=2.0, window_sigmas=6.0, ramp=5.0) if src else None
        h = (S + 40.0) / (n_r - 1)
        dt = W.stable_dt(a, m, -2, h, n_th)
        out.append(W.instance(a=a, m=m, n_r=n_r, n_theta=n_th, rstar_min=-40.0, rstar_max=S, dt=dt,
                              rstar_obs=S if lay else S - 5.0, extract_every=3, init=init, source=source,
                              layer_start=R if lay else 0.0,
                              name=f"layer.{n_r}x{n_th}.a{a}.m{m}.R{R}.S{S}"))
    return out


def test_layer_small_grids_vs_oracle():
    insts = layered_instances()
    steps = 400
    say("layered contexts", [i["name"] for i in insts])
    res = gpu_run(insts, steps)
    for inst, got in zip(insts, res):
        check(inst, steps, got, oracle_run(inst, steps))


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
def test_layer_graph_and_chunks_bitwise(precision):
    insts = layered_instances()[:3]
    a = gpu_run(insts, 250, precision=precision)
    cnt = {}
    b = gpu_run(insts, 250, graph=40, chunks=[7, 120, 123], counters=cnt, precision=precision)
    assert cnt["graphs_instantiated"] == 1 and cnt["graph_launches"] == 6, cnt  # 3 + 3 replays of 40 steps
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_layer_row_chunks_kernels_and_autotune():
    """Three forms step a layered FP64 context: the two-step marching pass
    (AUTO, FUSED2), the one-step marching pass (FUSED), both with the layer's
    coefficients beyond rho = R and null infinity extrapolated inside the
    pass, and the two-pass layer kernels.  FUSED2 is bitwise FUSED, whole
    strips or chunks of rows (and an odd step count); within each form every
    chunking of rows gives the same bits; the two-pass form agrees to
    rounding (it orders the interior arithmetic differently), and so does the
    autotuner's choice."""
    insts = layered_instances()
    ref = {}
    for kernel in (tk.TK_KERNEL_FUSED, tk.TK_KERNEL_TWO_PASS):
        ref[kernel] = gpu_run(insts, 120, kernel=kernel)
        for rows in (3, 8, 64, 200):
            got = gpu_run(insts, 120, rows=rows, kernel=kernel)
            for x, y in zip(ref[kernel], got):
                for u, v in zip(x, y):
                    assert np.array_equal(u, v), (kernel, rows)
    for rows in (0, 4, 16):
        got = gpu_run(insts, 120, rows=rows, kernel=tk.TK_KERNEL_FUSED2)
        for x, y in zip(ref[tk.TK_KERNEL_FUSED], got):
            for u, v in zip(x, y):
                assert np.array_equal(u, v), ("FUSED2", rows)
    odd = gpu_run(insts, 121, kernel=tk.TK_KERNEL_FUSED2)
    odd1 = gpu_run(insts, 121, kernel=tk.TK_KERNEL_FUSED)
    for x, y in zip(odd1, odd):
        for u, v in zip(x, y):
            assert np.array_equal(u, v), "odd step count"
    auto = gpu_run(insts, 120)
    for x, y in zip(ref[tk.TK_KERNEL_FUSED], auto):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    tuned = gpu_run(insts, 120, autotune=True)
    for inst, a, b, c in zip(insts, ref[tk.TK_KERNEL_FUSED], ref[tk.TK_KERNEL_TWO_PASS], tuned):
        for u, v, w in zip(a, b, c):
            assert rel(v, u) <= 1e-13 and rel(w, u) <= 1e-13, inst["name"]


@pytest.mark.parametrize("n_r", [121, 122, 125, 126])
def test_layer_last_strip_holds_null_infinity(n_r):
    """Radial sizes that leave the marching kernels' last strip (62 columns
    one-step, 60 two-step) with one or two columns: that strip is moved back
    to hold the last three, so that null infinity is extrapolated inside it.
    Against the oracle, and the two-step pass bitwise the one-step one."""
    S = 40.0
    h = (S + 40.0) / (n_r - 1)
    inst = W.instance(a=0.7, m=2, n_r=n_r, n_theta=11, rstar_min=-40.0, rstar_max=S, layer_start=20.0,
                      dt=W.stable_dt(0.7, 2, -2, h, 11), rstar_obs=S, extract_every=3,
                      init=dict(center=10.0, width=3.0, amps={2: 1.0 - 0.5j}), name=f"layer.{n_r}x11.tail")
    steps = 300
    one, = gpu_run([inst], steps, kernel=tk.TK_KERNEL_FUSED)
    two, = gpu_run([inst], steps, kernel=tk.TK_KERNEL_FUSED2)
    for u, v in zip(one, two):
        assert np.array_equal(u, v)
    check(inst, steps, two, oracle_run(inst, steps))
    # the compensated form: the same bitwise relation, and within its bar of FP64
    one32, = gpu_run([inst], steps, kernel=tk.TK_KERNEL_FUSED, precision=tk.TK_FP32_COMP)
    two32, = gpu_run([inst], steps, kernel=tk.TK_KERNEL_FUSED2, precision=tk.TK_FP32_COMP)
    for u, v in zip(one32, two32):
        assert np.array_equal(u, v)
    e = [rel(a, b) for a, b in zip(two32, two)]
    say(inst["name"], "fp32c vs fp64", [f"{x:.2e}" for x in e])
    assert max(e) <= 2e-5, e


def test_layer_random_grids_vs_oracle():
    """Seeded random layered grids (ragged radial sizes around the strip
    widths, 5 to 41 rows, layers from two cells to half the domain, spins
    and m of both pole rules, sourced and source-free) in one context, the
    two-step layered form in whole strips (AUTO) and in 4-row chunks, each
    against the oracle's layer after 200 steps, and the two bitwise equal."""
    rng = W.rng_for(2024)
    insts = []
    for k in range(8):
        n_r = int(rng.choice([61, 62, 63, 64, 119, 120, 121, 122, 181, 183]))
        n_th = int(rng.choice([5, 6, 9, 17, 23, 41]))
        a = float(rng.choice([0.0, 0.5, 0.9, 0.99]))
        m = int(rng.choice([-3, -2, 1, 2, 3, 4]))
        S = float(rng.uniform(25.0, 60.0))
        h = (S + 40.0) / (n_r - 1)
        R = float(rng.uniform(max(0.5 * S, 10.0), S - 2.5 * h))
        src = k % 2 == 1
        init = None if src else dict(center=0.5 * R, width=3.0, amps={max(abs(m), 2): 1.0 + 0.3j})
        source = dict(r0=6.0 + 2 * rng.uniform(), phase0=0.4, sigma_r_cells=2.0, sigma_th_cells=1.5,
                      window_sigmas=5.0, ramp=3.0) if src else None
        insts.append(W.instance(a=a, m=m, n_r=n_r, n_theta=n_th, rstar_min=-40.0, rstar_max=S,
                                dt=W.stable_dt(a, m, -2, h, n_th), rstar_obs=S, extract_every=4, init=init,
                                source=source, layer_start=R, name=f"rnd{k}.{n_r}x{n_th}.a{a}.m{m}.R{R:.1f}.S{S:.1f}"))
    steps = 200
    say("random layered grids", [i["name"] for i in insts])
    whole = gpu_run(insts, steps)
    chunks = gpu_run(insts, steps, kernel=tk.TK_KERNEL_FUSED2, rows=4)
    for inst, a, b in zip(insts, whole, chunks):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), inst["name"]
        check(inst, steps, a, oracle_run(inst, steps))


def test_layer_strips_chunked_beside_whole_ones():
    """With whole strips asked for (rows_per_tile 0), the strips whose lanes
    reach the layer are cut into chunks of 32 rows and the others run whole,
    in one pass of the chunked two-step kernel.  73 rows (chunks of 32, 32,
    9): bitwise the one-step pass and uniform chunks, and the oracle."""
    S = 40.0
    n_r, n_th = 250, 73
    h = (S + 40.0) / (n_r - 1)
    inst = W.instance(a=0.9, m=2, n_r=n_r, n_theta=n_th, rstar_min=-40.0, rstar_max=S, layer_start=20.0,
                      dt=W.stable_dt(0.9, 2, -2, h, n_th), rstar_obs=S, extract_every=5,
                      init=dict(center=10.0, width=3.0, amps={2: 1.0, 3: 0.25j}), name="layer.250x73.mixed")
    steps = 160
    mixed, = gpu_run([inst], steps, kernel=tk.TK_KERNEL_FUSED2)
    for kernel, rows in ((tk.TK_KERNEL_FUSED, 0), (tk.TK_KERNEL_FUSED2, 16)):
        other, = gpu_run([inst], steps, kernel=kernel, rows=rows)
        for u, v in zip(mixed, other):
            assert np.array_equal(u, v), (kernel, rows)
    check(inst, steps, mixed, oracle_run(inst, steps))
    mixed32, = gpu_run([inst], steps, kernel=tk.TK_KERNEL_FUSED2, precision=tk.TK_FP32_COMP)
    for kernel, rows in ((tk.TK_KERNEL_FUSED, 0), (tk.TK_KERNEL_FUSED2, 16)):
        other, = gpu_run([inst], steps, kernel=kernel, rows=rows, precision=tk.TK_FP32_COMP)
        for u, v in zip(mixed32, other):
            assert np.array_equal(u, v), ("fp32c", kernel, rows)
    e = [rel(a, b) for a, b in zip(mixed32, mixed)]
    say(inst["name"], "fp32c vs fp64", [f"{x:.2e}" for x in e])
    assert max(e) <= 2e-5, e


def test_layer_second_workload_size():
    """8001 x 129 on [-300, 300] with a layer on [250, 300]: the second
    workload's grid, read at null infinity; 300 steps against the oracle."""
    inst = W.instance(a=0.9, m=2, n_r=8001, n_theta=129, rstar_min=-300.0, rstar_max=300.0,
                      layer_start=250.0, extract_every=20,
                      init=dict(center=240.0, width=4.0, amps={2: 1.0 + 0.5j}), name="layer.8001x129.a0.9")
    steps = 300
    say(inst["name"], "steps", steps)
    got, = gpu_run([inst], steps, graph=100)
    check(inst, steps, got, oracle_run(inst, steps))


def test_layer_16001x129_pulse_in_the_layer():
    """16001 x 129 on [-300, 300]M with a layer on [250, 300]M, the six-mode
    workload's grid, with a pulse placed inside the layer so that the layer's
    columns and null infinity carry the field from the first step: 400 steps
    of the autotuner's default shape (two steps a pass, the layer's strips in
    chunks beside whole strips) against the oracle's layer, the waveform read
    at null infinity."""
    inst = W.instance(a=0.9, m=2, n_r=16001, n_theta=129, rstar_min=-300.0, rstar_max=300.0, layer_start=250.0,
                      extract_every=20, init=dict(center=275.0, width=5.0, amps={2: 1.0 - 0.5j, 3: 0.3j}),
                      name="layer.16001x129.a0.9.pulse_in_layer")
    steps = 400
    say(inst["name"], "steps", steps)
    got, = gpu_run([inst], steps, graph=100)
    check(inst, steps, got, oracle_run(inst, steps))


def test_layer_fp32c_vs_fp64():
    """FP32-compensated storage with layers: the marching kernels' layered
    compensated form (the layer's coefficients in the differences form's
    FP32, null infinity extrapolated in double on f + c).  Against the FP64
    run after 150 steps: the FP32C bar of the plain grids (fields within
    relative L2 2e-5), the waveform at null infinity too; the two-step pass
    (AUTO, FUSED2 in whole strips and in chunks) bitwise the one-step one in
    any chunking, odd step counts included."""
    insts = layered_instances()
    ref = gpu_run(insts, 150)
    got = gpu_run(insts, 150, precision=tk.TK_FP32_COMP)
    for inst, (p64, q64, w64), (p32, q32, w32) in zip(insts, ref, got):
        e = dict(phi=rel(p32, p64), pi=rel(q32, q64), wave=rel(w32, w64))
        say(inst["name"], "fp32c vs fp64", {k: f"{v:.2e}" for k, v in e.items()})
        assert max(e.values()) <= 2e-5, e
    for kernel, rows in ((tk.TK_KERNEL_FUSED, 0), (tk.TK_KERNEL_FUSED, 3), (tk.TK_KERNEL_FUSED, 64),
                         (tk.TK_KERNEL_FUSED2, 4), (tk.TK_KERNEL_FUSED2, 16)):
        again = gpu_run(insts, 150, precision=tk.TK_FP32_COMP, rows=rows, kernel=kernel)
        for x, y in zip(got, again):
            for u, v in zip(x, y):
                assert np.array_equal(u, v), (kernel, rows)
    odd = gpu_run(insts, 151, precision=tk.TK_FP32_COMP, kernel=tk.TK_KERNEL_FUSED2)
    odd1 = gpu_run(insts, 151, precision=tk.TK_FP32_COMP, kernel=tk.TK_KERNEL_FUSED)
    for x, y in zip(odd1, odd):
        for u, v in zip(x, y):
            assert np.array_equal(u, v), "odd step count"


def test_layer_rejections():
    inst = layered_instances()[0]
    st = tk.Stepper([inst], precision=tk.TK_FP32_COMP)
    try:
        with pytest.raises(tk.TkError):   # the two passes keep an FP64 half-step array
            st.set_tuning(kernel=tk.TK_KERNEL_TWO_PASS)
    finally:
        st.close()
    st = tk.Stepper([inst], precision=tk.TK_FP32_COMP)
    try:
        st.set_tuning(kernel=tk.TK_KERNEL_FUSED2)
        with pytest.raises(tk.TkError):
            st.set_tuning(kernel=tk.TK_KERNEL_TILED, rows_per_tile=4)
    finally:
        st.close()
    st = tk.Stepper([inst])
    try:
        st.set_tuning(kernel=tk.TK_KERNEL_FUSED2)
        with pytest.raises(tk.TkError):
            st.set_tuning(kernel=tk.TK_KERNEL_TILED, rows_per_tile=4)
        with pytest.raises(tk.TkError):   # the particle inside the layer
            st.set_source(0, dict(r0=35.0))
        st.set_source(0, dict(r0=8.0))
    finally:
        st.close()
