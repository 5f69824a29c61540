"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (FP64), element by element on the same seeded inputs:
  * the state u = (Phi, Pi) jointly: relative L2 <= 1e-12;
  * each field and the waveform samples: relative L2 <= max(1e-12, 4 e_ld),
    where e_ld is the FP64 oracle's own distance to its long-double build on
    the same run (only computed when a field misses 1e-12).  When a field
    decays by orders of magnitude while rounding noise accumulates (Pi on the
    801 x 33 workload loses 100x in 100M), no FP64 evaluation order can do
    better than that floor.
Determinism checks (batched vs alone, tile shapes, graph vs eager,
checkpoint/resume) are bitwise.
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


def oracle_run(inst, steps, phi0=None, pi0=None, kind="f64"):
    g = oracle.Grid(M=inst["M"], a=inst["a"], s=inst["s"], m=inst["m"], n_r=inst["n_r"],
                    n_theta=inst["n_theta"], rstar_min=inst["rstar_min"],
                    rstar_max=inst["rstar_max"], dt=inst["dt"], i_obs=inst["i_obs"],
                    extract_every=inst["extract_every"], source=inst.get("source"), kind=kind)
    if phi0 is None:
        phi0, pi0 = W.initial_data(inst)
    g.set_state(phi0, pi0)
    g.run(steps)
    phi, pi = g.get_state()
    return phi, pi, g.waveform()


def joint_rel(phi, pi, ophi, opi):
    num = np.sqrt(np.linalg.norm(phi - ophi) ** 2 + np.linalg.norm(pi - opi) ** 2)
    den = np.sqrt(np.linalg.norm(ophi) ** 2 + np.linalg.norm(opi) ** 2)
    return num / (den if den > 0 else 1.0)


def check_parity(inst, steps, got, ref, phi0=None, pi0=None):
    """Apply the FP64 parity bar; returns the error tuple."""
    phi, pi, wave = got
    ophi, opi, owave = ref
    e = dict(joint=joint_rel(phi, pi, ophi, opi), phi=rel(phi, ophi), pi=rel(pi, opi),
             wave=rel(wave, owave) if owave.size else 0.0)
    say(inst.get("name", ""), {k: f"{v:.2e}" for k, v in e.items()})
    assert wave.shape == owave.shape
    assert e["joint"] <= TOL, e
    if max(e["phi"], e["pi"], e["wave"]) > TOL:
        lphi, lpi, lwave = oracle_run(inst, steps, phi0, pi0, kind="ld")
        floor = dict(phi=rel(ophi, lphi), pi=rel(opi, lpi),
                     wave=rel(owave, lwave) if owave.size else 0.0)
        say("  oracle double vs long double:", {k: f"{v:.2e}" for k, v in floor.items()})
        for k in ("phi", "pi", "wave"):
            assert e[k] <= max(TOL, 4 * floor[k]), (k, e[k], floor[k])
    return e


def gpu_run(insts, steps, kernel=tk.TK_KERNEL_AUTO, rows=0, graph=0, inits=None, chunks=None,
            prefetch=0, nt=True, waves=0, precision=tk.TK_FP64, counters=None):
    st = tk.Stepper(insts, force_dt=True, precision=precision)
    assert st.stream.cuda_stream != 0  # a capturable stream of the Stepper's own
    st.set_tuning(kernel=kernel, rows_per_tile=rows, graph_steps=graph, prefetch_rows=prefetch, nt_stores=nt,
                  waves_per_simd=waves)
    for k, inst in enumerate(insts):
        phi0, pi0 = W.initial_data(inst) if inits is None else inits[k]
        st.set_fields(k, phi0, pi0)
    for n in (chunks or [steps]):
        st.step(n)
    out = [st.get_fields(k) + (st.extract(k, max_samples=4096),) for k in range(len(insts))]
    if counters is not None:
        counters.update(st.counters())
    st.close()
    return out


def expect_graph_replays(cnt, steps_chunks, G):
    """The counters of a run stepped in `steps_chunks` with graph_steps G: one
    graph instantiated, one replay per whole block of G inside each call."""
    replays = sum(n // G for n in steps_chunks) if G > 0 else 0
    assert cnt["graph_launches"] == replays, (cnt, replays)
    assert cnt["graphs_instantiated"] == (1 if replays else 0), cnt


def source_window(inst):
    """Rows and columns of the particle source's window (6 sigma of the
    two-cell Gaussian around the particle), or None without a source."""
    src = inst.get("source")
    if not src:
        return None
    M, a = inst["M"], inst["a"]
    rp = M + np.sqrt(M * M - a * a)
    rsp = oracle.tortoise(M, a, src["r0"] - rp)
    h = (inst["rstar_max"] - inst["rstar_min"]) / (inst["n_r"] - 1)
    dth = np.pi / (inst["n_theta"] - 1)
    rs = inst["rstar_min"] + h * np.arange(inst["n_r"])
    th = dth * np.arange(inst["n_theta"])
    wr = src.get("window_sigmas", 6.0) * src.get("sigma_r_cells", 2.0) * h
    wt = src.get("window_sigmas", 6.0) * src.get("sigma_th_cells", 2.0) * dth
    cols = np.nonzero(np.abs(rs - rsp) <= wr + h)[0]
    rows = np.nonzero(np.abs(th - np.pi / 2) <= wt + dth)[0]
    return rows, cols


def check_local(inst, steps, got, ref, bar=TOL, global_scale=()):
    """Element-wise bar where the solution is most delicate: the source
    window and the rows at and next to the poles.  Each region's largest
    pointwise difference over its largest reference value, per field (over
    the field's largest value anywhere for the regions named in
    global_scale); a region whose reference is exactly zero (odd m + s
    poles) must be exactly zero too.  With the FP64 bar, a region that misses
    it is held to max(bar, 4 e_ld) instead, e_ld being the FP64 oracle's own
    distance to its long-double build in that region: where a region's
    values are orders of magnitude below the rest of the field (the poles of
    a high-m mode), rounding at the scale of the whole field sets the floor,
    whatever the evaluation order."""
    nt = inst["n_theta"]
    regions = {"poles": (np.array([0, 1, nt - 2, nt - 1]), np.arange(inst["n_r"]))}
    win = source_window(inst)
    if win is not None:
        regions["source"] = win
    out = {}
    lref = []
    for name, (rows, cols) in regions.items():
        for k, f in ((0, "phi"), (1, "pi")):
            g, r = got[k], ref[k]
            gs, rs_ = g[np.ix_(rows, cols)], r[np.ix_(rows, cols)]
            scale = np.abs(r).max() if name in global_scale else np.abs(rs_).max()
            if scale == 0.0:
                assert np.all(gs == 0.0), (inst.get("name"), name, f)
                out[f"{name}.{f}"] = 0.0
                continue
            e = float(np.abs(gs - rs_).max() / scale)
            out[f"{name}.{f}"] = e
            if e > bar and bar == TOL:
                if not lref:
                    lref.append(oracle_run(inst, steps, kind="ld"))
                ls = lref[0][k][np.ix_(rows, cols)]
                floor = float(np.abs(rs_ - ls).max() / scale)
                say(f"  {name}.{f}: {e:.2e} against the oracle's long-double distance {floor:.2e}")
                assert e <= max(bar, 4 * floor), (inst.get("name"), name, f, e, floor)
            else:
                assert e <= bar, (inst.get("name"), name, f, e)
    say("  local max-relative:", {k: f"{v:.2e}" for k, v in out.items()})
    return out


def small_instances():
    # ragged sizes (none a multiple of a strip width), 5 to 33 rows, a from 0
    # to 0.99, even and odd m + s (both pole rules), m = 0, spin weights
    # -2, -1, +1, +2, with and without a source
    rng = W.rng_for(99)
    out = []
    for (n_r, n_th, a, m, src, s) in [(101, 9, 0.0, 2, None, -2), (130, 17, 0.9, 2, "s", -2),
                                      (77, 11, 0.6, 3, None, -2), (200, 13, 0.3, -1, "s", -2),
                                      (63, 5, 0.99, 8, None, -2), (125, 33, 0.5, 4, "s", -2),
                                      (96, 7, 0.5, 0, None, -2), (70, 9, 0.8, 1, "s", -1),
                                      (88, 11, 0.3, 2, None, 2), (75, 13, 0.6, -2, None, 1)]:
        init = None if src else dict(center=2.0, width=3.0,
                                     amps={max(abs(m), abs(s), 2): complex(rng.standard_normal(),
                                                                            rng.standard_normal())})
        source = dict(r0=6.0 + 3 * rng.uniform(), phase0=float(rng.uniform(0, 6.28)),
                      sigma_r_cells=2.0, sigma_th_cells=2.0, window_sigmas=6.0) if src else None
        out.append(W.instance(a=a, s=s, m=m, n_r=n_r, n_theta=n_th, rstar_min=-20.0, rstar_max=25.0,
                              rstar_obs=20.0, extract_every=3, init=init, source=source,
                              name=f"small.{n_r}x{n_th}.a{a}.m{m}.s{s}"))
    return out


@pytest.mark.parametrize("kernel", [tk.TK_KERNEL_FUSED2, tk.TK_KERNEL_FUSED, tk.TK_KERNEL_TWO_PASS, tk.TK_KERNEL_TILED])
def test_small_grids_vs_oracle(kernel):
    insts = small_instances()
    steps = 150
    say("small grids", [i["name"] for i in insts], "kernel", kernel)
    res = gpu_run(insts, steps, kernel=kernel, rows=4 if kernel == tk.TK_KERNEL_TILED else 0)
    for inst, got in zip(insts, res):
        check_parity(inst, steps, got, oracle_run(inst, steps))


def test_first_workload_full_run():
    inst = W.schwarzschild_801x33()["instances"][0]
    steps = W.schwarzschild_801x33()["steps"]
    say("Schwarzschild 801x33, steps", steps)
    got, = gpu_run([inst], steps)
    assert got[2].shape == (100, 33)
    check_parity(inst, steps, got, oracle_run(inst, steps))


@pytest.mark.timeout(900)
def test_second_workload_prefix():
    # 8001 x 129, a = 0.9: 3000 steps (10M) in graph replays of 100 steps
    inst = W.kerr_8001x129()["instances"][0]
    steps = 3000
    say("Kerr 8001x129, a=0.9, steps", steps)
    cnt = {}
    got, = gpu_run([inst], steps, graph=100, counters=cnt)
    expect_graph_replays(cnt, [steps], 100)
    ref = oracle_run(inst, steps)
    check_parity(inst, steps, got, ref)
    check_local(inst, steps, got, ref)


@pytest.mark.timeout(900)
def test_third_workload_sourced_prefix():
    # 16001 x 257, sourced: 2000 steps (2.9M), long enough for the field to
    # fill the source's neighbourhood; graph replays of 100 steps
    inst = W.kerr_sourced_16001x257()["instances"][0]
    steps = 2000
    say("Kerr 16001x257 sourced, steps", steps)
    cnt = {}
    got, = gpu_run([inst], steps, graph=100, counters=cnt)
    expect_graph_replays(cnt, [steps], 100)
    ref = oracle_run(inst, steps)
    assert np.linalg.norm(ref[0]) > 0
    check_parity(inst, steps, got, ref)
    check_local(inst, steps, got, ref)


@pytest.mark.timeout(900)
def test_six_mode_workload_prefix():
    # 16001 x 129, sourced, at the size and launch shape of the precision
    # study: 2000 steps (4M) in both precisions against the oracle
    inst = W.six_modes_16001x129()["instances"][0]
    steps = 2000
    say("six-mode 16001x129 sourced, steps", steps)
    got, = gpu_run([inst], steps, graph=100)
    ref = oracle_run(inst, steps)
    check_parity(inst, steps, got, ref)
    check_local(inst, steps, got, ref)
    c, = gpu_run([inst], steps, graph=100, precision=tk.TK_FP32_COMP)
    e = joint_rel(c[0], c[1], ref[0], ref[1])
    say("  FP32C joint rel L2 vs oracle", f"{e:.2e}")
    assert e < 1e-5
    # FP32C in the source window, where the increment is accumulated in FP64,
    # to 1e-4 of the window's values; at the poles, where the field is still
    # tiny after 4M, FP32 rounding is relative to the whole field, so there
    # to 1e-4 of the largest value anywhere
    loc = check_local(inst, steps, c, ref, bar=1e-4, global_scale=("poles",))
    say("  FP32C local", loc)


@pytest.mark.timeout(1200)
def test_batched_uneven_workload_vs_oracle():
    # the benchmark's path: 40 uneven instances, the AUTO kernel (two steps
    # per pass over whole strips), 200 steps in graph replays of 100 steps
    insts = W.batched_40_uneven()["instances"]
    steps = 200
    say("batched 40 instances, steps", steps, "points", W.points(insts))
    cnt = {}
    res = gpu_run(insts, steps, graph=100, counters=cnt)
    expect_graph_replays(cnt, [steps], 100)
    assert cnt["eager_launches"] == 0
    worst = 0.0
    for inst, got in zip(insts, res):
        ref = oracle_run(inst, steps)
        e = check_parity(inst, steps, got, ref)
        check_local(inst, steps, got, ref)
        worst = max(worst, e["joint"])
    say("worst joint rel L2", worst)


def test_batched_equals_alone_bitwise():
    insts = small_instances()
    steps = 40
    together = gpu_run(insts, steps)
    for k, inst in enumerate(insts):
        (phi, pi, wave), = gpu_run([inst], steps)
        assert np.array_equal(phi, together[k][0]) and np.array_equal(pi, together[k][1])
        assert np.array_equal(wave, together[k][2])


@pytest.mark.parametrize("rows", [3, 4, 7, 16])
def test_row_chunking_bitwise(rows):
    insts = small_instances()
    steps = 30
    base = gpu_run(insts, steps, rows=0)
    other = gpu_run(insts, steps, rows=rows)
    for (a, b) in zip(base, other):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
def test_launch_variants_bitwise(precision):
    # prefetch depth and store kind change scheduling only, never arithmetic
    insts = small_instances()
    base = gpu_run(insts, 40, prefetch=3, precision=precision)
    for pf, nt, rows in [(1, False, 0), (3, False, 0), (1, True, 0), (1, True, 5), (3, True, 7), (3, False, 64),
                         (1, False, 16)]:
        other = gpu_run(insts, 40, prefetch=pf, nt=nt, rows=rows, precision=precision)
        for (a, b) in zip(base, other):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
@pytest.mark.parametrize("rows,steps", [(4, 40), (5, 41), (7, 40), (16, 40)])
def test_two_step_chunks_bitwise(precision, rows, steps):
    # the two-step kernel on chunks of rows (level 1 recomputing a two-row
    # halo of u^{n+1}; an odd count ends with one one-step launch on the same
    # work list) against the whole-strip two-step kernel
    insts = small_instances()
    base = gpu_run(insts, steps, precision=precision)
    other = gpu_run(insts, steps, kernel=tk.TK_KERNEL_FUSED2, rows=rows, precision=precision)
    for (a, b) in zip(base, other):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
@pytest.mark.parametrize("rows,nt", [(4, True), (8, False), (8, True)])
def test_tiled_kernel_equals_marching_bitwise(precision, rows, nt):
    # tiles of 4 or 8 rows (the last chunk up to two more) staged in LDS
    # compute every point with the marching kernels' row functions
    insts = small_instances()
    base = gpu_run(insts, 40, precision=precision)
    other = gpu_run(insts, 40, kernel=tk.TK_KERNEL_TILED, rows=rows, nt=nt, precision=precision)
    for (a, b) in zip(base, other):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("kernel,G,rows", [(tk.TK_KERNEL_FUSED2, 20, 0), (tk.TK_KERNEL_FUSED2, 7, 0),
                                           (tk.TK_KERNEL_FUSED, 20, 0), (tk.TK_KERNEL_TILED, 20, 8),
                                           (tk.TK_KERNEL_FUSED2, 7, 5)])
def test_graph_replay_equals_eager_bitwise(kernel, G, rows):
    # an odd block size ends each replay with a one-step launch and flips the
    # state buffer an odd number of times per replay
    insts = small_instances()
    c_eager, c_graph = {}, {}
    eager = gpu_run(insts, 70, kernel=kernel, rows=rows, graph=0, counters=c_eager)
    chunks = [25, 20, 5, 20]
    graph = gpu_run(insts, 70, kernel=kernel, rows=rows, graph=G, chunks=chunks, counters=c_graph)
    expect_graph_replays(c_eager, [70], 0)
    expect_graph_replays(c_graph, chunks, G)  # the replays really ran
    for (a, b) in zip(eager, graph):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
@pytest.mark.parametrize("steps", [40, 41])
def test_two_step_kernel_equals_one_step_bitwise(precision, steps):
    # two time levels per pass change where u^{n+1} lives (registers instead
    # of HBM), never the arithmetic; waveform samples of the middle level
    # included (extract_every = 3)
    insts = small_instances()
    one = gpu_run(insts, steps, kernel=tk.TK_KERNEL_FUSED, precision=precision)
    for pf in (3, 1):
        two = gpu_run(insts, steps, kernel=tk.TK_KERNEL_FUSED2, prefetch=pf, precision=precision)
        for (a, b) in zip(one, two):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("n_r", [122, 123, 124, 183])
def test_two_step_interior_waves_bitwise(n_r):
    # the two-step kernel runs the waves whose 64 lanes all hold interior
    # columns without the Dirichlet mask: strips start every 60 columns, so
    # the strip at column 60 is such a wave from N_r = 123 on (its last lane
    # at N_r - 2) and not at 122 (its last lane on the Dirichlet column)
    rng = np.random.default_rng(n_r)
    inst = W.instance(a=0.7, m=2, n_r=n_r, n_theta=13, rstar_min=-20.0, rstar_max=25.0, rstar_obs=20.0,
                      extract_every=3, init=dict(center=2.0, width=3.0,
                                                 amps={2: complex(rng.standard_normal(), rng.standard_normal())}),
                      source=dict(r0=7.0, phase0=0.4, sigma_r_cells=2.0, sigma_th_cells=2.0, window_sigmas=6.0),
                      name=f"interior.{n_r}")
    say("interior waves, n_r", n_r)
    one = gpu_run([inst], 30, kernel=tk.TK_KERNEL_FUSED)
    for pf in (3, 1):
        two = gpu_run([inst], 30, kernel=tk.TK_KERNEL_FUSED2, prefetch=pf)
        assert all(np.array_equal(x, y) for x, y in zip(one[0], two[0]))
    check_parity(inst, 30, one[0], oracle_run(inst, 30))


def test_checkpoint_resume_bitwise():
    insts = small_instances()
    full = gpu_run(insts, 60)
    st = tk.Stepper(insts, force_dt=True)
    for k, inst in enumerate(insts):
        st.set_fields(k, *W.initial_data(inst))
    st.step(31)
    saved = [st.get_fields(k) for k in range(len(insts))]
    st.close()
    st2 = tk.Stepper(insts, force_dt=True)
    st2.set_step(31)
    for k in range(len(insts)):
        st2.set_fields(k, *saved[k])
    st2.step(29)
    for k in range(len(insts)):
        phi, pi = st2.get_fields(k)
        assert np.array_equal(phi, full[k][0]) and np.array_equal(pi, full[k][1])
    assert st2.step_index == 60
    st2.close()


@pytest.mark.parametrize("precision", [tk.TK_FP64, tk.TK_FP32_COMP])
def test_autotune_leaves_the_simulation_unchanged(precision):
    insts = small_instances()
    ref = gpu_run(insts, 40, precision=precision)
    st = tk.Stepper(insts, force_dt=True, precision=precision)
    for k, inst in enumerate(insts):
        st.set_fields(k, *W.initial_data(inst))
    st.step(20)
    ms, n = st.autotune(warmup=2, steps=4)
    t = st.get_tuning()
    say("autotune:", n, "shapes, best", f"{ms:.4f} ms/step", t)
    assert n >= 16 and ms > 0 and st.step_index == 20
    st.step(20)
    for k in range(len(insts)):
        phi, pi = st.get_fields(k)
        wave = st.extract(k)
        if t["kernel"] == tk.TK_KERNEL_TWO_PASS:  # another evaluation order
            assert rel(phi, ref[k][0]) < 1e-13 and rel(pi, ref[k][1]) < 1e-13
        else:  # every fused shape computes the same bits
            assert np.array_equal(phi, ref[k][0]) and np.array_equal(pi, ref[k][1])
            assert np.array_equal(wave, ref[k][2])
    st.close()


def test_two_pass_and_fused_agree():
    insts = small_instances()
    a = gpu_run(insts, 100, kernel=tk.TK_KERNEL_FUSED)
    b = gpu_run(insts, 100, kernel=tk.TK_KERNEL_TWO_PASS)
    for x, y in zip(a, b):
        assert rel(x[0], y[0]) < 1e-13 and rel(x[1], y[1]) < 1e-13


def test_extract_overrun_and_nonfinite():
    inst = W.instance(a=0.3, m=2, n_r=64, n_theta=9, rstar_min=-20.0, rstar_max=20.0,
                      rstar_obs=10.0, extract_every=1, init=dict(center=0.0, width=3.0, amps={2: 1.0}))
    st = tk.Stepper([inst], wave_capacity=8)
    st.set_fields(0, *W.initial_data(inst))
    st.step(9)
    with pytest.raises(tk.TkError) as ei:
        st.extract(0)
    assert ei.value.status == tk.TK_E_STATE
    st.set_step(st.step_index)  # restart sampling
    st.step(5)
    assert st.extract(0).shape == (5, 9)
    phi, pi = W.initial_data(inst)
    phi[4, inst["i_obs"]] = np.nan  # the sampled column itself
    st.set_fields(0, phi, pi)
    st.step(2)
    with pytest.raises(tk.TkError) as ei:
        st.extract(0)
    assert ei.value.status == tk.TK_E_NONFINITE
    st.close()
