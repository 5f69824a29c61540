"""Temporal segments (Section 4): the source's time origin, the plan/patch
helpers, the oracle's segments against its long run, and the GPU's batched
segments against the oracle's."""
import numpy as np
import pytest

import oracle
from paper_1206_0270_amd import segments as SEG
from paper_1206_0270_amd import workloads as W


def _grid(inst, kind="f64"):
    return oracle.Grid(M=inst["M"], a=inst["a"], s=inst["s"], m=inst["m"], n_r=inst["n_r"],
                       n_theta=inst["n_theta"], rstar_min=inst["rstar_min"], rstar_max=inst["rstar_max"],
                       dt=inst["dt"], i_obs=inst["i_obs"], extract_every=inst["extract_every"],
                       source=inst.get("source"), kind=kind)


def _inst(**kw):
    base = dict(a=0.7, m=2, n_r=121, n_theta=9, rstar_min=-20.0, rstar_max=40.0, rstar_obs=15.0,
                source=dict(r0=7.0, phase0=0.3))
    base.update(kw)
    return W.instance(**base)


def test_source_time_origin_continues_a_run():
    # 2N steps in one run, against N steps whose state seeds a run with the
    # source's time origin at N dt: the source phase continues, so the end
    # states agree to rounding (t = N dt + n' dt is formed as a sum there)
    inst = _inst()
    N = 120
    a = _grid(inst)
    a.set_state(*W.initial_data(inst))
    a.run(N)
    mid = a.get_state()
    a.run(N)
    src = dict(inst["source"], t0=N * inst["dt"])
    b = _grid(dict(inst, source=src))
    b.set_state(*mid)
    b.run(N)
    pa, qa = a.get_state()
    pb, qb = b.get_state()
    scale = np.max(np.abs(pa)) + np.max(np.abs(qa))
    assert np.max(np.abs(pa - pb)) + np.max(np.abs(qa - qb)) < 1e-12 * scale
    # and a wrong origin is visible
    c = _grid(dict(inst, source=dict(inst["source"], t0=(N + 7) * inst["dt"])))
    c.set_state(*mid)
    c.run(N)
    assert np.max(np.abs(c.get_state()[0] - pa)) > 1e-3 * np.max(np.abs(pa))


def _switch_on(g, t, T_on, rstar, theta):
    """The oracle's ramp factor at time t: F with the ramp over F without."""
    return g.source_value(t, rstar, theta) / g.unramped.source_value(t, rstar, theta)


def switch_on_check(kind="f64"):
    """F(t) = s(t / T_on) F_full(t), t the time since step 0 whatever the
    orbit's time origin t0: s vanishes for t <= 0 with every derivative
    (flat: below any power of t near 0), is 1 from T_on on, 1/2 at the
    midpoint, and s(x) + s(1 - x) = 1 (the step is built symmetric); between,
    it rises monotonically."""
    T_on = 40.0
    inst = _inst(source=dict(r0=7.0, phase0=0.3, t0=15.0, ramp=T_on))
    g = _grid(inst, kind)
    g.unramped = _grid(_inst(source=dict(r0=7.0, phase0=0.3, t0=15.0)), kind)
    rs, _ = g.radial()
    xp = oracle.tortoise(1.0, 0.7, 7.0 - (1 + np.sqrt(1 - 0.49)))
    r = rs[int(np.argmin(np.abs(rs - xp)))]
    th = np.pi / 2
    s = lambda x: _switch_on(g, x * T_on, T_on, r, th)
    assert g.source_value(-1.0, r, th) == 0 and g.source_value(0.0, r, th) == 0
    assert abs(s(1.0) - 1) < 1e-15 and abs(s(1.7) - 1) < 1e-15 and abs(s(0.5) - 0.5) < 1e-14
    for x in (0.05, 0.2, 0.37, 0.8):
        assert abs(s(x) + s(1 - x) - 1) < 1e-13
        assert abs(s(x).imag) < 1e-13
    xs = np.linspace(0.01, 0.99, 99)
    v = np.array([s(x).real for x in xs])
    assert np.all(np.diff(v) >= 0) and np.all(np.diff(v[10:-10]) > 0)  # it reaches 1.0 in double near x = 1
    for k in (2, 4, 8):  # flat at the start: s(x) / x^k -> 0
        assert s(0.02).real / 0.02 ** k < 1e-3


def test_source_switch_on_shape():
    switch_on_check()


def test_plan_and_patch_bookkeeping():
    inst = _inst()
    segs, info = SEG.plan(inst, t_total=30.0, n_seg=3, overlap=4.0)
    K, dt = inst["extract_every"], inst["dt"]
    assert info["steps"] == (info["samples_per_segment"] + info["overlap_samples"]) * K
    assert [s["source"]["t0"] for s in segs] == pytest.approx([k * info["L"] - info["overlap"] for k in range(3)])
    # patched sample i of segment k is the long run's sample k n_L + i
    waves = [np.arange(info["steps"] // K) + 1000 * k for k in range(3)]
    p = SEG.patch(waves, info)
    n_L, n_ov = info["samples_per_segment"], info["overlap_samples"]
    assert len(p) == 3 * n_L and p[0] == n_ov and p[n_L] == 1000 + n_ov
    with pytest.raises(ValueError):
        SEG.plan(dict(inst, source=None), 30.0, 3, 4.0)


def test_oracle_segments_reproduce_the_long_run_after_the_overlap():
    # A source-driven run settles to a quasi steady state once the switch-on
    # burst has passed the observer (here ~200M).  Segments whose overlap
    # covers that burst reproduce the long run inside their intervals; the
    # domain is long enough that no reflection from the outer boundary
    # returns within the run.
    inst = W.instance(a=0.7, m=2, n_r=2001, n_theta=9, rstar_min=-20.0, rstar_max=980.0, rstar_obs=40.0,
                      source=dict(r0=7.0, phase0=0.3))
    T, n = 900.0, 3
    g = _grid(inst)
    g.set_state(*W.initial_data(inst))
    n_total = int(round(T / (inst["extract_every"] * inst["dt"])))
    g.run(n_total * inst["extract_every"])
    long_w = g.waveform()[:, 4]  # equator row
    errs = {}
    for ov in (200.0, 400.0):
        segs, info = SEG.plan(inst, T, n, ov)
        waves = []
        for s in segs:
            gs = _grid(s)
            gs.set_state(*W.initial_data(s))
            gs.run(info["steps"])
            waves.append(gs.waveform()[:, 4])
        p = SEG.patch(waves, info)
        n_L = info["samples_per_segment"]
        # intervals after the long run's own burst: segments 1 .. n-1
        errs[ov] = max(np.max(np.abs(p[k * n_L:(k + 1) * n_L] - long_w[k * n_L:(k + 1) * n_L])) /
                       np.max(np.abs(long_w[k * n_L:(k + 1) * n_L])) for k in range(1, n))
    assert errs[400.0] < 1e-4 and errs[200.0] > 10 * errs[400.0], errs
    # a single segment with no overlap is the long run
    segs, info = SEG.plan(inst, T / n, 1, 0.0)
    gs = _grid(segs[0])
    gs.set_state(*W.initial_data(segs[0]))
    gs.run(info["steps"])
    n_L = info["samples_per_segment"]
    assert np.array_equal(gs.waveform()[:, 4][:n_L], long_w[:n_L])


@pytest.mark.gpu
def test_batched_gpu_segments_match_the_oracle_segments():
    import test_gpu_parity as GP
    from paper_1206_0270_amd import tk
    inst = _inst(source=dict(r0=7.0, phase0=0.3, ramp=4.0))  # each segment switches its source on smoothly
    segs, info = SEG.plan(inst, 30.0, 4, 6.0)
    res = GP.gpu_run(segs, info["steps"])  # one batched context, every segment one instance
    gp, op = [], []
    for s, got in zip(segs, res):
        ref = GP.oracle_run(s, info["steps"])
        GP.check_parity(s, info["steps"], got, ref)
        gp.append(got[2])
        op.append(ref[2])
    a, b = SEG.patch(gp, info), SEG.patch(op, info)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
