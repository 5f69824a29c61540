"""Benchmark: grid-point updates per second of the batched Teukolsky step.

One step advances every instance of the workload by one full two-step
Lax-Wendroff update (Eqs. (3)-(4), boundary conditions, source injection,
waveform sampling).  Inputs are seeded and synthetic and resident in HBM
before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|single]
                    [--precision fp64|fp32c] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/sec (batched modes) + % HBM roofline; FP32-comp vs FP64"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"fp64": 64, "fp32c": 48}
# Vector-ALU peaks of the MI355X (256 CUs at 2.4 GHz): FP64 78.6 TFLOP/s, FP32
# 157.3 TFLOP/s (the FP32 figure counts packed instructions; the kernels are
# built without them, so their FP32 issues at the FP64 rate).
ALU_PEAK_TFLOPS = {"fp64": 78.6, "fp32c": 157.3}
# Floating-point operations per point update (both stages of Eqs. (3)-(4))
# as the fused kernels' formulas are written, an FMA counting two: FP64, per
# stage, the radial difference and average (12), the coefficients at the
# point (33: Sigma-hat^2 (2), its inverse square root with two Newton steps
# (12), and the factored coefficients with the metric factor W left out of
# the Pi row (19)), the bracket with the angular neighbour sums (44: 4 sums,
# the Pi row's sum 22 times W once, the Phi row 4, the Pi row's b du 6) and
# the update (8): 97, 194 per update.  The compensated form, per stage, adds the
# Kahan terms to every difference (radial 12, angular column differences 20),
# keeps the average and the half step as two-sum pairs (32 + 32 in Eq. (3),
# 32 for the update of Eq. (4)) and drops a Newton step and the folded
# weights: 312 FP32 operations per update.
FLOPS_PER_UPDATE = {"fp64": 194, "fp32c": 312}
# The two-step kernels form Sigma-hat and 1/Sigma-hat once for both levels
# (level 2 takes level 1's value at the same point): per level-2 stage point
# the multiply-add of Sigma-hat^2 (2) and the inverse square root are not
# formed again.  FP64: 12 for the root (the estimate, x/2, two Newton steps
# of 5), 28 per level-2 update, 14 per update on average.  FP32C: 7 for the
# root (one Newton step), 18 per level-2 update, 9 per update.
FLOPS_SHARED_TWO_STEP = {"fp64": 14, "fp32c": 9}


def flops_per_update(precision, two_step):
    """FP64 / FP32 operations per point update the launch's formulas need."""
    return FLOPS_PER_UPDATE[precision] - (FLOPS_SHARED_TWO_STEP[precision] if two_step else 0)


KERNEL_POLICY = {"fp64": "PolicyF64", "fp32c": "PolicyF32C"}
KERNEL_SOURCES = ["paper_1206_0270_amd/csrc/tk_kernels.hip", "paper_1206_0270_amd/csrc/tk_device.h",
                  "paper_1206_0270_amd/csrc/tk_internal.h"]


def _code_only(text):
    """C/C++ source without its comments and blank lines: what the compiler
    sees of it, so that a comment edit leaves the hash (and the counters
    recorded under it) valid.  No string literal in the kernel sources holds a
    comment marker."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.split("\n") if l.strip())


def kernel_hash():
    """Hash of the kernel sources' code (comments left out)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def workload(name):
    from paper_1206_0270_amd import workloads as W
    if name == "batched":
        insts = W.batched_40_uneven()["instances"]
        desc = ("batched uneven: 40 instances, m=1..8 x a in {0,0.3,0.6,0.9,0.99}, "
                "N_r 4001-16001, N_theta 33-257, r* in [-300,300]M, half Gaussian data, "
                "half circular-orbit sources")
    elif name == "single":
        insts = W.kerr_8001x129()["instances"]
        desc = "single instance: Kerr a=0.9, s=-2, m=2, 8001 x 129 on [-300,300]M, Gaussian data"
    elif name == "precision":
        insts = W.six_modes_16001x129()["instances"]
        desc = ("precision-study workload: 6 instances m=2,3,4 x a=0.5,0.9, circular orbits r0=8M, "
                "16001 x 129 on [-300,300]M")
    else:
        raise SystemExit(f"unknown workload {name}")
    return insts, desc


def kernel_name(prec, prefetch, nt, waves, two_step=False, chunked=False):
    """The fused kernel variant as rocprofv3 names it (template arguments:
    prefetch depth, non-temporal stores, occupancy target).  The compensated
    form runs its two-step march on whole strips with the chunked kernel."""
    k = ("k_fused2c" if chunked or prec == "fp32c" else "k_fused2") if two_step else "k_fused"
    return f"{k}<{KERNEL_POLICY[prec]}<{prefetch}, {'true' if nt else 'false'}, {waves or 1}>>"


def traffic_entry(name, wl):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(f"{name}:{wl}")
        if not ent or ent.get("kernel_hash") != kernel_hash():
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def valu_entry(name, wl, updates_per_s):
    """Vector-ALU issue figures of the kernel from the committed rocprofv3
    SQ counter summary, if taken on the current kernel source: VALU busy
    fraction, wave64 VALU instructions per point update, resident waves per
    SIMD, executed floating-point operations per update, and the update rate
    at which every SIMD would issue one VALU instruction every cycle at the
    2.4 GHz peak clock (the issue peak; 1024 SIMDs, 16 lanes each, so a wave64
    instruction takes 4 cycles)."""
    path = os.path.join(ROOT, "profiles", "issue.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(f"{name}:{wl}")
        if not ent or ent.get("kernel_hash") != kernel_hash():
            return None
        peak = 1024 * 2.4e9 * 64 / (4 * ent["lane_instr_per_update"])
        return {"valu_busy": ent["valu_busy"], "lane_instr_per_update": ent["lane_instr_per_update"],
                "waves_per_simd": ent["waves_per_simd"], "flops_per_update_executed": ent["flops_per_update_executed"],
                "issue_peak_updates_per_s": peak, "frac_of_issue_peak": updates_per_s / peak,
                "source": ent.get("source")}
    except Exception:
        return None


def cpu_baseline(insts, target_s=15.0, steps=70):
    """The oracle as it stands, timed on this host on a bounded sample of the
    same workload: instances in workload order, `steps` steps each, until
    about target_s seconds of stepping (grid setup excluded)."""
    import oracle
    from paper_1206_0270_amd import workloads as W

    threads = oracle.get_threads()
    done_upd, spent, used = 0, 0.0, 0
    for inst in insts:
        g = oracle.Grid(M=inst["M"], a=inst["a"], s=inst["s"], m=inst["m"], n_r=inst["n_r"],
                        n_theta=inst["n_theta"], rstar_min=inst["rstar_min"],
                        rstar_max=inst["rstar_max"], dt=inst["dt"], i_obs=inst["i_obs"],
                        extract_every=inst["extract_every"], source=inst.get("source"))
        g.set_state(*W.initial_data(inst))
        t0 = time.perf_counter()
        g.run(steps)
        spent += time.perf_counter() - t0
        done_upd += inst["n_r"] * inst["n_theta"] * steps
        used += 1
        del g
        if spent >= target_s:
            break
    return dict(value=done_upd / spent, unit="grid-point updates/s", cores=threads, kind="oracle",
                sample=f"first {used} of {len(insts)} instances of the same workload, {steps} steps each "
                       f"({done_upd:.3g} updates in {spent:.1f} s, grid setup excluded); FP64 C oracle "
                       f"with OpenMP over theta rows")


def projected_waveform(inst, wave):
    """Waveform samples [k][theta] projected onto the s=-2 spin-weighted
    harmonic with l = max(|m|, 2)."""
    from paper_1206_0270_amd import workloads as W
    import numpy as np
    nt = inst["n_theta"]
    th = np.arange(nt) * np.pi / (nt - 1)
    Y = W.swsh_profile(-2, inst["m"], max(abs(inst["m"]), 2), th)
    return wave @ (Y * 2 * np.pi * np.sin(th) * (np.pi / (nt - 1)))


def waveform_errors(w_ref, w, floor=1e-3):
    """Amplitude error max ||w| - |w_ref|| / |w_ref| and phase error
    max |arg(w / w_ref)| over samples with |w_ref| >= floor * max |w_ref|."""
    import numpy as np
    sel = np.abs(w_ref) >= floor * np.abs(w_ref).max()
    if not sel.any():
        return None, None
    amp = float(np.max(np.abs(np.abs(w[sel]) - np.abs(w_ref[sel])) / np.abs(w_ref[sel])))
    ph = float(np.max(np.abs(np.angle(w[sel] / w_ref[sel]))))
    return amp, ph


def precision_study(args):
    """The six-mode workload (m = 2, 3, 4 x a = 0.5, 0.9; circular orbits at
    r0 = 8M; 16001 x 129 on [-300, 300]M; dt = 1/500) in FP64 and in the
    FP32-compensated form on the GPU over a window of window_M, and on a short
    prefix against the FP64 oracle.  One JSON line."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    insts = W.six_modes_16001x129()["instances"]
    if args.study_ramp > 0:  # every source switched on smoothly over study_ramp
        insts = [dict(i, source=dict(i["source"], ramp=args.study_ramp)) for i in insts]
    if args.study_layer > 0:  # grids ending in a layer on [study_layer, 300]M, waveform read at null infinity
        insts = [dict(i, layer_start=args.study_layer, rstar_obs=i["rstar_max"], i_obs=i["n_r"] - 1) for i in insts]
    dt = insts[0]["dt"]
    steps = int(round(args.study_window / dt))
    steps -= steps % 200
    points = W.points(insts)
    forms = {}
    for name, prec in (("fp64", tk.TK_FP64), ("fp32c", tk.TK_FP32_COMP)):
        st = tk.Stepper(insts, precision=prec, wave_capacity=int(args.study_window) + 64)
        for k, inst in enumerate(insts):
            st.set_fields(k, *W.initial_data(inst))
        st.autotune(warmup=2, steps=6)
        t = st.get_tuning()
        t["graph_steps"] = 100
        st.set_tuning(**t)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st.stream)
        chunk = 100000
        for done in range(0, steps, chunk):
            st.step(min(chunk, steps - done))
            if steps > chunk:
                st.synchronize()
                print(f"# {name}: {min(done + chunk, steps)} of {steps} steps", file=sys.stderr, flush=True)
        ev1.record(st.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        waves = [projected_waveform(inst, st.extract(k, max_samples=int(args.study_window) + 64))
                 for k, inst in enumerate(insts)]
        st.close()
        forms[name] = dict(updates_per_s=points * steps / (ms / 1e3), seconds=ms / 1e3, tuning=t, waves=waves)
        print(f"# {name}: {steps} steps in {ms / 1e3:.1f} s", file=sys.stderr, flush=True)
    K = insts[0]["extract_every"]
    per_inst = []
    worst = {}
    for k, inst in enumerate(insts):
        wa, wb = forms["fp64"]["waves"][k], forms["fp32c"]["waves"][k]
        row = {"name": inst["name"]}
        for T in args.study_checkpoints:
            n = min(len(wa), int(round(T / (K * dt))))
            amp, ph = waveform_errors(wa[:n], wb[:n])
            row[f"T{int(T)}"] = {"amp": amp, "phase": ph}
            if amp is not None:
                w = worst.setdefault(int(T), [0.0, 0.0])
                w[0], w[1] = max(w[0], amp), max(w[1], ph)
        per_inst.append(row)
    # short prefix against the oracle, first instance, both forms
    import oracle
    inst = insts[0]
    g = oracle.Grid(M=inst["M"], a=inst["a"], s=inst["s"], m=inst["m"], n_r=inst["n_r"], n_theta=inst["n_theta"],
                    rstar_min=inst["rstar_min"], rstar_max=inst["rstar_max"], dt=inst["dt"], i_obs=inst["i_obs"],
                    extract_every=inst["extract_every"], source=inst.get("source"),
                    layer_R=inst.get("layer_start", 0.0))
    g.set_state(*W.initial_data(inst))
    g.run(args.study_oracle_steps)
    ophi, opi = g.get_state()
    den = np.sqrt(np.linalg.norm(ophi) ** 2 + np.linalg.norm(opi) ** 2)
    pref = {}
    for name, prec in (("fp64", tk.TK_FP64), ("fp32c", tk.TK_FP32_COMP)):
        st = tk.Stepper([inst], precision=prec)
        st.set_fields(0, *W.initial_data(inst))
        st.step(args.study_oracle_steps)
        phi, pi = st.get_fields(0)
        st.close()
        pref[name] = float(np.sqrt(np.linalg.norm(phi - ophi) ** 2 + np.linalg.norm(pi - opi) ** 2) / den)
    out = {
        "metric": "waveform amplitude / phase relative error of the FP32-compensated form vs FP64; updates/s of both",
        "workload": "6 instances m=2,3,4 x a=0.5,0.9, circular orbit r0=8M, 16001 x 129 on [-300,300]M, dt=1/500, "
                    + (f"ending in a hyperboloidal layer on [{args.study_layer},300]M, waveform at null infinity"
                       if args.study_layer > 0 else "waveform at r*=290M")
                    + " projected on the l=max(|m|,2) harmonic"
                    + (f"; sources switched on over {args.study_ramp}M" if args.study_ramp > 0 else ""),
        "layer_start": args.study_layer,
        "ramp_M": args.study_ramp,
        "window_M": steps * dt, "steps": steps, "points": points,
        "fp64_updates_per_s": forms["fp64"]["updates_per_s"], "fp32c_updates_per_s": forms["fp32c"]["updates_per_s"],
        "fp32c_speedup": forms["fp32c"]["updates_per_s"] / forms["fp64"]["updates_per_s"],
        "tuning": {k: forms[k]["tuning"] for k in forms},
        "worst_by_window": {f"T{T}": {"amp": v[0], "phase": v[1]} for T, v in worst.items()},
        "per_instance": per_inst,
        "oracle_prefix": {"instance": inst["name"], "steps": args.study_oracle_steps,
                          "joint_rel_l2_vs_oracle": pref},
    }
    print(json.dumps(out), flush=True)


def noise_study(args):
    """How the scheme carries rounding-sized noise on the six-mode workload's
    grid: FP64, no source, (Phi, Pi) set to white noise of 1e-20 per value,
    stepped for noise_window M; the field norm and the position of its
    largest value every 50M, at the workload's r* spacing and time step and
    with each halved or doubled.  One JSON line.  A growth that changes with
    h or dt would be a property of the discretisation; one that does not is
    the equation's own."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    cases = [("h=0.0375 dt=1/500 (six-mode workload)", 16001, 1 / 500), ("h=0.075 dt=1/500", 8001, 1 / 500),
             ("h=0.0375 dt=1/1000", 16001, 1 / 1000), ("h=0.01875 dt=1/500", 32001, 1 / 500)]
    out = {}
    for name, n_r, dt in cases:
        inst = W.instance(a=0.9, m=2, n_r=n_r, n_theta=129, rstar_min=-300.0, rstar_max=300.0, dt=dt,
                          extract_every=0)
        rng = np.random.default_rng(3)
        shp = (inst["n_theta"], n_r)

        def noise():
            x = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 1e-20
            x[:, 0] = 0
            x[:, -1] = 0
            return x

        st = tk.Stepper([inst], precision=tk.TK_FP64, force_dt=True)
        phi0, pi0 = noise(), noise()
        st.set_fields(0, phi0, pi0)
        norm0 = float(np.sqrt(np.linalg.norm(phi0) ** 2 + np.linalg.norm(pi0) ** 2))
        chunk = int(round(50.0 / dt))
        rows = []
        for k in range(int(args.noise_window / 50)):
            st.step(chunk)
            phi, pi = st.get_fields(0)
            a = np.abs(phi)
            j, i = np.unravel_index(np.argmax(a), a.shape)
            norm = float(np.sqrt(np.sum(a ** 2) + np.sum(np.abs(pi) ** 2)))
            rows.append({"t": 50.0 * (k + 1), "norm_over_initial": norm / norm0,
                         "argmax_rstar": inst["rstar_min"] + i * (inst["rstar_max"] - inst["rstar_min"]) / (n_r - 1),
                         "argmax_row": int(j)})
            print(f"# {name}: t={rows[-1]['t']:.0f}M norm x{rows[-1]['norm_over_initial']:.3g} "
                  f"max at r*={rows[-1]['argmax_rstar']:.1f}M row {j}", file=sys.stderr, flush=True)
        st.close()
        out[name] = rows
    print(json.dumps({"metric": "growth of white noise (1e-20 per value) under the FP64 scheme, no source",
                      "instance": "a=0.9, s=-2, m=2, 129 theta rows, r* in [-300,300]M, Dirichlet ends",
                      "cases": out}), flush=True)


def sensitivity_study(args):
    """One mode of the six-mode workload (index sens_instance) with the source
    switched on abruptly and over 200M: the FP64 run; an FP64 run whose state
    at sens_at M is perturbed value by value by a relative N(0, 2^-24) (one
    FP32 rounding of every value); and the FP32-compensated run.  Waveform
    (projected on l = max(|m|, 2) at the observer) relative differences to the
    FP64 run at checkpoints.  One JSON line."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    res = {}
    for ramp in (0.0, 200.0):
        inst = W.six_modes_16001x129()["instances"][args.sens_instance]
        if ramp:
            inst = dict(inst, source=dict(inst["source"], ramp=ramp))
        dt = inst["dt"]
        n1 = int(round(args.sens_at / dt))
        n2 = int(round(args.sens_window / dt))
        cap = int(args.sens_window) + 64

        def stepper(prec):
            st = tk.Stepper([inst], precision=prec, wave_capacity=cap)
            st.set_tuning(kernel=tk.TK_KERNEL_AUTO, rows_per_tile=0, graph_steps=100)
            return st

        a = stepper(tk.TK_FP64)
        a.set_fields(0, *W.initial_data(inst))
        a.step(n1)
        wa1 = a.extract(0, cap)
        phi, pi = a.get_fields(0)
        rng = np.random.default_rng(1)

        def perturb(x):
            e = 2.0 ** -24
            return x.real * (1 + e * rng.standard_normal(x.shape)) + 1j * x.imag * (1 + e * rng.standard_normal(x.shape))

        b = stepper(tk.TK_FP64)
        b.set_fields(0, perturb(phi), perturb(pi))
        b.set_step(n1)
        a.step(n2 - n1)
        b.step(n2 - n1)
        w64 = projected_waveform(inst, np.concatenate([wa1, a.extract(0, cap)]))
        w64p = projected_waveform(inst, b.extract(0, cap))
        a.close()
        b.close()
        c = stepper(tk.TK_FP32_COMP)
        c.set_fields(0, *W.initial_data(inst))
        for k in range(0, n2, 100000):
            c.step(min(100000, n2 - k))
            c.synchronize()
            print(f"# ramp {ramp}: fp32c {min(k + 100000, n2)} of {n2} steps", file=sys.stderr, flush=True)
        w32 = projected_waveform(inst, c.extract(0, cap))
        c.close()
        K = inst["extract_every"]
        rows = []
        for T in args.sens_checkpoints:
            i = int(round(T / (K * dt))) - 1
            j = i - (len(w64) - len(w64p))
            rows.append({"t": T, "abs_w64": float(abs(w64[i])),
                         "fp32c": float(abs(w32[i] - w64[i]) / abs(w64[i])),
                         "fp64_perturbed": float(abs(w64p[j] - w64[i]) / abs(w64[i])) if j >= 0 else None})
        res[f"ramp {ramp:g}M"] = rows
    print(json.dumps({"metric": "relative waveform difference to the FP64 run at the observer: FP32C, and FP64 "
                                f"with every value of the state perturbed by one FP32 rounding at {args.sens_at:g}M",
                      "instance": W.six_modes_16001x129()["instances"][args.sens_instance]["name"], "cases": res}), flush=True)


def richardson_study(args):
    """Section 2.3 item 3 / Section 5.1 footnote on the GPU: one sourced Kerr
    mode at three resolutions (grid spacings and time step halved), the
    projected waveforms extrapolated by the library, and the error estimate
    from the two extrapolants over the window in which only outgoing
    radiation reaches the observer.  One JSON line."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    n_r = int(round(300.0 / args.rich_h)) + 1
    base = W.instance(a=0.9, m=2, n_r=n_r, n_theta=args.rich_nth, rstar_min=-60.0, rstar_max=240.0,
                      rstar_obs=180.0, name="kerr a=0.9 m=2 sourced",
                      source=dict(r0=10.0, phase0=0.7, sigma_r_cells=args.rich_sigma_r / args.rich_h,
                                  sigma_th_cells=args.rich_sigma_th))
    fam = W.richardson_family(base)
    T = args.rich_window
    waves, runs = [], []
    total_upd, total_s = 0, 0.0
    for inst in fam:
        steps = int(round(T / inst["dt"]))
        steps -= steps % 2
        st = tk.Stepper([inst], wave_capacity=int(T) + 64)
        st.set_fields(0, *W.initial_data(inst))
        st.autotune(warmup=2, steps=6)
        t = st.get_tuning()
        t["graph_steps"] = 100
        st.set_tuning(**t)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st.stream)
        st.step(steps)
        ev1.record(st.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        waves.append(projected_waveform(inst, st.extract(0, max_samples=int(T) + 64)))
        st.close()
        upd = inst["n_r"] * inst["n_theta"] * steps
        total_upd += upd
        total_s += ms / 1e3
        runs.append(dict(n_r=inst["n_r"], n_theta=inst["n_theta"], dt=inst["dt"], steps=steps,
                         updates_per_s=upd / (ms / 1e3), kernel=t["kernel"], rows_per_tile=t["rows_per_tile"]))
    n = min(len(w) for w in waves)
    ext, est = tk.richardson(*[w[:n] for w in waves])
    dt_s = fam[0]["extract_every"] * fam[0]["dt"]
    times = (np.arange(n) + 1) * dt_s
    # outgoing-only window at the observer: from the arrival of the direct
    # signal to the return of its reflection from the outer boundary
    r_obs, r_b, r_src = base["rstar_obs"], base["rstar_max"], 10.0
    t0, t1 = r_obs - r_src, 2 * r_b - r_obs - r_src
    win = (times >= t0) & (times <= t1) & (np.abs(ext) >= 1e-3 * np.abs(ext).max())
    r12 = (4 * waves[1][:n] - waves[0][:n]) / 3  # the coarse pair's extrapolant
    out = {
        "metric": "Richardson-extrapolated waveform: error estimate from two extrapolants (Section 5.1)",
        "workload": f"Kerr a=0.9, s=-2, m=2, circular orbit r0=10M (source widths {args.rich_sigma_r} M in r*, "
                    f"{args.rich_sigma_th} coarse theta cells); "
                    f"r* in [-60,240]M, observer 180M; coarse h = {args.rich_h} M, {args.rich_nth} theta rows; "
                    f"three levels halving h, dtheta and dt",
        "window_M": [t0, t1],
        "levels": runs,
        "gpu_updates_per_s_all_levels": total_upd / total_s,
        "estimate_max_in_window": float(np.max(est[win])),
        "estimate_median_in_window": float(np.median(est[win])),
        "amplitude_estimate_max": float(np.max(np.abs(np.abs(ext[win]) - np.abs(r12[win])) / np.abs(ext[win]))),
        "phase_estimate_max": float(np.max(np.abs(np.angle(ext[win] / r12[win])))),
        "finest_vs_extrapolated_max": float(np.max(np.abs(waves[2][:n][win] - ext[win]) / np.abs(ext[win]))),
        # self-convergence factor |w1 - w2| / |w2 - w3|: 4 for a second-order result
        "convergence_factor_median": float(np.median(np.abs(waves[0][:n][win] - waves[1][:n][win]) /
                                                     np.abs(waves[1][:n][win] - waves[2][:n][win]))),
        "samples_in_window": int(win.sum()),
    }
    print(json.dumps(out), flush=True)


def state_bytes_per_update(kernel, precision="fp64"):
    """State traffic per update of a layered context's step: one read and one
    write (64 B FP64, 48 B for the compensated storage) for a one-step pass,
    half that for the two-step pass; the two-pass layer kernels (FP64) also
    write and read the half-step array and read u^n twice (160 B)."""
    from paper_1206_0270_amd import tk
    if precision == "fp32c":  # one read and one write of f (16 B) and c (8 B)
        return 24.0 if kernel == tk.TK_KERNEL_FUSED2 else 48.0
    return {tk.TK_KERNEL_TWO_PASS: 160.0, tk.TK_KERNEL_FUSED2: 32.0}.get(kernel, 64.0)


def layer_throughput(args):
    """Step rate of a layered batch that fills the GPU, with the kernel the
    autotuner picks: the six modes (m = 2, 3, 4 x a = 0.5,
    0.9; 16001 x 129 on [-300, 300]M), each ending in a layer on [250, 300]M,
    sourced; in the precision --precision names."""
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    thr = [W.instance(a=a, m=m, n_r=16001, n_theta=129, rstar_min=-300.0, rstar_max=300.0, layer_start=250.0,
                      extract_every=500, source=dict(r0=8.0, phase0=0.3 * m, ramp=200.0), name=f"m{m} a{a}")
           for m in (2, 3, 4) for a in (0.5, 0.9)]
    dt_t = min(i["dt"] for i in thr)
    for i in thr:
        i["dt"] = dt_t
    st = tk.Stepper(thr, precision=tk.TK_FP32_COMP if args.precision == "fp32c" else tk.TK_FP64)
    for k, i in enumerate(thr):
        st.set_fields(k, *W.initial_data(i))
    st.autotune(warmup=2, steps=10)
    tuning = st.get_tuning()
    tuning["graph_steps"] = 100
    st.set_tuning(**tuning)
    st.prepare(args.layer_steps)  # work list and graph capture, outside the timed region
    st.step(args.layer_warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(st.stream)
    st.step(args.layer_steps)
    ev1.record(st.stream)
    torch.cuda.synchronize()
    ms_t = ev0.elapsed_time(ev1)
    st.close()
    pts_t = sum(i["n_r"] * i["n_theta"] for i in thr)
    ups_t = pts_t * args.layer_steps / (ms_t / 1e3)
    print(f"# throughput: {pts_t} points, {args.layer_steps} steps in {ms_t / 1e3:.2f} s", file=sys.stderr,
          flush=True)
    lay_bytes = state_bytes_per_update(tuning["kernel"], args.precision)
    return {"workload": "6 x 16001 x 129 on [-300,300]M, layers on [250,300]M, sourced", "precision": args.precision,
            "points": pts_t,
            "steps": args.layer_steps, "ms_per_step": ms_t / args.layer_steps, "updates_per_s": ups_t,
            "tuning": tuning, "bytes_per_update": lay_bytes, "achieved_GBps": ups_t * lay_bytes / 1e9,
            "frac_of_8TBps": ups_t * lay_bytes / 8e12}


def layer_study(args):
    """Section 2.3 item 2 on the GPU: a Kerr mode (a = 0.9, m = 2) driven by a
    circular orbit at r0 = 10M (switched on over 100M) on three domains with
    the same h, dtheta and dt: [-300, 100]M ending in a hyperboloidal layer on
    [R, 100]M whose last node is null infinity; the same domain closed by the
    Dirichlet wall; and [-300, 700]M, long enough that nothing returns from
    its wall within the window.  The projected waveform at r* = 50M of the two
    short domains against the long one's, over the window after the direct
    signal arrives; the waveform at null infinity beside it; and the step
    rates of the contexts, with the kernels the autotuner picks.  One JSON
    line."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    h, nth, T, R = args.layer_h, args.layer_nth, args.layer_window, args.layer_start
    src = dict(r0=10.0, phase0=0.7, ramp=100.0)

    def mk(rmax, layer, obs, name):
        return W.instance(a=0.9, m=2, n_r=int(round((rmax + 300.0) / h)) + 1, n_theta=nth, rstar_min=-300.0,
                          rstar_max=rmax, rstar_obs=obs, layer_start=layer, source=src, name=name)

    def mk2(rmax, layer, obs, name):
        i = mk(rmax, layer, obs, name)
        return W.instance(a=0.9, m=2, n_r=2 * (i["n_r"] - 1) + 1, n_theta=nth, rstar_min=-300.0, rstar_max=rmax,
                          rstar_obs=obs, layer_start=layer, source=src, name=name + " h/2")

    cases = {"layer": [mk(100.0, R, 50.0, "layer r*=50"), mk(100.0, R, 100.0, "layer scri")],
             "wall": [mk(100.0, 0.0, 50.0, "wall r*=50")],
             "long": [mk(700.0, 0.0, 50.0, "long r*=50")],
             "layer_h2": [mk2(100.0, R, 50.0, "layer r*=50")],
             "long_h2": [mk2(700.0, 0.0, 50.0, "long r*=50")]}
    dt = min(i["dt"] for c in cases.values() for i in c)
    out = {}
    for key, insts in cases.items():
        for i in insts:
            i["dt"] = dt
            i["extract_every"] = max(1, int(round(1.0 / dt)))
        steps = int(round(T / dt))
        steps -= steps % 2
        cap = int(T) + 64
        st = tk.Stepper(insts, wave_capacity=cap)
        st.autotune(warmup=2, steps=6)
        t = st.get_tuning()
        t["graph_steps"] = 100
        st.set_tuning(**t)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st.stream)
        st.step(steps)
        ev1.record(st.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        pts = sum(i["n_r"] * i["n_theta"] for i in insts)
        out[key] = dict(waves=[projected_waveform(i, st.extract(k, max_samples=cap)) for k, i in enumerate(insts)],
                        updates_per_s=pts * steps / (ms / 1e3), ms_per_step=ms / steps, points=pts, steps=steps,
                        kernel=t["kernel"])
        st.close()
        print(f"# {key}: {pts} points, {steps} steps in {ms / 1e3:.2f} s", file=sys.stderr, flush=True)
    n = min(len(out[k]["waves"][0]) for k in out)
    times = (np.arange(n) + 1) * cases["long"][0]["extract_every"] * dt
    w_long = out["long"]["waves"][0][:n]
    win = times >= args.layer_from
    scale = np.abs(w_long[win]).max()
    diff = {k: float(np.abs(out[k]["waves"][0][:n][win] - w_long[win]).max() / scale) for k in ("layer", "wall")}
    w_long2 = out["long_h2"]["waves"][0][:n]
    diff["layer_h2"] = float(np.abs(out["layer_h2"]["waves"][0][:n][win] - w_long2[win]).max()
                             / np.abs(w_long2[win]).max())

    thr = layer_throughput(args)
    w_scri = out["layer"]["waves"][1][:n]
    tail = times >= T - 100.0
    lay_bytes = state_bytes_per_update(out["layer"]["kernel"])
    ups = out["layer"]["updates_per_s"]
    res = {
        "metric": "hyperboloidal layer: waveform at r*=50M against a domain 7x longer; step rate of its kernels",
        "workload": f"a=0.9 m=2, circular orbit r0=10M switched on over 100M; h={h}M, {nth} theta rows, dt={dt:.6g}; "
                    f"layer [-300,100]M with R={R}M vs wall [-300,100]M vs long [-300,700]M; window {T}M",
        "max_rel_diff_vs_long": {"layer": diff["layer"], "layer_h/2": diff["layer_h2"], "wall": diff["wall"],
                                 "from_t": args.layer_from},
        "scri_over_r50_amplitude_last_100M": float(np.abs(w_scri[tail]).mean() / np.abs(w_long[tail]).mean()),
        "updates_per_s": {k: out[k]["updates_per_s"] for k in out},
        "layer_kernels_study_grid": {"ms_per_step": out["layer"]["ms_per_step"], "points": out["layer"]["points"],
                                     "bytes_per_update": lay_bytes, "achieved_GBps": ups * lay_bytes / 1e9,
                                     "frac_of_8TBps": ups * lay_bytes / 8e12},
        "layer_kernels_throughput": thr,
        "kernels": {k: out[k]["kernel"] for k in out},
    }
    print(json.dumps(res), flush=True)


def source_study(args):
    """Section 2.3 item 1 on the GPU: one Kerr mode driven by the same
    circular orbit with three representations of the point particle (the
    two-cell Gaussian, the step delta and the linear delta), each at three
    resolutions halving h, dtheta and dt (the Gaussian keeps its width in
    cells, so all three tend to the point particle).  Per form and level the
    projected waveform's distance, over the outgoing-only window, to the
    Richardson extrapolant of the linear delta; the observed convergence
    factor; and how far each form's own extrapolant lies from that limit.
    The three forms of a level advance together in one batch.  One JSON line."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    n_r = int(round(300.0 / args.src_h)) + 1
    shapes = ("gaussian", "step_delta", "linear_delta")
    fams = []
    for shape in shapes:
        base = W.instance(a=0.9, m=2, n_r=n_r, n_theta=args.src_nth, rstar_min=-60.0, rstar_max=240.0,
                          rstar_obs=180.0, name=f"kerr a=0.9 m=2 {shape}",
                          source=dict(r0=10.0, phase0=0.7, shape=shape))
        fams.append(W.richardson_family(base, 3, point_limit=True))
    T = args.src_window
    waves = {sh: [] for sh in shapes}
    runs = []
    for lev in range(3):
        insts = [f[lev] for f in fams]
        steps = int(round(T / insts[0]["dt"]))
        steps -= steps % 2
        st = tk.Stepper(insts, wave_capacity=int(T) + 64)
        for k, inst in enumerate(insts):
            st.set_fields(k, *W.initial_data(inst))
        st.autotune(warmup=2, steps=6)
        t = st.get_tuning()
        t["graph_steps"] = 100
        st.set_tuning(**t)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st.stream)
        st.step(steps)
        ev1.record(st.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        for k, sh in enumerate(shapes):
            waves[sh].append(projected_waveform(insts[k], st.extract(k, max_samples=int(T) + 64)))
        st.close()
        upd = 3 * insts[0]["n_r"] * insts[0]["n_theta"] * steps
        runs.append(dict(n_r=insts[0]["n_r"], n_theta=insts[0]["n_theta"], dt=insts[0]["dt"], steps=steps,
                         updates_per_s=upd / (ms / 1e3), kernel=t["kernel"]))
        print(f"# level {lev}: {insts[0]['n_r']} x {insts[0]['n_theta']}, {steps} steps x 3 forms in "
              f"{ms / 1e3:.1f} s", file=sys.stderr, flush=True)
    n = min(len(w) for ws in waves.values() for w in ws)
    ext = {sh: tk.richardson(*[w[:n] for w in waves[sh]])[0] for sh in shapes}
    ref = ext["linear_delta"]
    dt_s = fams[0][0]["extract_every"] * fams[0][0]["dt"]
    times = (np.arange(n) + 1) * dt_s
    t0, t1 = 180.0 - 10.0, 2 * 240.0 - 180.0 - 10.0  # direct signal .. its outer-boundary reflection
    win = (times >= t0) & (times <= t1) & (np.abs(ref) >= 1e-3 * np.abs(ref).max())
    nrm = lambda x: float(np.linalg.norm(x[:n][win]))
    forms = {}
    for sh in shapes:
        w = waves[sh]
        forms[sh] = {
            "rel_l2_vs_limit_by_level": [nrm(wl[:n] - ref) / nrm(ref) for wl in w],
            "convergence_factor": nrm(w[0][:n] - w[1][:n]) / nrm(w[1][:n] - w[2][:n]),
            "own_extrapolant_vs_limit": nrm(ext[sh] - ref) / nrm(ref),
        }
    out = {
        "metric": "point-particle representations (Section 2.3 item 1): waveform error vs the point-particle "
                  "limit at three resolutions",
        "workload": f"Kerr a=0.9, s=-2, m=2, circular orbit r0=10M; r* in [-60,240]M, observer 180M; coarse h = "
                    f"{args.src_h} M, {args.src_nth} theta rows; three levels halving h, dtheta and dt; "
                    f"limit = Richardson extrapolant of the linear delta",
        "window_M": [t0, t1], "samples_in_window": int(win.sum()),
        "levels": runs,
        "forms": forms,
        "gaussian_over_linear_error_by_level": [forms["gaussian"]["rel_l2_vs_limit_by_level"][k] /
                                                forms["linear_delta"]["rel_l2_vs_limit_by_level"][k]
                                                for k in range(3)],
    }
    print(json.dumps(out), flush=True)


def segments_study(args):
    """Section 4's temporal decomposition on one GPU: one sourced mode run
    for T in one context, against the same T split into segments that start
    `overlap` earlier, advance together as one batch and are patched.  Time
    to solution of both and the patched waveform against the long run after
    the switch-on burst.  One JSON line."""
    import numpy as np
    import torch
    from paper_1206_0270_amd import segments as SEG
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    inst = W.instance(a=0.9, m=2, n_r=8001, n_theta=33, rstar_min=-20.0, rstar_max=1980.0, rstar_obs=40.0,
                      source=dict(r0=10.0, phase0=0.7, ramp=args.seg_ramp), name="kerr a=0.9 m=2 r0=10")
    T, n, ov = args.seg_total, args.seg_count, args.seg_overlap
    segs, info = SEG.plan(inst, T, n, ov)
    K, dt = inst["extract_every"], inst["dt"]

    def timed(insts, steps):
        st = tk.Stepper(insts, wave_capacity=steps // K + 64)
        for k, i in enumerate(insts):
            st.set_fields(k, *W.initial_data(i))
        st.autotune(warmup=2, steps=6)
        t = st.get_tuning()
        t["graph_steps"] = 100
        st.set_tuning(**t)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st.stream)
        st.step(steps)
        ev1.record(st.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        eq = insts[0]["n_theta"] // 2
        waves = [st.extract(k, max_samples=steps // K + 64)[:, eq] for k in range(len(insts))]
        st.close()
        return ms / 1e3, waves, t

    n_total = n * info["samples_per_segment"]
    t_long, (w_long,), tune_long = timed([inst], n_total * K)
    t_seg, waves, tune_seg = timed(segs, info["steps"])
    p = SEG.patch(waves, info)
    n_L = info["samples_per_segment"]
    # compare where the long run has settled too: intervals starting after
    # one overlap (the long run switched its source on at t = 0)
    k0 = int(np.ceil(info["overlap"] / info["L"] - 1e-9))
    per_seg = [float(np.max(np.abs(p[k * n_L:(k + 1) * n_L] - w_long[k * n_L:(k + 1) * n_L])) /
                     np.max(np.abs(w_long[k * n_L:(k + 1) * n_L]))) for k in range(k0, n)]
    err = max(per_seg)
    amp_long = [float(np.max(np.abs(w_long[k * n_L:(k + 1) * n_L]))) for k in range(n)]
    amp_patch = [float(np.max(np.abs(p[k * n_L:(k + 1) * n_L]))) for k in range(n)]
    pts = inst["n_r"] * inst["n_theta"]
    out = {
        "metric": "temporal segments (Section 4) on one GPU: time to solution of a long waveform, one run vs "
                  "batched segments, and the patched waveform's agreement with the long run",
        "workload": f"Kerr a=0.9, s=-2, m=2, circular orbit r0=10M; 8001 x 33 on [-20,1980]M, observer 40M "
                    f"(equator row); T = {n_total * K * dt:.0f}M; every run switches its source on over "
                    f"{args.seg_ramp}M",
        "segments": n, "segment_M": info["L"], "overlap_M": info["overlap"], "ramp_M": args.seg_ramp,
        "long_run": {"seconds": t_long, "steps": n_total * K, "updates_per_s": pts * n_total * K / t_long,
                     "tuning": tune_long},
        "batched_segments": {"seconds": t_seg, "steps": info["steps"], "instances": n,
                             "updates_per_s": pts * n * info["steps"] / t_seg, "tuning": tune_seg},
        "time_to_solution_speedup": t_long / t_seg,
        "work_ratio": n * info["steps"] / (n_total * K),
        "compared_from_M": k0 * info["L"],
        "patched_vs_long_max_rel_err": err,
        "patched_vs_long_rel_err_by_segment": per_seg,
        "long_run_max_amplitude_by_segment": amp_long,
        "patched_max_amplitude_by_segment": amp_patch,
    }
    print(json.dumps(out), flush=True)


def launch_plan(steps, graph_steps, two_step):
    """The launches tk_step(steps) issues: replays of the captured graph of
    graph_steps steps, then the rest directly; with the two-step kernel each
    pair of steps is one launch and an odd count ends with one one-step
    launch (per graph and per direct remainder).  Every graph and every
    direct run ends with one control-block bump."""
    if steps < 0 or graph_steps < 0:
        raise ValueError("steps and graph_steps must be >= 0")

    def split(n):
        return (n // 2, n % 2) if two_step else (0, n)

    G = graph_steps
    replays = steps // G if G > 0 else 0
    rest = steps - replays * G
    g2, g1 = split(G) if G > 0 else (0, 0)
    r2, r1 = split(rest)
    return {"graph_replays": replays, "two_step_launches": replays * g2 + r2,
            "one_step_launches": replays * g1 + r1, "bumps": replays + (1 if rest else 0)}


def bench_graph_steps(steps, graph_steps, two_step):
    """Graph block length for a timed run of `steps`: the requested length,
    cut to the timed count so that the timed steps go through graph replays,
    and even for the two-step kernel (whole launches)."""
    G = min(graph_steps, steps)
    if two_step:
        G -= G % 2
    return max(G, 0)


def run_leg(args, insts, inits, precision):
    """One timed throughput run of the stepper on `insts` in `precision`:
    autotune (or the manual shape), graph capture, W warm-up steps, then K
    timed steps bracketed by HIP events on the context's stream.  The timed
    K are issued as two calls, the whole launches of the dominant kernel
    first (even count for the two-step kernel), so its average launch time
    is measured on its own; the second call holds the odd last step, if any."""
    import torch
    from paper_1206_0270_amd import tk

    prec = tk.TK_FP64 if precision == "fp64" else tk.TK_FP32_COMP
    points = sum(i["n_r"] * i["n_theta"] for i in insts)
    st = tk.Stepper(insts, precision=prec)
    for k, (phi, pi) in enumerate(inits):
        st.set_fields(k, phi, pi)
    if args.tune == "auto":
        tune_ms, tried = st.autotune(warmup=2, steps=6)
        t = st.get_tuning()
        print(f"# {precision}: autotune {tried} launch shapes, best {tune_ms:.4f} ms/step: {t}", file=sys.stderr,
              flush=True)
    else:
        kern = {"fused2": tk.TK_KERNEL_FUSED2, "fused": tk.TK_KERNEL_FUSED,
                "two_pass": tk.TK_KERNEL_TWO_PASS, "tiled": tk.TK_KERNEL_TILED}[args.kernel]
        st.set_tuning(kernel=kern, rows_per_tile=args.rows, graph_steps=0, prefetch_rows=args.prefetch,
                      nt_stores=not args.no_nt)
        t = st.get_tuning()
    kernel = {tk.TK_KERNEL_FUSED2: "fused2", tk.TK_KERNEL_FUSED: "fused",
              tk.TK_KERNEL_TWO_PASS: "two_pass", tk.TK_KERNEL_TILED: "tiled"}[t["kernel"]]
    if t["kernel"] == tk.TK_KERNEL_AUTO:
        kernel = "fused2" if t["rows_per_tile"] == 0 else "fused"
    two_step = kernel == "fused2"
    K = args.steps
    K_main = K - (K % 2) if two_step else K
    t["graph_steps"] = bench_graph_steps(K_main, args.graph_steps, two_step)
    st.set_tuning(**t)
    st.prepare(K_main)  # work list and graph capture, outside the timed region
    print(f"# {precision}: {len(insts)} instances, {points} points, {st.workspace_bytes / 2**30:.2f} GiB workspace, "
          f"kernel {kernel}, graph of {t['graph_steps']} steps", file=sys.stderr, flush=True)
    st.step(args.warmup)
    torch.cuda.synchronize()
    stream = st.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    c0 = st.counters()
    t0 = time.perf_counter()
    ev[0].record(stream)
    st.step(K_main)
    ev[1].record(stream)
    st.step(K - K_main)
    ev[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = st.counters()
    main_ms = ev[0].elapsed_time(ev[1])
    gpu_ms = ev[0].elapsed_time(ev[2])
    elapsed = max(wall, gpu_ms / 1e3)
    print(f"# {precision}: timed {K} steps: events {gpu_ms:.3f} ms, wall {wall * 1e3:.3f} ms, "
          f"graph replays {c1['graph_launches'] - c0['graph_launches']}", file=sys.stderr, flush=True)
    plan = launch_plan(K_main, t["graph_steps"], two_step)
    # Roofline of the dominant kernel.  One launch reads the state u^n once
    # and writes the new state once (32 + 32 B per point in FP64; 24 + 24 B in
    # the FP32-compensated form), whether it advances one step or two: those
    # are the bytes it must move.  The launch time is the first timed call's
    # event time over its launches (its graph's control-block bump, a few
    # microseconds, included).
    spl = 2 if two_step else 1
    n_launch = plan["two_step_launches"] if two_step else plan["one_step_launches"]
    bpp = BYTES_PER_UPDATE[precision]  # per point and launch: one read and one write of the state
    if kernel == "two_pass":
        kname = "k_two_pass_half + k_two_pass_full"
    elif kernel == "tiled":
        kname = (f"k_tiled<{KERNEL_POLICY[precision]}<1, {'true' if t['nt_stores'] else 'false'}, 1>, "
                 f"{t['rows_per_tile'] + 2}>")
    else:
        kname = kernel_name(precision, t["prefetch_rows"], t["nt_stores"], t["waves_per_simd"], two_step,
                            t["rows_per_tile"] > 0)
    roof = None
    if n_launch > 0:
        launch_s = main_ms / 1e3 / n_launch
        upd = points * spl  # point updates per launch
        moved = points * bpp
        gbs = moved / launch_s / 1e9
        fpu = flops_per_update(precision, two_step)
        tflops = fpu * upd / launch_s / 1e12
        issue = valu_entry(kname, args.workload, upd / launch_s)
        # The fused kernels are bound by vector-ALU issue (the counters show
        # the VALU busy most cycles at a fraction of the HBM bandwidth), so the
        # roofline is the ALU one; the bytes the launch moves are reported
        # beside it against the HBM peak.
        roof = {"bound": "alu", "achieved": tflops, "peak": ALU_PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                "frac": tflops / ALU_PEAK_TFLOPS[precision], "traffic": traffic_entry(kname, args.workload),
                "kernel": kname, "avg_launch_ms": launch_s * 1e3, "launches_timed": n_launch,
                "flops_per_update": fpu, "updates_per_point_per_launch": spl,
                "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "bytes_per_launch": moved, "bytes_per_point_per_launch": bpp,
                        # the same launch priced at one read and one write of the state per update: twice
                        # the bytes actually moved for the two-step kernel
                        "effective_GBps_at_per_update_bytes": upd * bpp / launch_s / 1e9},
                "issue": issue}
    st.close()
    del st
    torch.cuda.empty_cache()
    return {"value": points * K / elapsed, "ms_per_step": elapsed * 1e3 / K, "kernel": kernel, "tuning": t,
            "plan": plan, "graph_replays_timed": c1["graph_launches"] - c0["graph_launches"], "roofline": roof}


def build_parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="batched", choices=["batched", "single", "precision"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c"])
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--tune", default="auto", choices=["auto", "manual"],
                    help="auto: the library's autotuner picks the launch shape before timing; "
                         "manual: the shape given by --kernel/--rows/--prefetch/--no-nt")
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--kernel", default="fused2", choices=["fused2", "fused", "two_pass", "tiled"],
                    help="fused2: two time steps per pass (needs --rows 0); fused: one step per pass; "
                         "two_pass: half-step array through HBM")
    ap.add_argument("--prefetch", type=int, default=3, choices=[1, 3])
    ap.add_argument("--no-nt", action="store_true", help="plain (not non-temporal) stores")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="time only --precision on --workload (no second precision, no single-mode or layered leg)")
    ap.add_argument("--precision-study", action="store_true",
                    help="instead of the throughput line, run the FP32-compensated vs FP64 waveform study")
    ap.add_argument("--study-window", type=float, default=600.0, help="precision study: simulated time (M)")
    ap.add_argument("--study-checkpoints", type=float, nargs="+", default=[300.0, 400.0, 500.0, 600.0])
    ap.add_argument("--study-oracle-steps", type=int, default=2000)
    ap.add_argument("--study-ramp", type=float, default=0.0,
                    help="precision study: switch-on time of the sources (M; 0 = abrupt)")
    ap.add_argument("--study-layer", type=float, default=0.0,
                    help="precision study: end the grids in a hyperboloidal layer from this r* (M) on and read the "
                         "waveform at null infinity (0 = the plain grids, observer at 290M)")
    ap.add_argument("--noise-study", action="store_true",
                    help="instead of the throughput line, evolve white noise under the FP64 scheme at four resolutions")
    ap.add_argument("--noise-window", type=float, default=500.0, help="noise study: simulated time (M)")
    ap.add_argument("--sensitivity-study", action="store_true",
                    help="instead of the throughput line, compare FP32C and a once-perturbed FP64 run with FP64")
    ap.add_argument("--sens-instance", type=int, default=1, help="sensitivity study: instance index in the six-mode workload")
    ap.add_argument("--sens-at", type=float, default=300.0, help="sensitivity study: perturbation time (M)")
    ap.add_argument("--sens-window", type=float, default=1000.0, help="sensitivity study: simulated time (M)")
    ap.add_argument("--sens-checkpoints", type=float, nargs="+",
                    default=[300.0, 350.0, 400.0, 450.0, 500.0, 600.0, 700.0, 800.0, 900.0, 1000.0])
    ap.add_argument("--richardson", action="store_true",
                    help="instead of the throughput line, run the three-resolution Richardson study")
    ap.add_argument("--rich-window", type=float, default=330.0, help="Richardson study: simulated time (M)")
    ap.add_argument("--rich-h", type=float, default=0.04, help="Richardson study: coarse r* spacing (M)")
    ap.add_argument("--rich-nth", type=int, default=33, help="Richardson study: coarse theta rows")
    ap.add_argument("--rich-sigma-r", type=float, default=0.5, help="Richardson study: source width in r* (M)")
    ap.add_argument("--rich-sigma-th", type=float, default=4.0, help="Richardson study: source width, coarse theta cells")
    ap.add_argument("--source-study", action="store_true",
                    help="compare the Gaussian and the two discrete-delta particles under refinement")
    ap.add_argument("--src-window", type=float, default=330.0, help="source study: simulated time (M)")
    ap.add_argument("--src-h", type=float, default=0.08, help="source study: coarse r* spacing (M)")
    ap.add_argument("--src-nth", type=int, default=33, help="source study: coarse theta rows")
    ap.add_argument("--segments", action="store_true",
                    help="instead of the throughput line, run the temporal-segments study")
    ap.add_argument("--seg-total", type=float, default=3600.0, help="segments study: length of the long run (M)")
    ap.add_argument("--seg-count", type=int, default=36, help="segments study: number of segments")
    ap.add_argument("--seg-overlap", type=float, default=300.0, help="segments study: overlap per segment (M)")
    ap.add_argument("--seg-ramp", type=float, default=0.0,
                    help="segments study: switch-on time of the source in every run (M; 0 = abrupt)")
    ap.add_argument("--layer-study", action="store_true",
                    help="hyperboloidal layer vs a wall and a long domain, and the layer kernels' step rate")
    ap.add_argument("--layer-h", type=float, default=0.075, help="layer study: r* spacing (M)")
    ap.add_argument("--layer-nth", type=int, default=65, help="layer study: theta rows")
    ap.add_argument("--layer-window", type=float, default=600.0, help="layer study: simulated time (M)")
    ap.add_argument("--layer-start", type=float, default=60.0, help="layer study: R, where the layer begins (M)")
    ap.add_argument("--layer-steps", type=int, default=600, help="layer study: timed steps of the throughput leg")
    ap.add_argument("--layer-warmup", type=int, default=100, help="layer study: warm-up steps of the throughput leg")
    ap.add_argument("--layer-throughput", action="store_true",
                    help="only the layer study's throughput leg (one JSON line; short enough to profile)")
    ap.add_argument("--layer-from", type=float, default=150.0,
                    help="layer study: compare waveforms from this time on (M)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="instead of the stepper, run a plain device copy of this many GiB "
                         "(calibrates the HBM byte counters)")
    return ap


def parse_args(argv=None):
    """Command line of the benchmark (no device is touched)."""
    ap = build_parser()
    args = ap.parse_args(argv)
    if args.steps < 1:
        ap.error("--steps must be >= 1")
    if args.warmup < 0 or args.graph_steps < 0:
        ap.error("--warmup and --graph-steps must be >= 0")
    return args


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the stepper's "
              f"multi-GPU sharding is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    if args.precision_study:
        precision_study(args)
        return
    if args.noise_study:
        noise_study(args)
        return
    if args.sensitivity_study:
        sensitivity_study(args)
        return
    if args.richardson:
        richardson_study(args)
        return
    if args.segments:
        segments_study(args)
        return
    if args.source_study:
        source_study(args)
        return
    if args.layer_study:
        layer_study(args)
        return
    if args.layer_throughput:
        print(json.dumps(dict(metric="hyperboloidal layer kernels: grid-point updates per second",
                              **layer_throughput(args))), flush=True)
        return
    import torch
    from paper_1206_0270_amd import tk
    from paper_1206_0270_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_gib > 0:
        n = int(args.copy_gib * 2 ** 30)
        x = torch.ones(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            y.copy_(x)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            y.copy_(x)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "ms_per_copy": ms,
                          "GB_per_s": 2 * n / ms / 1e6}), flush=True)
        return
    insts, desc = workload(args.workload)
    inits = [W.initial_data(inst) for inst in insts]
    points = W.points(insts)
    main_leg = run_leg(args, insts, inits, args.precision)
    other = "fp32c" if args.precision == "fp64" else "fp64"
    legs = {args.precision: main_leg}
    if not args.no_legs:
        legs[other] = run_leg(args, insts, inits, other)
    del inits
    single = None
    if not args.no_legs and args.workload != "single":
        s_insts, s_desc = workload("single")
        single = run_leg(args, s_insts, [W.initial_data(i) for i in s_insts], "fp64")
        single["workload"] = s_desc
    layered = None
    if not args.no_legs and args.workload == "batched":
        # the six 16001 x 129 modes ending in hyperboloidal layers, timed over
        # the same step counts; reported beside the line, never in its place
        la = argparse.Namespace(**vars(args))
        la.layer_steps, la.layer_warmup, la.precision = args.steps, args.warmup, "fp64"
        try:
            layered = layer_throughput(la)
        except Exception as exc:
            print(f"# layered leg not measured: {exc}", file=sys.stderr, flush=True)

    leg = main_leg
    out = {
        "metric": METRIC,
        "value": leg["value"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+bf16comp",
        "data": "synthetic",
        "config": {"workload": desc, "instances": len(insts), "points": points,
                   "precision": args.precision, "kernel": leg["kernel"], "tuning": args.tune,
                   "graph_steps": leg["tuning"]["graph_steps"], "rows_per_tile": leg["tuning"]["rows_per_tile"],
                   "prefetch_rows": leg["tuning"]["prefetch_rows"], "nt_stores": leg["tuning"]["nt_stores"],
                   "launches": leg["plan"], "graph_replays_timed": leg["graph_replays_timed"]},
        "roofline": leg["roofline"],
    }
    if "fp64" in legs and "fp32c" in legs:
        f64, f32 = legs["fp64"], legs["fp32c"]
        out["fp32c"] = {"value": f32["value"], "ms_per_step": f32["ms_per_step"], "kernel": f32["kernel"],
                        "tuning": f32["tuning"], "roofline": f32["roofline"],
                        "fp32c_over_fp64": f32["value"] / f64["value"]}
    if single is not None:
        out["fp64_single_mode"] = {"workload": single["workload"], "value": single["value"],
                                   "ms_per_step": single["ms_per_step"], "kernel": single["kernel"],
                                   "tuning": single["tuning"],
                                   "note": "about 1e6 points: the state (66 MB) stays in the 256 MB Infinity "
                                           "Cache, so no HBM roofline is claimed for it"}
        if "fp32c" in legs:
            out["fp32c"]["fp32c_batched_over_fp64_single_mode"] = legs["fp32c"]["value"] / single["value"]
    if layered is not None:
        out["fp64_layered"] = {"workload": layered["workload"], "value": layered["updates_per_s"],
                               "ms_per_step": layered["ms_per_step"], "tuning": layered["tuning"],
                               "bytes_per_update": layered["bytes_per_update"],
                               "frac_of_8TBps": layered["frac_of_8TBps"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(insts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
