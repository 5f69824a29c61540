"""Rounding study on the CPU model of FP32 arithmetic forms (tests/fp32c_model.c).

TEST INFRASTRUCTURE (not collected by pytest).  One sourced Kerr mode
(a = 0.9, m = 2, s = -2, circular orbit at r0 = 8M, dt = 1/500 as in the
six-mode workload) on a short r* grid, run in FP64 and in the FP32 forms named
on the command line; prints the waveform amplitude and phase errors of each
form against the FP64 run (the error of the six-mode workload's precision study:
projection on the l = max(|m|, 2) harmonic, samples above 1e-3 of the peak).

    python tests/fp32c_study.py [--probe wall|layer] [--nth 33] [--h 0.0375]
        [--window 250] [--ramp 0] [--forms values differences store]

Probes: "wall" ends the grid at r* = 150M with the Dirichlet condition of
Section 2.2 and reads the waveform at 140M (the reflection from the wall
amplifies ingoing errors, which makes the probe sensitive); "layer" ends it
in a hyperboloidal layer on [100, 150]M and reads the waveform at null
infinity.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import bench  # noqa: E402  (waveform projection and error metric)
import fp32c_model as FM  # noqa: E402
from paper_1206_0270_amd import workloads as W  # noqa: E402


def probe_instance(probe, nth, h, ramp, rmin=-100.0, rmax=150.0):
    n_r = int(round((rmax - rmin) / h)) + 1
    src = dict(r0=8.0, amplitude=1.0, phase0=float(W.rng_for(5).uniform(0, 2 * math.pi)),
               sigma_r_cells=2.0, sigma_th_cells=2.0, window_sigmas=6.0, ramp=ramp)
    if probe == "wall":
        return W.instance(a=0.9, m=2, n_r=n_r, n_theta=nth, rstar_min=rmin, rstar_max=rmax, dt=1.0 / 500,
                          rstar_obs=rmax - 10.0, source=src, name=f"probe-wall-{nth}")
    return W.instance(a=0.9, m=2, n_r=n_r, n_theta=nth, rstar_min=rmin, rstar_max=rmax, dt=1.0 / 500,
                      source=src, layer_start=100.0, name=f"probe-layer-{nth}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--probe", choices=["wall", "layer"], default="wall")
    ap.add_argument("--nth", type=int, default=33)
    ap.add_argument("--h", type=float, default=0.0375)
    ap.add_argument("--window", type=float, default=250.0)
    ap.add_argument("--ramp", type=float, default=0.0)
    ap.add_argument("--checkpoints", type=float, nargs="+", default=None)
    ap.add_argument("--forms", nargs="+", default=["values", "differences", "store"])
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args(argv)
    if args.threads:
        FM.set_threads(args.threads)
    inst = probe_instance(args.probe, args.nth, args.h, args.ramp)
    steps = int(round(args.window / inst["dt"]))
    cps = args.checkpoints or [args.window * k / 5 for k in range(1, 6)]
    planes = FM.planes_of(inst)
    init = W.initial_data(inst)
    waves = {}
    for form in ["fp64"] + [f for f in args.forms if f != "fp64"]:
        t = time.time()
        m = FM.Model(inst, form, planes)
        m.set_state(*init)
        m.run(steps)
        waves[form] = bench.projected_waveform(inst, m.waveform())
        print(f"# {form}: {steps} steps in {time.time() - t:.0f} s", file=sys.stderr, flush=True)
        del m
    K = inst["extract_every"]
    rows = []
    for form in args.forms:
        row = {"form": form, "flags": FM.FORMS[form]}
        for T in cps:
            n = min(len(waves["fp64"]), int(round(T / (K * inst["dt"]))))
            amp, ph = bench.waveform_errors(waves["fp64"][:n], waves[form][:n])
            row[f"T{int(T)}"] = {"amp": amp, "phase": ph}
        rows.append(row)
    out = {"probe": args.probe, "instance": {k: inst[k] for k in ("a", "m", "s", "n_r", "n_theta", "rstar_min",
                                                                  "rstar_max", "dt", "rstar_obs", "layer_start")},
           "ramp_M": args.ramp, "window_M": args.window, "steps": steps, "errors_vs_fp64": rows}
    print(json.dumps(out), flush=True)
    for r in rows:
        print(f"# {r['form']:12s} " + "  ".join(
            f"T{int(T)}: {r[f'T{int(T)}']['amp']:.2e}/{r[f'T{int(T)}']['phase']:.2e}" for T in cps), file=sys.stderr)


if __name__ == "__main__":
    main()
