"""Temporal segments (Section 4): a long run split into short runs that
advance together as one batch, then patched into one waveform.

For a linear problem driven by a source whose time history is known in
advance, segment k (k = 0 .. n-1) covers [k L, (k+1) L) of the long run with
L = T / n.  It starts from zero fields at t0 = k L - overlap (the source's
time origin, tk_source_desc.t0), so that the burst of junk radiation from
switching the source on has passed the observer before its own interval
begins.  All segments take the same number of steps, so one batched context
advances them together.  Patching keeps each segment's samples inside its
interval.  The overlap is the price: (L + overlap) / L times the work of the
long run, traded for n times the parallelism.
"""
import numpy as np


def plan(inst, t_total, n_seg, overlap):
    """Segment instances for a sourced instance (dict as in workloads) and the
    steps each takes.  L and the overlap are rounded to whole waveform
    sampling intervals (extract_every steps)."""
    if not inst.get("source"):
        raise ValueError("temporal segments need a source (the forcing that drives the solution)")
    if n_seg < 1 or t_total <= 0 or overlap < 0:
        raise ValueError("need n_seg >= 1, t_total > 0, overlap >= 0")
    dt, K = inst["dt"], inst["extract_every"]
    if K <= 0:
        raise ValueError("segments are patched from waveform samples: extract_every must be > 0")
    n_L = int(round(t_total / n_seg / (K * dt)))      # samples per segment interval
    n_ov = int(np.ceil(overlap / (K * dt) - 1e-9))    # samples of overlap
    if n_L < 1:
        raise ValueError("segments shorter than one sampling interval")
    L, ov = n_L * K * dt, n_ov * K * dt
    segs = []
    for k in range(n_seg):
        src = dict(inst["source"])
        src["t0"] = src.get("t0", 0.0) + k * L - ov
        segs.append(dict(inst, source=src, name=f"{inst.get('name', '')}/seg{k}"))
    info = dict(n_seg=n_seg, samples_per_segment=n_L, overlap_samples=n_ov, L=L, overlap=ov,
                steps=(n_L + n_ov) * K)
    return segs, info


def patch(waves, info):
    """One waveform from the segments' samples ([segment][sample][...]):
    segment k contributes the n_L samples after its n_ov overlap samples,
    i.e. the long run's samples k n_L .. (k+1) n_L - 1."""
    n_L, n_ov = info["samples_per_segment"], info["overlap_samples"]
    parts = []
    for w in waves:
        w = np.asarray(w)
        if len(w) < n_ov + n_L:
            raise ValueError("a segment has fewer samples than its overlap and interval")
        parts.append(w[n_ov:n_ov + n_L])
    return np.concatenate(parts)
