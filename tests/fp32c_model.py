"""ctypes wrapper of the CPU model of FP32 arithmetic forms of the scheme
(tests/fp32c_model.c).

TEST INFRASTRUCTURE: used by the test suite and by the rounding study
(tests/fp32c_study.py).  The model takes the oracle's FP64 coefficient planes
and source space factor, and re-runs Eqs. (3)-(4) with FP32 rounding switched
on where its flags say.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fp32c_model.c")
LIB = os.path.join(HERE, "_fp32c_model.so")

ARITH32, STORE32, DIFF_RAD, DIFF_ANG, HALF_PAIR, COEF64 = 1, 2, 4, 8, 16, 32

# named arithmetic forms
FORMS = {
    "fp64": 0,
    # FP32 + bf16 storage with FP64 arithmetic: the storage format alone
    "store": STORE32,
    # the stencil in FP32 on the stored FP32 value alone, the angular operator
    # as one weighted sum of values, FP32 half-step values, compensated update
    "values": ARITH32 | STORE32,
    # + radial differences from value and Kahan term
    "values+rad": ARITH32 | STORE32 | DIFF_RAD,
    # + angular operator as differences first (from value and Kahan term)
    "values+ang": ARITH32 | STORE32 | DIFF_ANG,
    # + compensated averages and half-step values
    "values+half": ARITH32 | STORE32 | HALF_PAIR,
    # every difference from compensated values, compensated half-step values
    "differences": ARITH32 | STORE32 | DIFF_RAD | DIFF_ANG | HALF_PAIR,
}


class FmDesc(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int), ("nth", ctypes.c_int),
        ("h", ctypes.c_double), ("dth", ctypes.c_double), ("dt", ctypes.c_double),
        ("pole_even", ctypes.c_int), ("layer", ctypes.c_int),
        ("i_obs", ctypes.c_int), ("extract_every", ctypes.c_int),
        ("m", ctypes.c_double), ("Omega", ctypes.c_double), ("t0", ctypes.c_double), ("ramp", ctypes.c_double),
        ("flags", ctypes.c_int),
    ]


_dp = ctypes.POINTER(ctypes.c_double)
_lib_cache = []


def build():
    subprocess.run(["gcc", "-std=c99", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wextra",
                    SRC, "-o", LIB + ".tmp", "-lm"], check=True)
    os.replace(LIB + ".tmp", LIB)


def _lib():
    if not _lib_cache:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        lib.fm_new.restype = ctypes.c_void_p
        lib.fm_new.argtypes = [ctypes.POINTER(FmDesc), _dp, _dp]
        lib.fm_free.restype = None
        lib.fm_free.argtypes = [ctypes.c_void_p]
        lib.fm_set_state.restype = None
        lib.fm_set_state.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_long]
        lib.fm_get_state.restype = None
        lib.fm_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        lib.fm_run.restype = ctypes.c_long
        lib.fm_run.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.fm_get_wave.restype = ctypes.c_long
        lib.fm_get_wave.argtypes = [ctypes.c_void_p, _dp, ctypes.c_long]
        lib.fm_set_threads.restype = None
        lib.fm_set_threads.argtypes = [ctypes.c_int]
        _lib_cache.append(lib)
    return _lib_cache[0]


def _p(a):
    return a.ctypes.data_as(_dp)


def oracle_grid(inst):
    """The oracle grid of an instance (workloads.instance dict)."""
    return oracle.Grid(a=inst["a"], s=inst["s"], m=inst["m"], n_r=inst["n_r"], n_theta=inst["n_theta"],
                       rstar_min=inst["rstar_min"], rstar_max=inst["rstar_max"], dt=inst["dt"],
                       i_obs=inst["i_obs"], extract_every=inst["extract_every"], source=inst.get("source"),
                       layer_R=inst.get("layer_start", 0.0))


def planes_of(inst):
    """Coefficient planes [q][j][12] and the source's space factor [q][j][2]
    (A g_r g_theta exp(-i m phase0), no time factor and no ramp) from the
    oracle, for q = 0 .. 2 n_r - 2."""
    g = oracle_grid(inst)
    nq, nth = 2 * inst["n_r"] - 1, inst["n_theta"]
    coef = np.zeros((nq, nth, 12))
    for q in range(nq):
        col = g.coeff_column(q)
        coef[q, :, 0] = col["b"]
        coef[q, :, 1] = col["cthth"]
        coef[q, :, 2] = col["cth"]
        coef[q, :, 3] = col["ct"].real
        coef[q, :, 4] = col["ct"].imag
        coef[q, :, 5] = col["c0"].real
        coef[q, :, 6] = col["c0"].imag
        coef[q, :, 7] = col["d"].real
        coef[q, :, 8] = col["d"].imag
        coef[q, :, 9] = col["bi"]
        coef[q, :, 10] = col["fw"]
    src = np.zeros((nq, nth, 2))
    s = inst.get("source")
    if s:
        plain = dict(s, t0=0.0, ramp=0.0)
        gs = oracle_grid(dict(inst, source=plain))
        rs, _ = gs.radial()
        th = np.arange(nth) * (math.pi / (nth - 1))
        for q in range(nq):
            if not np.isfinite(rs[q]) or gs.source_value(0.0, rs[q], math.pi / 2) == 0 and \
                    all(gs.source_value(0.0, rs[q], t) == 0 for t in th[1:-1]):
                continue
            for j in range(1, nth - 1):
                v = gs.source_value(0.0, rs[q], th[j])
                src[q, j] = (v.real, v.imag)
    return coef, src


class Model:
    """One model instance in one arithmetic form (a FORMS key or flags)."""

    def __init__(self, inst, form, planes=None):
        self.lib = _lib()
        flags = FORMS[form] if isinstance(form, str) else int(form)
        coef, src = planes if planes is not None else planes_of(inst)
        self._keep = (np.ascontiguousarray(coef), np.ascontiguousarray(src))
        d = FmDesc()
        d.nr, d.nth = inst["n_r"], inst["n_theta"]
        d.h = (inst["rstar_max"] - inst["rstar_min"]) / (inst["n_r"] - 1)
        d.dth = math.pi / (inst["n_theta"] - 1)
        d.dt = inst["dt"]
        d.pole_even = int((inst["m"] + inst["s"]) % 2 == 0)
        d.layer = int(inst.get("layer_start", 0.0) > 0)
        d.i_obs, d.extract_every = inst["i_obs"], inst["extract_every"]
        s = inst.get("source")
        d.m = inst["m"]
        d.Omega = oracle.orbit_omega(inst["M"], inst["a"], s["r0"]) if s else 0.0
        d.t0 = s.get("t0", 0.0) if s else 0.0
        d.ramp = s.get("ramp", 0.0) if s else 0.0
        d.flags = flags
        self.inst = inst
        self._h = self.lib.fm_new(ctypes.byref(d), _p(self._keep[0]), _p(self._keep[1]))
        if not self._h:
            raise MemoryError("model allocation failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.lib.fm_free(h)
            self._h = None

    def set_state(self, phi, pi, step=0):
        phi = np.ascontiguousarray(phi, np.complex128)
        pi = np.ascontiguousarray(pi, np.complex128)
        self.lib.fm_set_state(self._h, _p(phi.view(np.float64)), _p(pi.view(np.float64)), int(step))

    def get_state(self):
        n_th, n_r = self.inst["n_theta"], self.inst["n_r"]
        phi = np.zeros((n_th, n_r), np.complex128)
        pi = np.zeros((n_th, n_r), np.complex128)
        self.lib.fm_get_state(self._h, _p(phi.view(np.float64)), _p(pi.view(np.float64)))
        return phi, pi

    def run(self, n):
        return self.lib.fm_run(self._h, int(n))

    def waveform(self):
        n = self.lib.fm_run(self._h, 0)
        out = np.zeros((max(n, 1), self.inst["n_theta"]), np.complex128)
        got = self.lib.fm_get_wave(self._h, _p(out.view(np.float64)), n)
        return out[:got]


def set_threads(n):
    _lib().fm_set_threads(int(n))
