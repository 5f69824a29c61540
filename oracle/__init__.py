"""ctypes wrapper around the plain C oracle (teuk_oracle.c).

TEST INFRASTRUCTURE.  Only tests/, the smoke check in __graft_entry__.py and
the cpu_baseline leg of bench.py may import this package.  The product path
(paper_1206_0270_amd) never imports it, and the two share no code.

The oracle evolves one azimuthal mode of the Teukolsky equation (Eq. (1),
decomposed by Eq. (2)) with the two-step Lax-Wendroff scheme of Eqs. (3)-(4)
and the boundary conditions of Section 2.2, in plain FP64 (or long double).
Host arrays are complex128 numpy arrays of shape (n_theta, n_r): theta rows,
r* fastest.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}


class OrDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_double), ("a", ctypes.c_double),
        ("s", ctypes.c_int), ("m", ctypes.c_int),
        ("n_r", ctypes.c_int), ("n_theta", ctypes.c_int),
        ("rstar_min", ctypes.c_double), ("rstar_max", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("i_obs", ctypes.c_int), ("extract_every", ctypes.c_int),
        ("src_kind", ctypes.c_int),
        ("src_r0", ctypes.c_double), ("src_amp", ctypes.c_double),
        ("src_phase0", ctypes.c_double),
        ("src_sigma_r_cells", ctypes.c_double),
        ("src_sigma_th_cells", ctypes.c_double),
        ("src_window_sigmas", ctypes.c_double),
        ("src_t0", ctypes.c_double),
        ("src_ramp", ctypes.c_double),
        ("layer_R", ctypes.c_double),
    ]


_dp = ctypes.POINTER(ctypes.c_double)


def _lib(kind="f64"):
    """kind: "f64", "ld", or the path of another build of teuk_oracle.c."""
    if kind not in _LIBS:
        if kind in _build.LIBS:
            path = _build.LIBS[kind]
            if not os.path.exists(path):
                _build.build()
        else:
            path = kind
        lib = ctypes.CDLL(path)
        lib.or_tortoise.restype = ctypes.c_double
        lib.or_tortoise.argtypes = [ctypes.c_double] * 3
        lib.or_x_of_rstar.restype = ctypes.c_double
        lib.or_x_of_rstar.argtypes = [ctypes.c_double] * 3
        lib.or_coeffs.restype = None
        lib.or_coeffs.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, _dp]
        lib.or_orbit_omega.restype = ctypes.c_double
        lib.or_orbit_omega.argtypes = [ctypes.c_double] * 3
        lib.or_grid_new.restype = ctypes.c_void_p
        lib.or_grid_new.argtypes = [ctypes.POINTER(OrDesc)]
        lib.or_grid_free.restype = None
        lib.or_grid_free.argtypes = [ctypes.c_void_p]
        lib.or_set_state.restype = None
        lib.or_set_state.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_long]
        lib.or_get_state.restype = None
        lib.or_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
        lib.or_get_step.restype = ctypes.c_long
        lib.or_get_step.argtypes = [ctypes.c_void_p]
        lib.or_step.restype = None
        lib.or_step.argtypes = [ctypes.c_void_p, _dp, _dp]
        lib.or_run.restype = ctypes.c_long
        lib.or_run.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.or_get_wave.restype = ctypes.c_long
        lib.or_get_wave.argtypes = [ctypes.c_void_p, _dp, ctypes.c_long]
        lib.or_get_radial.restype = None
        lib.or_get_radial.argtypes = [ctypes.c_void_p, _dp, _dp]
        lib.or_rhs_column.restype = None
        lib.or_rhs_column.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
        lib.or_get_coeff_column.restype = None
        lib.or_get_coeff_column.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        lib.or_layer_map.restype = None
        lib.or_layer_map.argtypes = [ctypes.c_double] * 3 + [_dp]
        lib.or_layer_coeffs.restype = None
        lib.or_layer_coeffs.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _dp]
        lib.or_source_value.restype = None
        lib.or_source_value.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _dp]
        lib.or_set_threads.restype = None
        lib.or_set_threads.argtypes = [ctypes.c_int]
        lib.or_get_threads.restype = ctypes.c_int
        lib.or_get_threads.argtypes = []
        lib.or_real_bytes.restype = ctypes.c_int
        lib.or_real_bytes.argtypes = []
        _LIBS[kind] = lib
    return _LIBS[kind]


def _ptr(a):
    return a.ctypes.data_as(_dp)


def tortoise(M, a, x, kind="f64"):
    """r*(x) with x = r - r_+ (closed form, integration constant 2M scale)."""
    return _lib(kind).or_tortoise(M, a, x)


def x_of_rstar(M, a, rstar, kind="f64"):
    """x = r - r_+ such that r*(r) = rstar (inverse tortoise coordinate)."""
    return _lib(kind).or_x_of_rstar(M, a, rstar)


def coeffs(M, a, s, m, x, theta, kind="f64"):
    """Coefficients of the first-order system at (r = r_+ + x, theta).

    Returns a dict with b, bp (= d b / d r*), cthth, cth, and complex ct, c1, c0,
    d, plus r and Delta."""
    out = np.zeros(14)
    _lib(kind).or_coeffs(M, a, s, m, x, theta, _ptr(out))
    return dict(b=out[0], bp=out[1], cthth=out[2], cth=out[3],
                ct=complex(out[4], out[5]), c1=complex(out[6], out[7]),
                c0=complex(out[8], out[9]), d=complex(out[10], out[11]),
                r=out[12], Delta=out[13])


def layer_map(R, S, rho, kind="f64"):
    """Hyperboloidal layer map at grid position rho: (r*, rho', H, rho'')."""
    out = np.zeros(4)
    _lib(kind).or_layer_map(R, S, rho, _ptr(out))
    return tuple(out)


def layer_coeffs(M, a, s, m, R, S, rho, theta, kind="f64"):
    """Coefficients of the layer system at grid position rho and theta: dict
    with bo, bi (outgoing / ingoing speeds), cthth, cth, fw, complex ct, c0,
    d, and r, Delta."""
    out = np.zeros(13)
    _lib(kind).or_layer_coeffs(M, a, s, m, R, S, rho, theta, _ptr(out))
    return dict(bo=out[0], bi=out[1], cthth=out[2], cth=out[3], fw=out[4],
                ct=complex(out[5], out[6]), c0=complex(out[7], out[8]),
                d=complex(out[9], out[10]), r=out[11], Delta=out[12])


def orbit_omega(M, a, r0):
    return _lib().or_orbit_omega(M, a, r0)


def set_threads(n, kind="f64"):
    _lib(kind).or_set_threads(int(n))


def get_threads(kind="f64"):
    return _lib(kind).or_get_threads()


# source shapes: the smeared Gaussian and the two discrete delta functions
SOURCE_SHAPES = {"gaussian": 1, "step_delta": 2, "linear_delta": 3}


class Grid:
    """One oracle instance: a grid, its coefficient planes and the state."""

    def __init__(self, M=1.0, a=0.0, s=-2, m=2, n_r=101, n_theta=17,
                 rstar_min=-50.0, rstar_max=50.0, dt=0.1, i_obs=None,
                 extract_every=0, source=None, layer_R=0.0, kind="f64"):
        self.kind = kind
        self.lib = _lib(kind)
        if i_obs is None:
            i_obs = n_r // 2
        d = OrDesc()
        d.M, d.a, d.s, d.m = M, a, s, m
        d.n_r, d.n_theta = n_r, n_theta
        d.rstar_min, d.rstar_max, d.dt = rstar_min, rstar_max, dt
        d.i_obs, d.extract_every = int(i_obs), int(extract_every)
        d.layer_R = layer_R
        if source is not None:
            d.src_kind = SOURCE_SHAPES[source.get("shape", "gaussian")]
            d.src_r0 = source["r0"]
            d.src_amp = source.get("amplitude", 1.0)
            d.src_phase0 = source.get("phase0", 0.0)
            d.src_sigma_r_cells = source.get("sigma_r_cells", 2.0)
            d.src_sigma_th_cells = source.get("sigma_th_cells", 2.0)
            d.src_window_sigmas = source.get("window_sigmas", 6.0)
            d.src_t0 = source.get("t0", 0.0)
            d.src_ramp = source.get("ramp", 0.0)
        self.desc = d
        self.n_r, self.n_theta = n_r, n_theta
        self.h = (rstar_max - rstar_min) / (n_r - 1)
        self.dtheta = np.pi / (n_theta - 1)
        self.dt = dt
        self._h = self.lib.or_grid_new(ctypes.byref(d))
        if not self._h:
            raise ValueError("oracle rejected the grid description")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.lib.or_grid_free(h)
            self._h = None

    def set_state(self, phi, pi, step=0):
        phi = np.ascontiguousarray(phi, dtype=np.complex128).reshape(self.n_theta, self.n_r)
        pi = np.ascontiguousarray(pi, dtype=np.complex128).reshape(self.n_theta, self.n_r)
        self.lib.or_set_state(self._h, _ptr(phi.view(np.float64)), _ptr(pi.view(np.float64)), int(step))

    def get_state(self):
        phi = np.zeros((self.n_theta, self.n_r), np.complex128)
        pi = np.zeros((self.n_theta, self.n_r), np.complex128)
        self.lib.or_get_state(self._h, _ptr(phi.view(np.float64)), _ptr(pi.view(np.float64)))
        return phi, pi

    @property
    def step_index(self):
        return self.lib.or_get_step(self._h)

    def step(self, F_half=None, F_node=None):
        """One step.  F_half: (n_theta, n_r - 1) forcing at half nodes and t^n;
        F_node: (n_theta, n_r) forcing at nodes and t^n + dt/2."""
        fh = fn = None
        if F_half is not None:
            full = np.zeros((self.n_theta, self.n_r), np.complex128)
            full[:, : self.n_r - 1] = F_half
            fh = _ptr(full.view(np.float64))
        if F_node is not None:
            fnode = np.ascontiguousarray(F_node, dtype=np.complex128)
            fn = _ptr(fnode.view(np.float64))
        self.lib.or_step(self._h, fh, fn)

    def run(self, n_steps):
        return self.lib.or_run(self._h, int(n_steps))

    def waveform(self):
        """(n_samples, n_theta) complex samples of Phi at the extraction column."""
        n = self.lib.or_run(self._h, 0)
        out = np.zeros((max(n, 1), self.n_theta), np.complex128)
        got = self.lib.or_get_wave(self._h, _ptr(out.view(np.float64)), n)
        return out[:got]

    def radial(self):
        """(r*_q, x_q) for q = 0 .. 2 n_r - 2 (even q: node q/2, odd: half node)."""
        nq = 2 * self.n_r - 1
        rs = np.zeros(nq)
        x = np.zeros(nq)
        self.lib.or_get_radial(self._h, _ptr(rs), _ptr(x))
        return rs, x

    def rhs_column(self, q, phi_col, pi_col):
        """Pi-component of S at radial position q on one theta column."""
        phi_col = np.ascontiguousarray(phi_col, dtype=np.complex128)
        pi_col = np.ascontiguousarray(pi_col, dtype=np.complex128)
        out = np.zeros(self.n_theta, np.complex128)
        self.lib.or_rhs_column(self._h, int(q), _ptr(phi_col.view(np.float64)),
                               _ptr(pi_col.view(np.float64)), _ptr(out.view(np.float64)))
        return out

    def coeff_column(self, q):
        out = np.zeros((self.n_theta, 12))
        self.lib.or_get_coeff_column(self._h, int(q), _ptr(out))
        return dict(b=out[:, 0], cthth=out[:, 1], cth=out[:, 2],
                    ct=out[:, 3] + 1j * out[:, 4], c0=out[:, 5] + 1j * out[:, 6],
                    d=out[:, 7] + 1j * out[:, 8], bi=out[:, 9], fw=out[:, 10])

    def source_value(self, t, rstar, theta):
        out = np.zeros(2)
        self.lib.or_source_value(self._h, t, rstar, theta, _ptr(out))
        return complex(out[0], out[1])


def project(samples, basis, dtheta):
    """Project waveform samples (n_samples, n_theta) onto angular profiles
    basis (n_l, n_theta): w_l(t) = 2 pi sum_j Phi_j Y_l(theta_j) sin(theta_j) dtheta
    (trapezoid rule; the pole terms vanish because sin = 0 there)."""
    n_theta = samples.shape[1]
    th = np.arange(n_theta) * dtheta
    wts = 2 * np.pi * np.sin(th) * dtheta
    return samples @ (np.conj(basis) * wts).T
