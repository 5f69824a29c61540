"""Python binding of libtk.so (the C ABI in include/tk.h).

Argument marshalling only: every step of the time stepper runs in the HIP
kernels behind the C ABI.  PyTorch supplies the device memory (the
workspace and the autotuner's save area, uint8 tensors on the current HIP
device) and the stream: by default each Stepper gets a torch stream of its
own, because the NULL stream cannot be captured into HIP graphs.  There is
no fallback: if libtk.so is missing or no HIP device is visible, calls
raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtk.so")

TK_OK, TK_E_INVALID, TK_E_NOMEM, TK_E_DEVICE, TK_E_STATE, TK_E_UNSTABLE, TK_E_NONFINITE = range(7)
TK_FP64, TK_FP32_COMP = 0, 1
TK_FLAG_FORCE_DT = 1
TK_SRC_NONE, TK_SRC_CIRCULAR_GAUSSIAN, TK_SRC_CIRCULAR_STEP_DELTA, TK_SRC_CIRCULAR_LINEAR_DELTA = 0, 1, 2, 3
SOURCE_KINDS = {"gaussian": TK_SRC_CIRCULAR_GAUSSIAN, "step_delta": TK_SRC_CIRCULAR_STEP_DELTA,
                "linear_delta": TK_SRC_CIRCULAR_LINEAR_DELTA}
TK_KERNEL_AUTO, TK_KERNEL_TWO_PASS, TK_KERNEL_FUSED, TK_KERNEL_FUSED2, TK_KERNEL_TILED = 0, 1, 2, 3, 4

_STATUS = {0: "TK_OK", 1: "TK_E_INVALID", 2: "TK_E_NOMEM", 3: "TK_E_DEVICE", 4: "TK_E_STATE",
           5: "TK_E_UNSTABLE", 6: "TK_E_NONFINITE"}

EXPORTS = ["tk_abi_version", "tk_init_grid", "tk_workspace_bytes", "tk_bind_workspace",
           "tk_set_fields", "tk_get_fields", "tk_set_source", "tk_step", "tk_prepare", "tk_get_counters",
           "tk_extract", "tk_get_step", "tk_set_step", "tk_set_tuning", "tk_get_tuning", "tk_autotune_bytes",
           "tk_autotune", "tk_autotune_static", "tk_synchronize", "tk_destroy", "tk_last_error", "tk_stable_dt",
           "tk_richardson"]
ABI_VERSION = 5
AUTOTUNE_STATIC_MAX_BYTES = 64 << 20


class TkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class InstanceDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("a", ctypes.c_double),
                ("s", ctypes.c_int), ("m", ctypes.c_int),
                ("n_r", ctypes.c_int), ("n_theta", ctypes.c_int),
                ("rstar_min", ctypes.c_double), ("rstar_max", ctypes.c_double),
                ("dt", ctypes.c_double), ("rstar_obs", ctypes.c_double),
                ("extract_every", ctypes.c_int), ("wave_capacity", ctypes.c_int),
                ("flags", ctypes.c_int), ("layer_start", ctypes.c_double)]


class SourceDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("r0", ctypes.c_double), ("amplitude", ctypes.c_double),
                ("phase0", ctypes.c_double), ("sigma_r_cells", ctypes.c_double),
                ("sigma_th_cells", ctypes.c_double), ("window_sigmas", ctypes.c_double),
                ("t0", ctypes.c_double), ("ramp", ctypes.c_double)]


TK_TUNE_NT_STORES = 1


class Counters(ctypes.Structure):
    _fields_ = [("graphs_instantiated", ctypes.c_long), ("graph_launches", ctypes.c_long),
                ("eager_launches", ctypes.c_long)]


class Tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("rows_per_tile", ctypes.c_int),
                ("graph_steps", ctypes.c_int), ("prefetch_rows", ctypes.c_int),
                ("flags", ctypes.c_int), ("waves_per_simd", ctypes.c_int)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def load():
    """Load libtk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    if lib.tk_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {lib.tk_abi_version()}, the binding {ABI_VERSION}: rebuild it")
    vp, st = ctypes.c_void_p, ctypes.c_int
    sig = {
        "tk_abi_version": (ctypes.c_int, []),
        "tk_init_grid": (st, [ctypes.POINTER(InstanceDesc), ctypes.c_int, ctypes.c_int, vp,
                              ctypes.POINTER(vp)]),
        "tk_workspace_bytes": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "tk_bind_workspace": (st, [vp, vp, ctypes.c_size_t]),
        "tk_set_fields": (st, [vp, ctypes.c_int, _dp, _dp]),
        "tk_get_fields": (st, [vp, ctypes.c_int, _dp, _dp]),
        "tk_set_source": (st, [vp, ctypes.c_int, ctypes.POINTER(SourceDesc)]),
        "tk_step": (st, [vp, ctypes.c_long]),
        "tk_prepare": (st, [vp, ctypes.c_long]),
        "tk_get_counters": (st, [vp, ctypes.POINTER(Counters)]),
        "tk_extract": (st, [vp, ctypes.c_int, _dp, ctypes.c_long, ctypes.POINTER(ctypes.c_long)]),
        "tk_get_step": (st, [vp, ctypes.POINTER(ctypes.c_long)]),
        "tk_set_step": (st, [vp, ctypes.c_long]),
        "tk_set_tuning": (st, [vp, ctypes.POINTER(Tuning)]),
        "tk_get_tuning": (st, [vp, ctypes.POINTER(Tuning)]),
        "tk_autotune_bytes": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "tk_autotune": (st, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, _dp,
                             ctypes.POINTER(ctypes.c_int)]),
        "tk_autotune_static": (st, [vp, ctypes.c_int, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int)]),
        "tk_synchronize": (st, [vp]),
        "tk_destroy": (st, [vp]),
        "tk_last_error": (ctypes.c_char_p, [vp]),
        "tk_stable_dt": (st, [ctypes.POINTER(InstanceDesc), _dp]),
        "tk_richardson": (st, [_dp, _dp, _dp, ctypes.c_long, ctypes.c_int, _dp, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status, ctx=None):
    if status != TK_OK:
        msg = load().tk_last_error(ctx)
        raise TkError(status, msg.decode() if msg else "")


def make_desc(inst, force_dt=False, wave_capacity=0):
    """tk_instance_desc from a workload dict (see workloads.instance)."""
    d = InstanceDesc()
    d.M, d.a, d.s, d.m = inst["M"], inst["a"], inst["s"], inst["m"]
    d.n_r, d.n_theta = inst["n_r"], inst["n_theta"]
    d.rstar_min, d.rstar_max, d.dt = inst["rstar_min"], inst["rstar_max"], inst["dt"]
    d.rstar_obs = inst["rstar_obs"]
    d.extract_every = inst.get("extract_every", 0) or 0
    d.wave_capacity = wave_capacity
    d.flags = TK_FLAG_FORCE_DT if force_dt else 0
    d.layer_start = inst.get("layer_start", 0.0) or 0.0
    return d


def make_source(src):
    s = SourceDesc()
    if src is None:
        s.kind = TK_SRC_NONE
        return s
    s.kind = SOURCE_KINDS[src.get("shape", "gaussian")]
    s.r0 = src["r0"]
    s.amplitude = src.get("amplitude", 1.0)
    s.phase0 = src.get("phase0", 0.0)
    s.sigma_r_cells = src.get("sigma_r_cells", 2.0)
    s.sigma_th_cells = src.get("sigma_th_cells", 2.0)
    s.window_sigmas = src.get("window_sigmas", 6.0)
    s.t0 = src.get("t0", 0.0)
    s.ramp = src.get("ramp", 0.0)
    return s


def stable_dt(inst):
    out = ctypes.c_double()
    _check(load().tk_stable_dt(ctypes.byref(make_desc(inst)), ctypes.byref(out)))
    return out.value


def richardson(w1, w2, w3, order=2):
    """Richardson extrapolant of three results at spacings 1, 1/2, 1/4 and
    the error estimate from two extrapolants (tk_richardson).  Returns
    (extrapolated array, relative error array), shaped like the inputs."""
    arrs = [np.ascontiguousarray(w, dtype=np.complex128) for w in (w1, w2, w3)]
    if not (arrs[0].shape == arrs[1].shape == arrs[2].shape):
        raise ValueError("the three results must have one shape")
    n = arrs[0].size
    ext = np.zeros(arrs[0].shape, np.complex128)
    err = np.zeros(arrs[0].shape, np.float64)
    ptr = [a.view(np.float64).ctypes.data_as(_dp) for a in arrs]
    _check(load().tk_richardson(ptr[0], ptr[1], ptr[2], n, int(order), ext.view(np.float64).ctypes.data_as(_dp),
                                err.ctypes.data_as(_dp)))
    return ext, err


class Stepper:
    """A context over one or more instances, with its workspace in a torch
    tensor on the current HIP device.  Work goes on `stream` if given, else
    on a new torch stream of default priority owned by the Stepper."""

    def __init__(self, instances, precision=TK_FP64, force_dt=False, wave_capacity=0,
                 stream=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the stepper has no CPU path")
        lib = load()
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.instances = list(instances)
        self.n_inst = len(self.instances)
        self.wave_capacity = wave_capacity if wave_capacity > 0 else 4096  # the library's default
        descs = (InstanceDesc * self.n_inst)(*[make_desc(i, force_dt, wave_capacity)
                                               for i in self.instances])
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream()
        ctx = ctypes.c_void_p()
        _check(lib.tk_init_grid(descs, self.n_inst, precision, ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(ctx)))
        self.ctx = ctx
        self.lib = lib
        nbytes = ctypes.c_size_t()
        _check(lib.tk_workspace_bytes(ctx, ctypes.byref(nbytes)), ctx)
        self.workspace_bytes = nbytes.value
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        # the tensor is allocated on torch's current stream and used on self.stream
        torch.cuda.current_stream(self.device).synchronize()
        self.workspace.record_stream(self.stream)
        _check(lib.tk_bind_workspace(ctx, ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value), ctx)
        for k, inst in enumerate(self.instances):
            if inst.get("source") is not None:
                self.set_source(k, inst["source"])

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self, k):
        return self.instances[k]["n_theta"], self.instances[k]["n_r"]

    def set_fields(self, k, phi, pi):
        shp = self._shape(k)
        phi = np.ascontiguousarray(phi, dtype=np.complex128).reshape(shp)
        pi = np.ascontiguousarray(pi, dtype=np.complex128).reshape(shp)
        _check(self.lib.tk_set_fields(self.ctx, k, phi.view(np.float64).ctypes.data_as(_dp),
                                      pi.view(np.float64).ctypes.data_as(_dp)), self.ctx)

    def get_fields(self, k):
        shp = self._shape(k)
        phi = np.zeros(shp, np.complex128)
        pi = np.zeros(shp, np.complex128)
        _check(self.lib.tk_get_fields(self.ctx, k, phi.view(np.float64).ctypes.data_as(_dp),
                                      pi.view(np.float64).ctypes.data_as(_dp)), self.ctx)
        return phi, pi

    def set_source(self, k, src):
        _check(self.lib.tk_set_source(self.ctx, k, ctypes.byref(make_source(src))), self.ctx)

    def step(self, n):
        _check(self.lib.tk_step(self.ctx, int(n)), self.ctx)

    def prepare(self, n):
        """Host-side work of a later step(n) done now: work list, and the HIP
        graph if graph_steps > 0 and n >= graph_steps."""
        _check(self.lib.tk_prepare(self.ctx, int(n)), self.ctx)

    def counters(self):
        c = Counters()
        _check(self.lib.tk_get_counters(self.ctx, ctypes.byref(c)), self.ctx)
        return dict(graphs_instantiated=c.graphs_instantiated, graph_launches=c.graph_launches,
                    eager_launches=c.eager_launches)

    def extract(self, k, max_samples=1 << 20):
        nth = self.instances[k]["n_theta"]
        n = ctypes.c_long()
        cap = min(int(max_samples), self.wave_capacity)  # more than the ring holds is an overrun
        out = np.zeros((max(cap, 1), nth), np.complex128)
        st = self.lib.tk_extract(self.ctx, k, out.view(np.float64).ctypes.data_as(_dp), cap,
                                 ctypes.byref(n))
        _check(st, self.ctx)
        return out[: n.value]

    @property
    def step_index(self):
        v = ctypes.c_long()
        _check(self.lib.tk_get_step(self.ctx, ctypes.byref(v)), self.ctx)
        return v.value

    def set_step(self, n):
        _check(self.lib.tk_set_step(self.ctx, int(n)), self.ctx)

    def set_tuning(self, kernel=TK_KERNEL_AUTO, rows_per_tile=0, graph_steps=0, prefetch_rows=0,
                   nt_stores=True, waves_per_simd=0):
        t = Tuning(kernel, rows_per_tile, graph_steps, prefetch_rows,
                   TK_TUNE_NT_STORES if nt_stores else 0, waves_per_simd)
        _check(self.lib.tk_set_tuning(self.ctx, ctypes.byref(t)), self.ctx)

    def get_tuning(self):
        t = Tuning()
        _check(self.lib.tk_get_tuning(self.ctx, ctypes.byref(t)), self.ctx)
        return dict(kernel=t.kernel, rows_per_tile=t.rows_per_tile, graph_steps=t.graph_steps,
                    prefetch_rows=t.prefetch_rows, nt_stores=bool(t.flags & TK_TUNE_NT_STORES),
                    waves_per_simd=t.waves_per_simd)

    def autotune(self, warmup=2, steps=10):
        """Time the compiled launch shapes on these instances, keep the
        fastest; the simulation state is left as it was.  Returns
        (ms per step of the winner, shapes tried)."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        nbytes = ctypes.c_size_t()
        _check(self.lib.tk_autotune_bytes(self.ctx, ctypes.byref(nbytes)), self.ctx)
        torch = self.torch
        save = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        try:
            _check(self.lib.tk_autotune(self.ctx, int(warmup), int(steps), ctypes.c_void_p(save.data_ptr()),
                                        nbytes.value, ctypes.byref(ms), ctypes.byref(n)), self.ctx)
        finally:
            del save  # tk_autotune is synchronous: the area is free again
        return ms.value, n.value

    def autotune_static(self, warmup=2, steps=10):
        """autotune() with the library's static scratch area as the save
        area (no device memory is allocated for the call); TkError with
        TK_E_NOMEM if the state is larger than that area."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        torch = self.torch
        torch.cuda.current_stream(self.device).synchronize()
        _check(self.lib.tk_autotune_static(self.ctx, int(warmup), int(steps), ctypes.byref(ms), ctypes.byref(n)),
               self.ctx)
        return ms.value, n.value

    def synchronize(self):
        _check(self.lib.tk_synchronize(self.ctx), self.ctx)
