"""CPU checks of the C ABI library: it loads, exports every entry point the
header declares, and its host-side logic (validation, stability bound) works
without a device.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_1206_0270_amd import tk
from paper_1206_0270_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tk.h")).read()
    return sorted(set(re.findall(r"^(?:tk_status|int|const char \*)\s*(tk_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = tk.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tk.EXPORTS)
    assert lib.tk_abi_version() == tk.ABI_VERSION == 5


def test_struct_layout_matches_header():
    # the ctypes mirrors must have the C sizes (x86-64 ABI)
    assert ctypes.sizeof(tk.InstanceDesc) == 88
    assert ctypes.sizeof(tk.SourceDesc) == 72
    assert ctypes.sizeof(tk.Tuning) == 24


def _init(insts):
    lib = tk.load()
    arr = (tk.InstanceDesc * len(insts))(*insts)
    ctx = ctypes.c_void_p()
    st = lib.tk_init_grid(arr, len(insts), tk.TK_FP64, None, ctypes.byref(ctx))
    return st, ctx


def test_init_validation_errors():
    good = W.schwarzschild_801x33()["instances"][0]
    lib = tk.load()
    for field, val in [("n_r", 3), ("a", 1.0), ("s", 3), ("dt", -1.0), ("rstar_obs", 1e9)]:
        d = tk.make_desc(good)
        setattr(d, field, val)
        st, ctx = _init([d])
        assert st == tk.TK_E_INVALID, field
        assert lib.tk_last_error(None)
    d = tk.make_desc(good)
    d.rstar_max = d.rstar_min
    assert _init([d])[0] == tk.TK_E_INVALID


def test_unstable_dt_rejected_unless_forced():
    inst = dict(W.schwarzschild_801x33()["instances"][0])
    inst["dt"] = 0.125  # dr*/2: above the angular stability bound
    st, ctx = _init([tk.make_desc(inst)])
    assert st == tk.TK_E_UNSTABLE
    assert b"stability" in tk.load().tk_last_error(None)
    st, ctx = _init([tk.make_desc(inst, force_dt=True)])
    assert st == tk.TK_OK
    lib = tk.load()
    n = ctypes.c_size_t()
    assert lib.tk_workspace_bytes(ctx, ctypes.byref(n)) == tk.TK_OK and n.value > 801 * 33 * 64
    # stepping (or tuning) without a bound workspace is a state error, not a crash
    assert lib.tk_step(ctx, 1) == tk.TK_E_STATE
    assert lib.tk_autotune(ctx, 2, 4, None, 0, None, None) == tk.TK_E_STATE
    assert lib.tk_destroy(ctx) == tk.TK_OK


@pytest.mark.parametrize("k", ["schwarzschild_801x33", "kerr_8001x129", "kerr_sourced_16001x257",
                               "six_modes_16001x129"])
def test_workload_dts_are_below_library_bound(k):
    for inst in W.WORKLOADS[k]()["instances"]:
        bound = tk.stable_dt(inst)
        assert inst["dt"] <= bound * (1 + 1e-12), (inst["name"], inst["dt"], bound)


def test_batched_workload_dts_are_below_library_bound():
    for inst in W.batched_40_uneven()["instances"]:
        assert inst["dt"] <= tk.stable_dt(inst) * (1 + 1e-12), inst["name"]


def test_tuning_validation():
    inst = W.schwarzschild_801x33()["instances"][0]
    st, ctx = _init([tk.make_desc(inst)])
    assert st == tk.TK_OK
    lib = tk.load()
    for bad in (tk.Tuning(7, 0, 0, 0, 0, 0), tk.Tuning(tk.TK_KERNEL_FUSED, 2, 0, 0, 0, 0),
                tk.Tuning(tk.TK_KERNEL_FUSED, 0, 0, 2, 0, 0), tk.Tuning(tk.TK_KERNEL_FUSED, 0, 0, 3, 8, 0),
                tk.Tuning(tk.TK_KERNEL_FUSED, 0, 0, 1, 1, 4), tk.Tuning(tk.TK_KERNEL_FUSED2, 3, 0, 3, 1, 0),
                tk.Tuning(tk.TK_KERNEL_FUSED, 0, 0, 3, tk.TK_TUNE_NT_STORES, 4),
                tk.Tuning(tk.TK_KERNEL_FUSED2, 0, 0, 3, tk.TK_TUNE_NT_STORES, 3),
                tk.Tuning(tk.TK_KERNEL_TILED, 0, 0, 3, 1, 0), tk.Tuning(tk.TK_KERNEL_TILED, 6, 0, 3, 1, 0),
                tk.Tuning(5, 0, 0, 3, 1, 0)):
        assert lib.tk_set_tuning(ctx, ctypes.byref(bad)) == tk.TK_E_INVALID
    # this context is on the NULL stream, which cannot be captured: graphs are refused there
    for kern in (tk.TK_KERNEL_TWO_PASS, tk.TK_KERNEL_FUSED, tk.TK_KERNEL_FUSED2):
        bad = tk.Tuning(kern, 0, 50, 1, tk.TK_TUNE_NT_STORES, 0)
        assert lib.tk_set_tuning(ctx, ctypes.byref(bad)) == tk.TK_E_INVALID
        assert b"NULL stream" in lib.tk_last_error(ctx)
    ok = tk.Tuning(tk.TK_KERNEL_TWO_PASS, 8, 0, 1, tk.TK_TUNE_NT_STORES, 0)
    assert lib.tk_set_tuning(ctx, ctypes.byref(ok)) == tk.TK_OK
    got = tk.Tuning()
    assert lib.tk_get_tuning(ctx, ctypes.byref(got)) == tk.TK_OK
    assert (got.kernel, got.rows_per_tile, got.graph_steps, got.prefetch_rows, got.flags) == (1, 8, 0, 1, 1)
    ok = tk.Tuning(tk.TK_KERNEL_FUSED, 0, 0, 3, 0, 0)
    assert lib.tk_set_tuning(ctx, ctypes.byref(ok)) == tk.TK_OK
    ok = tk.Tuning(tk.TK_KERNEL_FUSED2, 0, 0, 1, tk.TK_TUNE_NT_STORES, 0)
    assert lib.tk_set_tuning(ctx, ctypes.byref(ok)) == tk.TK_OK
    for rows in (4, 8):
        ok = tk.Tuning(tk.TK_KERNEL_TILED, rows, 0, 3, 0, 0)
        assert lib.tk_set_tuning(ctx, ctypes.byref(ok)) == tk.TK_OK
    for rows in (4, 16):
        ok = tk.Tuning(tk.TK_KERNEL_FUSED2, rows, 0, 1, 0, 0)
        assert lib.tk_set_tuning(ctx, ctypes.byref(ok)) == tk.TK_OK
    lib.tk_destroy(ctx)


C_PROGRAM = r"""
#include "tk.h"
#include <stdio.h>
int main(void)
{
    tk_instance_desc d = {1.0, 0.5, -2, 2, 101, 9, -20.0, 25.0, 0.0, 20.0, 3, 0, 0, 0.0};
    double dt = 0.0, w[6] = {1, 0, 2, 0, 3, 0}, e[2], err[1];
    tk_ctx *ctx = NULL;
    size_t bytes = 0;
    if (tk_abi_version() != TK_ABI_VERSION) return 1;
    if (tk_stable_dt(&d, &dt) != TK_OK || !(dt > 0)) return 2;
    d.dt = dt;
    if (tk_init_grid(&d, 1, TK_FP64, NULL, &ctx) != TK_OK) return 3;
    if (tk_workspace_bytes(ctx, &bytes) != TK_OK || bytes == 0) return 4;
    if (tk_step(ctx, 1) != TK_E_STATE) return 5; /* no workspace bound yet */
    if (tk_destroy(ctx) != TK_OK) return 6;
    if (tk_richardson(w, w + 2, w + 4, 1, 2, e, err) != TK_OK) return 7;
    printf("%.17g %.17g\n", dt, e[0]);
    return 0;
}
"""


def test_abi_from_plain_c(tmp_path):
    # the header is C, and a C program links libtk.so and calls it (host-side
    # entry points only: no device here)
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    lib_dir = os.path.dirname(tk.LIB_PATH)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe), "-L", lib_dir, "-ltk", "-Wl,-rpath," + lib_dir], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    dt = float(out[0])
    same = W.instance(a=0.5, m=2, n_r=101, n_theta=9, rstar_min=-20.0, rstar_max=25.0, rstar_obs=20.0)
    assert dt == tk.stable_dt(same)
    assert float(out[1]) == pytest.approx(10.0 / 3.0)


def test_binding_refuses_without_the_library(monkeypatch, tmp_path):
    # no CPU fallback: without libtk.so the binding raises instead of
    # computing anything
    monkeypatch.setattr(tk, "_lib", None)
    monkeypatch.setattr(tk, "LIB_PATH", str(tmp_path / "libtk.so"))
    with pytest.raises(RuntimeError, match="missing"):
        tk.load()


def test_stepper_refuses_without_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is visible here")
    inst = W.schwarzschild_801x33()["instances"][0]
    with pytest.raises(RuntimeError, match="no HIP device"):
        tk.Stepper([inst])


def test_layer_descriptions_are_validated():
    """Hyperboloidal layer: accepted on the s = -2 field, in FP64 and in the
    FP32-compensated form, with the layer inside the grid; every other
    description is refused at init."""
    base = W.instance(a=0.5, m=2, n_r=201, n_theta=17, rstar_min=-40.0, rstar_max=50.0, layer_start=30.0)
    assert base["i_obs"] == 200  # the waveform is read at null infinity by default
    lib = tk.load()
    st, ctx = _init([tk.make_desc(base)])
    assert st == tk.TK_OK
    lib.tk_destroy(ctx)
    for change in (dict(layer_start=50.0), dict(layer_start=49.9), dict(layer_start=-10.0),
                   dict(layer_start=float("nan")), dict(s=-1)):
        inst = dict(base)
        inst.update(change)
        st, ctx = _init([tk.make_desc(inst)])
        assert st == tk.TK_E_INVALID, change
    arr = (tk.InstanceDesc * 1)(tk.make_desc(base))
    ctx = ctypes.c_void_p()
    assert lib.tk_init_grid(arr, 1, tk.TK_FP32_COMP, None, ctypes.byref(ctx)) == tk.TK_OK
    lib.tk_destroy(ctx)
