"""The oracle's pins are sharp enough: each plausible mistake planted in a
copy of the oracle source (a dropped term, a wrong sign, a wrong index or
time level, a first-order pole condition, a misplaced or mis-scaled discrete
delta) makes at least one pin fail.

Each mutant is compiled from an edited copy of oracle/teuk_oracle.c into a
temporary library; the committed oracle is never modified.
"""
import os
import tempfile

import pytest

import oracle
from oracle import build as orbuild

import test_layer as LAYER
import test_oracle_pins as PINS
import test_segments as SEGS
import test_source_shapes as SHAPES

# (name, original text (must occur exactly once), replacement, pins to run)
MUTANTS = [
    ("c0 drops 4 i m s a (r-M)", "4 * IU * m * s * a * (r - M) - Delta * Vth",
     "0 * IU * m * s * a * (r - M) - Delta * Vth", ["mms_even"]),
    ("ct sign of i a Delta cos", "+ IU * a * Delta * cs)) / Sh2", "- IU * a * Delta * cs)) / Sh2",
     ["mms_even"]),
    ("d misses the b ct term", "c.d = -(c.c1 - c.b * c.bp - c.b * c.ct);", "c.d = -(c.c1 - c.b * c.bp);",
     ["mms_even"]),
    ("b' misses a^2", "c.bp = (Delta / rho) * a * a * sn2", "c.bp = (Delta / rho) * a * sn2",
     ["mms_even", "principal"]),
    ("cot term sign", "c.cth = c.cthth * cs / sn;", "c.cth = -c.cthth * cs / sn;", ["eig"]),
    ("first-order pole condition", "return (4 * x1 - x2) / 3;", "return x1;", ["eig", "mms_even"]),
    ("advection sign on Pi", "cplx adv_pi = (g->d[c] * dphi - g->bi[c] * dpi) / h;\n            g->hphi",
     "cplx adv_pi = (g->d[c] * dphi + g->bi[c] * dpi) / h;\n            g->hphi", ["mms_even"]),
    ("source at t^n in the second step", "F = source_at(g, th_half, g->rstar[q], th);",
     "F = source_at(g, tn, g->rstar[q], th);", ["source"]),
    ("forcing of Eq. (4) taken one node off",
     "F = F_node[2 * IDX(g, j, i)] + IU * F_node[2 * IDX(g, j, i) + 1];",
     "F = F_node[2 * IDX(g, j, i - 1)] + IU * F_node[2 * IDX(g, j, i - 1) + 1];", ["mms_even"]),
    ("angular stencil uses row j twice", "(phip - 2 * phi0 + phim)", "(phip - 2 * phi0 + phi0)", ["eig"]),
    ("c1 misses 2 r Delta", "2 * s * (r - M) * rho + 2 * r * Delta + 2 * IU", "2 * s * (r - M) * rho + 2 * IU",
     ["mms_odd"]),
    ("tortoise: r- weight with the wrong sign", "val -= k->Am * log(", "val += k->Am * log(", ["tortoise"]),
    ("step delta: value 1 at the jump", "        return 0;\n    return (real)0.5;", "        return 0;\n    return 1;",
     ["delta_theta"]),
    ("step delta: forward difference",
     "(heaviside(x + dx - xp, dx) - heaviside(x - dx - xp, dx)) / (2 * dx)",
     "(heaviside(x + dx - xp, dx) - heaviside(x - xp, dx)) / dx", ["delta_step"]),
    ("linear delta: ramp over the cell above the particle", "real v = y / dx + 1;", "real v = y / dx;",
     ["delta_linear"]),
    ("radial delta on half the spacing", "discrete_delta(d->src_kind, rstar, g->src_rstar_p, g->h);",
     "discrete_delta(d->src_kind, rstar, g->src_rstar_p, g->h / 2);", ["delta_linear", "delta_step"]),
    ("theta delta takes the radial spacing", "discrete_delta(d->src_kind, th, PI_R / 2, g->dth);",
     "discrete_delta(d->src_kind, th, PI_R / 2, g->h);", ["delta_theta"]),
    ("switch-on not mirrored", "real a = bump_tail(x), b = bump_tail(1 - x);",
     "real a = bump_tail(x), b = bump_tail(x);", ["switch_on"]),
    ("switch-on counted from the orbit's origin", "switch_on(t / (real)d->src_ramp)",
     "switch_on((t + (real)d->src_t0) / (real)d->src_ramp)", ["switch_on"]),
    ("layer ct drops the d H term", "o.ct = (c.ct * w + c.d * L->H + c.b", "o.ct = (c.ct * w + c.b", ["layer_eq"]),
    ("layer ingoing speed over w", "o.bi = c.b * L->rhop / v;", "o.bi = c.b * L->rhop / w;", ["layer_eq"]),
    ("layer w without 1 - b", "real w = L->rhop * c.b + one_minus_b;", "real w = L->rhop * c.b;", ["layer_eq"]),
    ("layer rho'' sign", "L.rhopp = (2 * Om * Om1 * q + Om * Om * rho * Om2)",
     "L.rhopp = (2 * Om * Om1 * q - Om * Om * rho * Om2)", ["layer_map"]),
    ("scri node held at zero", "g->nphi[IDX(g, j, nr - 1)] = 2 * g->nphi[IDX(g, j, nr - 2)] - g->nphi[IDX(g, j, nr - 3)];",
     "g->nphi[IDX(g, j, nr - 1)] = 0;", ["layer_dyn"]),
]


def run_pin(name, kind):
    if name == "mms_even":
        PINS.mms_check(0.9, 2, kind=kind, levels=((201, 17), (401, 33)))
    elif name == "mms_odd":
        PINS.mms_check(0.6, 3, kind=kind, levels=((201, 17), (401, 33)))
    elif name == "eig":
        for m in (2, 1):
            PINS.angular_eigen_check(m, kind=kind)
    elif name == "tortoise":
        for a in (0.3, 0.9):
            rp, rm = PINS.horizons(1.0, a)
            for x in (0.1, 1.0, 7.0):
                got = oracle.tortoise(1.0, a, x, kind=kind)
                want = PINS.tortoise_closed(1.0, a, rp + x, x=x)
                assert abs(got - want) <= 1e-13 * max(1.0, abs(want))
    elif name == "principal":
        PINS.principal_part_check(kind=kind)
    elif name == "source":
        PINS.source_consistency_check(kind=kind)
    elif name == "delta_linear":
        for q0 in (0, 1):
            SHAPES.linear_delta_check(9.01, q0, kind=kind)
    elif name == "delta_step":
        for q0 in (0, 1):
            SHAPES.step_delta_check(q0, kind=kind)
    elif name == "switch_on":
        SEGS.switch_on_check(kind=kind)
    elif name == "layer_eq":
        LAYER.eq1_check(0.9, 2, kind=kind)
    elif name == "layer_map":
        for rho in LAYER.MAP_POINTS:
            LAYER.map_check(rho, kind=kind)
    elif name == "layer_dyn":
        LAYER.interior_check(0.5, 2, kind=kind)
        LAYER.decay_check(kind=kind)
    elif name == "delta_theta":
        for case in SHAPES.THETA_CASES:
            SHAPES.theta_delta_check(*case, kind=kind)
    else:
        raise KeyError(name)


@pytest.fixture(scope="module")
def src_text():
    with open(orbuild.SRC) as f:
        return f.read()


def test_unmutated_source_passes_the_detectors(src_text):
    for pin in ("mms_even", "mms_odd", "eig", "tortoise", "source", "delta_linear", "delta_step", "delta_theta",
                "switch_on", "layer_eq", "layer_map", "layer_dyn"):
        run_pin(pin, "f64")


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(src_text, tmp_path, name, old, new, pins):
    assert src_text.count(old) == 1, f"mutation anchor not unique: {old!r}"
    path = os.path.join(str(tmp_path), "mutant.c")
    with open(path, "w") as f:
        f.write(src_text.replace(old, new))
    lib = os.path.join(str(tmp_path), "libmutant.so")
    orbuild.build_one(path, lib)
    caught = []
    for pin in pins:
        try:
            run_pin(pin, lib)
        except AssertionError as e:
            caught.append((pin, str(e)[:120]))
    assert caught, f"mutant '{name}' passed {pins}"
