"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle source (on the
CPU, in a temporary directory), builds it, and runs the pins against it: at
least one pin has to fail.  The real oracle is never modified.
"""
import importlib.util
import os
import shutil
import subprocess

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vrt_oracle.c")

MUTATIONS = {
    "gamma_minus_root": ("double gamma = -mu * c + sg * sqrt(D);",
                         "double gamma = -mu * c - sg * sqrt(D);"),
    "mu_inverted": ("double mu = n_last / ni; /* mu_i = n_{i-1} / n_i */",
                    "double mu = ni / n_last;"),
    "tir_step_uses_n_i": ("                    reflect(I, N, c, R);\n                    Delta = q->dL0 / n_last;",
                          "                    reflect(I, N, c, R);\n                    Delta = q->dL0 / ni;"),
    "reflection_factor": ("v[a] = I[a] - 2.0 * c * N[a];", "v[a] = I[a] - c * N[a];"),
    "step_times_n": ("                    snell(I, N, mu, c, D, R);\n                    Delta = q->dL0 / ni;",
                     "                    snell(I, N, mu, c, D, R);\n                    Delta = q->dL0 * ni;"),
    "grid_transposed": ("((size_t)k * m->ny + j) * m->nx + i", "((size_t)i * m->ny + j) * m->nx + k"),
    "gaussian_grad_sign": ("g[a] += -e * d[a] / (s * s);", "g[a] += e * d[a] / (s * s);"),
    "exit_mu_inverted": ("double mu = n_last / m->n_amb;", "double mu = m->n_amb / n_last;"),
    "entry_mu_inverted": ("double mu = m->n_amb / n_in;", "double mu = n_in / m->n_amb;"),
    "tangent_half_dropped": ("double h = dn / (2.0 * ni);", "double h = dn / ni;"),
    "critical_angle_acos": ("double th_c = asin(1.0 / mu);", "double th_c = acos(1.0 / mu);"),
    "no_n_last_update": ("        n_last = ni; /* P_i becomes the previous point of the next one */",
                         ""),
    "tir_condition_strict": ("                if (D <= 0.0) {\n                    /* case (v)",
                             "                if (D < -1e-9) {\n                    /* case (v)"),
    "luneburg_grad_factor": ("g[a] = -d[a] / (R * R * nv);", "g[a] = -d[a] / (R * nv);"),
    "fiber_grad_sign": ("double k = -2.0 * Dl * nc * nc / (R * R * nv);",
                        "double k = 2.0 * Dl * nc * nc / (R * R * nv);"),
    "box_exit_face_swapped": ("bf = R[a] > 0.0 ? a + 3 : a;", "bf = R[a] > 0.0 ? a : a + 3;"),
    "grid_interior_forward_difference": (
        "        lo[axis] = idx[axis] - 1;\n        hi[axis] = idx[axis] + 1;\n        span = 2.0 * h;",
        "        hi[axis] = idx[axis] + 1;\n        span = h;"),
    "tie_distance_along_ray": ("double dist = fabs(tx - Delta) * fabs(dot3(R, Ne));",
                               "double dist = fabs(tx - Delta);"),
    "grazing_window_mu_above_one": ("if (mu < 1.0 && fabs(c) < 10.0 * q->crit_rad) {",
                                    "if (mu > 1.0 && fabs(c) < 10.0 * q->crit_rad) {"),
}

PINS = [getattr(pins, n) for n in dir(pins) if n.startswith("test_")]


def _mutant(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/present"
    d = tmp_path / name
    d.mkdir()
    (d / "vrt_oracle.c").write_text(src.replace(old, new))
    shutil.copy(os.path.join(ROOT, "oracle", "vrt_oracle.h"), d / "vrt_oracle.h")
    so = d / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(so), str(d / "vrt_oracle.c"), "-lm"], check=True)
    spec = importlib.util.spec_from_file_location(f"oracle_mut_{name}",
                                                  os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._SRC = str(d / "vrt_oracle.c")
    mod._LIB_PATH = str(so)
    mod._lib = None
    return mod


def _run_pin(fn, orc):
    import inspect

    sig = inspect.signature(fn)
    if "medium" in sig.parameters:  # parametrized gradient pin
        for m in [{"kind": "luneburg", "params": pins.np.array([1.3, 0.1, -0.2, 0.05])},
                  {"kind": "fiber", "params": pins.np.array([1.38, 0.2, 5.0, 0.3, -0.1])},
                  pins.workloads.gaussian_medium(2)]:
            fn(orc, m)
    elif "orc" in sig.parameters:
        fn(orc)
    else:
        fn()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(tmp_path, name):
    orc = _mutant(tmp_path, name)
    caught = []
    for fn in PINS:
        try:
            _run_pin(fn, orc)
        except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError):
            caught.append(fn.__name__)
            break
    assert caught, f"no pin detects mutation {name}"
