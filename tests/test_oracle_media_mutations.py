"""The pins of the later media must catch plausible mistakes in them.

As test_oracle_mutations.py, for the spherical freeform medium (Eq. (26)),
the N2P lens (Eq. (27)) and the Zernike-Legendre lens of Sec. V: each case
plants one mistake in a private copy of the oracle source (on the CPU, in a
temporary directory), builds it, and runs the pins of those media
(test_oracle_design_pins.py, test_oracle_zernike_pins.py) against it; at
least one has to fail.  The real oracle is never modified.
"""
import inspect
import itertools

import pytest

import test_oracle_design_pins as design_pins
import test_oracle_zernike_pins as zernike_pins
from test_oracle_mutations import _mutant, MUTATIONS as BASE_MUTATIONS

MUTATIONS = {
    # spherical medium
    "sph_G1_factor": ("double G1 = 0.3 * (r * r - 1.0);", "double G1 = 0.3 * (r * r + 1.0);"),
    "sph_G2_order": ("double G2 = r * cos(5.0 * th);", "double G2 = r * cos(3.0 * th);"),
    "sph_G3_phi": ("double G3 = r * r * st * st * cos(2.0 * ph);",
                   "double G3 = r * r * st * st * sin(2.0 * ph);"),
    "sph_theta_sign": ("double et[3] = {ct * cp, ct * sp, -st};",
                       "double et[3] = {ct * cp, ct * sp, st};"),
    # N2P lens
    "n2p_rho_not_halved": ("double w = (R * R - (rho / 2.0) * (rho / 2.0)) / (F * F);",
                           "double w = (R * R - rho * rho) / (F * F);"),
    "n2p_exponents_swapped": ("double u = 1.0 + pow(w, be);\n        *n = pow(u, ga);",
                              "double u = 1.0 + pow(w, ga);\n        *n = pow(u, be);"),
    "n2p_slope_factor": ("* (-rho / (2.0 * F * F));", "* (-rho / (F * F));"),
    # Zernike-Legendre lens
    "zern_term8_cosine": ("{3, 1, 0}, {3, 1, 1}, {4, 0, 0}", "{3, 1, 0}, {3, 1, 0}, {4, 0, 0}"),
    "zern_radial_sign": ("double c = ((k % 2) ? -1.0 : 1.0) * fact(n - k) /",
                         "double c = fact(n - k) /"),
    "zern_polar_gradient_sign": ("double Zu = dR * ct * T - Rr * dT * st;",
                                 "double Zu = dR * ct * T + Rr * dT * st;"),
    "zern_axial_scale": ("double u = P[0] / rm, v = P[1] / rm, w = 2.0 * P[2] / zm - 1.0;",
                         "double u = P[0] / rm, v = P[1] / rm, w = P[2] / zm - 1.0;"),
    "zern_axial_chain_factor": ("g[2] += dn * c * Z * dV * 2.0 / zm;",
                                "g[2] += dn * c * Z * dV / zm;"),
    "zern_legendre_recursion": ("double p2 = ((2 * k + 1) * w * p1 - k * p0) / (k + 1);",
                                "double p2 = ((2 * k + 1) * w * p1 + k * p0) / (k + 1);"),
    "zern_half_contrast": ("double n0 = 0.5 * (nhi + nlo), dn = 0.5 * (nhi - nlo);",
                           "double n0 = 0.5 * (nhi + nlo), dn = nhi - nlo;"),
}

PINS = ([getattr(design_pins, n) for n in dir(design_pins) if n.startswith("test_")] +
        [getattr(zernike_pins, n) for n in dir(zernike_pins) if n.startswith("test_")])
SLOW = {"test_oracle_design_loop_reproduces_the_paper",
        "test_paper_design_pairs_focus_and_settle_the_gamma_order"}


def _calls(fn):
    """Every parameter combination of a pin's parametrize marks."""
    marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
    axes = []
    for m in marks:
        names = [s.strip() for s in m.args[0].split(",")]
        vals = [v if len(names) > 1 else (v,) for v in m.args[1]]
        axes.append([dict(zip(names, v)) for v in vals])
    for combo in itertools.product(*axes):
        kw = {}
        for d in combo:
            kw.update(d)
        yield kw


def _run_pin(fn, orc, tmp_path):
    params = inspect.signature(fn).parameters
    for kw in _calls(fn):
        if "orc" in params:
            kw["orc"] = orc
        if "tmp_path" in params:
            kw["tmp_path"] = tmp_path
        fn(**kw)


def test_mutations_are_new_and_anchored():
    import os

    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "oracle", "vrt_oracle.c")).read()
    for name, (old, _) in MUTATIONS.items():
        assert name not in BASE_MUTATIONS
        assert src.count(old) == 1, name


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_media_pins_catch_planted_mistake(tmp_path, monkeypatch, name):
    import test_oracle_mutations as base

    monkeypatch.setitem(base.MUTATIONS, name, MUTATIONS[name])
    orc = _mutant(tmp_path, name)
    caught = []
    for fn in PINS:
        if fn.__name__ in SLOW:
            continue
        try:
            _run_pin(fn, orc, tmp_path)
        except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError):
            caught.append(fn.__name__)
            break
    assert caught, f"no pin detects mutation {name}"
