"""Pins of the FP64 oracle against things the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each checks it against an
independent closed form (scalar Snell geometry, unfolded mirror paths, the
catenary of a linear medium, the Luneburg focus), an exact discrete invariant
of the vectorial law, the paper's own worked example (Sec. IV helix), an
independent ODE integration of the ray equation, or a twin medium that must
give the same march.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def P(dL0, max_steps=200000, **kw):
    return workloads.trace_params(dL0, max_steps, **kw)


def homogeneous(n, boundary, n_amb=1.0):
    return {"kind": "homogeneous", "params": np.array([n]), "boundary": boundary, "n_amb": n_amb}


def sphere(r=1.0, c=(0, 0, 0)):
    return {"kind": "sphere", "params": np.array([c[0], c[1], c[2], r], dtype=float)}


def box(lo, hi):
    return {"kind": "box", "params": np.array(list(lo) + list(hi), dtype=float)}


def scalar_snell(d, N, n1, n2):
    """Refraction by the scalar law n1 sin(t1) = n2 sin(t2) (Eq. (1)), built from
    angles: the transmitted ray lies in the plane of d and N."""
    dn = float(np.dot(d, N))
    nin = N if dn > 0 else -N  # normal oriented along propagation
    cos1 = abs(dn)
    t = d - dn * N
    tl = np.linalg.norm(t)
    if tl == 0.0:
        return d.copy()
    sin2 = n1 * math.sqrt(max(0.0, 1.0 - cos1 * cos1)) / n2
    assert sin2 < 1.0
    return math.sqrt(1.0 - sin2 * sin2) * nin + sin2 * (t / tl)


# ---------------------------------------------------------------------------
# medium evaluation: gradient consistent with the index (all analytic kinds)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("medium", [
    {"kind": "linear", "params": np.array([1.5, 0.1, -0.2, 0.3])},
    {"kind": "luneburg", "params": np.array([1.3, 0.1, -0.2, 0.05])},
    {"kind": "fiber", "params": np.array([1.38, 0.2, 5.0, 0.3, -0.1])},
    workloads.gaussian_medium(2),
])
def test_gradient_matches_finite_difference(orc, medium):
    medium = dict(medium)
    medium.setdefault("boundary", box((0, 0, 0), (1, 1, 1)))
    medium.setdefault("n_amb", 1.0)
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.05, 0.95, (64, 3))
    n, g = orc.evaluate(medium, pts)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (orc.evaluate(medium, pts + e)[0] - orc.evaluate(medium, pts - e)[0]) / (2 * h)
        assert np.allclose(g[:, a], fd, rtol=1e-6, atol=1e-8)


def test_luneburg_and_fiber_index_closed_form(orc):
    lun = {"kind": "luneburg", "params": np.array([1.0, 0, 0, 0]), "boundary": sphere(),
           "n_amb": 1.0}
    n, _ = orc.evaluate(lun, np.array([[0, 0, 0], [1, 0, 0], [0, 0.6, 0.8]]))
    assert np.allclose(n, [math.sqrt(2), 1.0, 1.0], rtol=0, atol=1e-15)
    # Eq. (21): n(rho=R) = n_c sqrt(1 - 2 Delta) = cladding index, n(0) = n_c
    fib = {"kind": "fiber", "params": np.array([1.38, 0.2, 5.0, 0, 0]),
           "boundary": sphere(), "n_amb": 1.0}
    n, g = orc.evaluate(fib, np.array([[0, 0, 0], [5, 0, 0], [3, 4, 1], [6, 0, 0]]))
    ncl = 1.38 * math.sqrt(0.6)
    assert np.allclose(n, [1.38, ncl, ncl, ncl], atol=1e-15)
    assert np.all(g[0] == 0) and np.all(g[3] == 0)


# ---------------------------------------------------------------------------
# P1: homogeneous media -> straight lines, scalar Snell at the surfaces
# ---------------------------------------------------------------------------
def test_homogeneous_ball_matches_scalar_snell_geometry(orc):
    nh, dL0 = 1.5, 1e-3
    med = homogeneous(nh, sphere(1.0))
    d = np.array([0.1, -0.05, 1.0])
    d /= np.linalg.norm(d)
    xs = np.linspace(-0.85, 0.85, 9)
    P0 = np.array([[x, y, -2.0] for x in xs for y in xs])
    d0 = np.tile(d, (len(P0), 1))
    r = orc.trace(med, (P0, d0), P(dL0))
    for i in range(len(P0)):
        b = P0[i] @ d
        c = P0[i] @ P0[i] - 1.0
        if b * b - c <= 0.0:
            assert r["status"][i] == orc.MISSED
            continue
        t = -b - math.sqrt(b * b - c)
        PB = P0[i] + t * d
        Rin = scalar_snell(d, PB, 1.0, nh)
        chord = -2.0 * PB @ Rin
        PE = PB + chord * Rin
        Rout = scalar_snell(Rin, PE, nh, 1.0)
        assert r["status"][i] == orc.EXITED
        assert np.allclose(r["P"][i], PE, atol=1e-12)
        assert np.allclose(r["D"][i], Rout, atol=1e-12)
        assert r["ntir"][i] == 0 and r["nbtir"][i] == 0
        q = chord / (dL0 / nh)
        if abs(q - round(q)) > 1e-6:
            assert r["steps"][i] == math.ceil(q)


def _fold(u):
    m = math.floor(u)
    f = u - m
    return (f if m % 2 == 0 else 1.0 - f), m


def test_homogeneous_cube_unfolded_mirror_paths(orc):
    """Side faces reflect by TIR (incidence > 77 deg > critical 41.8 deg); the
    path inside is the straight unfolded line folded back into the cube and
    the exit direction is the launch direction with mirrored signs."""
    nh, dL0 = 1.5, 2e-3
    med = homogeneous(nh, box((0, 0, 0), (1, 1, 1)))
    P0, d0 = workloads.face_cone_rays(400, seed=11, cone_deg=20.0)
    r = orc.trace(med, (P0, d0), P(dL0))
    assert np.all(r["status"] == orc.EXITED)
    for i in range(len(P0)):
        d = d0[i] / np.linalg.norm(d0[i])
        R = scalar_snell(d, np.array([0, 0, -1.0]), 1.0, nh)
        X, Y = P0[i, 0] + R[0] / R[2], P0[i, 1] + R[1] / R[2]
        fx, mx = _fold(X)
        fy, my = _fold(Y)
        assert np.allclose(r["P"][i], [fx, fy, 1.0], atol=1e-12)
        sx, sy = (-1) ** (mx % 2), (-1) ** (my % 2)
        assert np.allclose(r["D"][i], [sx * d[0], sy * d[1], d[2]], atol=1e-12)
        assert r["nbtir"][i] == abs(mx) + abs(my)
        assert r["ntir"][i] == 0
        # steps: each straight piece between surface events is cut into
        # ceil(length / Delta) moves
        ts = sorted([(k - P0[i, 0]) / R[0] for k in range(-3, 5) if R[0] != 0
                     and 0 < (k - P0[i, 0]) / R[0] < 1 / R[2]] +
                    [(k - P0[i, 1]) / R[1] for k in range(-3, 5) if R[1] != 0
                     and 0 < (k - P0[i, 1]) / R[1] < 1 / R[2]])
        cuts = [0.0] + ts + [1.0 / R[2]]
        Delta = dL0 / nh
        qs = [(b - a) / Delta for a, b in zip(cuts[:-1], cuts[1:])]
        if all(abs(q - round(q)) > 1e-6 for q in qs):
            assert r["steps"][i] == sum(math.ceil(q) for q in qs)


# ---------------------------------------------------------------------------
# P2: stratified media n(z): exact tangential invariant and catenary paths
# ---------------------------------------------------------------------------
def linear_slab(n0, g, n_amb=1.0):
    return {"kind": "linear", "params": np.array([n0, 0.0, 0.0, g]),
            "boundary": box((-50, -50, 0), (50, 50, 1)), "n_amb": n_amb}


def test_stratified_slab_preserves_tangential_momentum_exactly(orc):
    """Every normal (gradient and both faces) is along z, so the vectorial law
    conserves n * I_perp exactly at entry, at every Snell step and at exit: with
    no TIR the exit direction equals the launch direction."""
    med = linear_slab(1.5, 0.3)
    P0, d0 = workloads.face_cone_rays(256, seed=12, cone_deg=60.0)
    r = orc.trace(med, (P0, d0), P(1e-3))
    dn = d0 / np.linalg.norm(d0, axis=1, keepdims=True)
    assert np.all(r["status"] == orc.EXITED) and np.all(r["ntir"] == 0)
    assert np.allclose(r["D"], dn, atol=1e-13)
    assert np.allclose(r["P"][:, 2], 1.0, atol=0)


def catenary_x(n0, g, T, z0, z1):
    """x-advance of a ray with invariant T = n sin(theta) in n = n0 + g z."""
    f = lambda z: (T / g) * math.acosh((n0 + g * z) / T)
    return f(z1) - f(z0)


def test_stratified_slab_path_converges_first_order(orc):
    n0, g = 1.5, 0.3
    med = linear_slab(n0, g)
    th = math.radians(50.0)
    d0 = np.array([[math.sin(th), 0.0, math.cos(th)]])
    P0 = np.array([[0.0, 0.0, 0.0]])
    T = math.sin(th)  # n_amb sin(theta0)
    xe = catenary_x(n0, g, T, 0.0, 1.0)
    errs = []
    for dL0 in (4e-3, 2e-3, 1e-3, 5e-4):
        r = orc.trace(med, (P0, d0), P(dL0))
        errs.append(abs(r["P"][0, 0] - xe))
    errs = np.array(errs)
    assert errs[-1] < 1e-4
    slope = np.polyfit(np.log([4e-3, 2e-3, 1e-3, 5e-4]), np.log(errs), 1)[0]
    assert 0.8 < slope < 1.2, (errs, slope)


def test_turning_point_tir_returns_ray_first_order(orc):
    """n = 1.2 - 0.5 z: a ray with T = sin(60 deg) turns where n = T and comes
    back to z = 0 after 2 (T/|g|) acosh(n0/T); the turn is made by case (v)."""
    n0, g = 1.2, -0.5
    med = linear_slab(n0, g)
    th = math.radians(60.0)
    T = math.sin(th)
    d0 = np.array([[math.sin(th), 0.0, math.cos(th)]])
    P0 = np.array([[0.0, 0.0, 0.0]])
    xe = 2.0 * (T / abs(g)) * math.acosh(n0 / T)
    errs = []
    for dL0 in (4e-4, 2e-4, 1e-4, 5e-5):
        r = orc.trace(med, (P0, d0), P(dL0))
        assert r["status"][0] == orc.EXITED and r["ntir"][0] >= 1
        assert abs(r["P"][0, 2]) == 0.0
        errs.append(math.hypot(r["P"][0, 0] - xe, r["P"][0, 1]))
        # continuous limit leaves mirrored: (sin, 0, -cos)
        assert np.allclose(r["D"][0], [math.sin(th), 0, -math.cos(th)], atol=5e-2)
    errs = np.array(errs)
    assert errs[-1] < 2e-3
    slope = np.polyfit(np.log([4e-4, 2e-4, 1e-4, 5e-5]), np.log(errs), 1)[0]
    assert 0.7 < slope < 1.3, (errs, slope)


def test_step_lengths_follow_eqs_4_and_20(orc):
    """Per-step OPL identity read off the polyline alone: in n(z) every normal
    is along z, so a step that flips the sign of the z-direction is a
    reflection and must have length dL0 / n(P_{i-1}) (Eq. (20)); every other
    interior step has length dL0 / n(P_i) (Eq. (4))."""
    n0, g = 1.2, -0.5
    med = linear_slab(n0, g)
    th = math.radians(60.0)
    dL0 = 1e-4
    path, res = orc.trace_path(med, np.zeros(3), np.array([math.sin(th), 0, math.cos(th)]),
                               P(dL0))
    pts = path[1:-1]  # interior points after the entry point, without the exit point
    seg = np.diff(path[1:], axis=0)
    lens = np.linalg.norm(seg, axis=1)
    n, _ = orc.evaluate(med, path[1:])
    n_tir = 0
    for i in range(1, len(seg) - 1):
        flipped = np.sign(seg[i, 2]) != np.sign(seg[i - 1, 2])
        nsz = n[i - 1] if flipped else n[i]
        assert abs(nsz * lens[i] / dL0 - 1.0) < 1e-10, (i, flipped)
        n_tir += flipped
    assert n_tir == res["ntir"] >= 1
    assert len(pts) > 100


# ---------------------------------------------------------------------------
# P3: Luneburg sphere (perfect focus), exact discrete Bouguer invariant
# ---------------------------------------------------------------------------
def test_luneburg_bouguer_vector_exact_through_entry_steps_and_exit(orc):
    med, (P0, d0), prm = workloads.luneburg_beam(n_side=32)
    r = orc.trace(med, (P0, d0), prm)
    ex = r["status"] == orc.EXITED
    h = np.hypot(P0[:, 0], P0[:, 1])
    assert np.all(ex == (h < 1.0))
    assert np.all(r["status"][~ex] == orc.MISSED)
    L0 = np.cross(P0, d0)
    L1 = np.cross(r["P"], r["D"])
    assert np.allclose(L1[ex], L0[ex], atol=1e-12)
    assert np.all(r["ntir"] == 0) and np.all(r["nbtir"] == 0)


def test_luneburg_bouguer_vector_every_step(orc):
    med, _, prm = workloads.luneburg_beam()
    for x0, y0 in [(0.3, 0.1), (-0.62, 0.41), (0.05, -0.9)]:
        path, res = orc.trace_path(med, np.array([x0, y0, -1.5]), np.array([0, 0, 1.0]), prm)
        pts = path[1:]  # from the entry point on
        seg = pts[1:] - pts[:-1]
        lens = np.linalg.norm(seg, axis=1)
        R = seg / lens[:, None]
        n, _ = orc.evaluate(med, pts[:-1])
        L = n[:, None] * np.cross(pts[:-1], R)
        assert np.allclose(L, [y0, -x0, 0.0], atol=1e-12)
        # P8: every step except the last (cut at the surface) has OPL dL0
        assert np.allclose(n[:-1] * lens[:-1], prm["dL0"], rtol=1e-12, atol=0)


def test_luneburg_focus_direction_and_steps(orc):
    """Continuous closed forms for R = 1: parallel rays focus at (0, 0, 1) and
    leave along (-x0, -y0, sqrt(1 - h^2)); the in-lens OPL is pi/2 + sqrt(1-h^2)."""
    errs = []
    for dL0 in (2e-3, 1e-3, 5e-4):
        med, (P0, d0), prm = workloads.luneburg_beam(n_side=24, dL0=dL0, max_steps=100000)
        r = orc.trace(med, (P0, d0), prm)
        h = np.hypot(P0[:, 0], P0[:, 1])
        m = (r["status"] == orc.EXITED) & (h < 0.9)
        pe = np.linalg.norm(r["P"][m] - [0, 0, 1], axis=1)
        De = np.stack([-P0[m, 0], -P0[m, 1], np.sqrt(1 - h[m] ** 2)], axis=1)
        de = np.linalg.norm(r["D"][m] - De, axis=1)
        errs.append(np.sqrt(np.mean(pe ** 2)))
        assert np.sqrt(np.mean(de ** 2)) < 0.6 * dL0
        opl = (math.pi / 2 + np.sqrt(1 - h[m] ** 2)) / dL0
        assert np.all(np.abs(r["steps"][m] - opl) < 0.01 * opl)
    errs = np.array(errs)
    assert errs[1] < 6e-4
    assert 1.6 < errs[0] / errs[1] < 2.5 and 1.6 < errs[1] / errs[2] < 2.5


def test_luneburg_axial_ray_normal_incidence_is_straight(orc):
    """Normal incidence must give R = I (Sec. II, after Eq. (10))."""
    med, _, prm = workloads.luneburg_beam()
    path, res = orc.trace_path(med, np.array([0.0, 0.0, -1.5]), np.array([0, 0, 1.0]), prm)
    assert res["status"] == orc.EXITED
    assert np.all(path[:, :2] == 0.0)
    assert np.array_equal(res["P"], [0.0, 0.0, 1.0])
    assert np.array_equal(res["D"], [0.0, 0.0, 1.0])


# ---------------------------------------------------------------------------
# P4: the paper's helix benchmark (Sec. IV)
# ---------------------------------------------------------------------------
def helix_setup():
    gold = json.load(open(os.path.join(GOLDEN, "helix_e1.json")))
    nc, Dl, R = gold["n_c"], gold["Delta"], gold["R"]
    rho0 = gold["P_I"][0]
    ncl = nc * math.sqrt(1 - 2 * Dl)  # surroundings = cladding index (Eq. (21), rho > R)
    om = nc * math.sqrt(2 * Dl) / R  # n^2 = n_c^2 - om^2 rho^2
    beta = math.sqrt(nc ** 2 - 2 * om ** 2 * rho0 ** 2)  # axial invariant of the helix
    kappa = om / beta
    sin_out = om * rho0 / ncl  # tangential momentum of the helix, seen outside
    L = 55.0  # length that holds the paper's m points at its dL0
    med = {"kind": "fiber", "params": np.array([nc, Dl, R, 0.0, 0.0]),
           "boundary": {"kind": "cylinder", "params": np.array([0.0, 0.0, R, 0.0, L])},
           "n_amb": ncl}
    d0 = np.array([0.0, sin_out, math.sqrt(1 - sin_out ** 2)])
    P0 = np.array(gold["P_I"]) - rho0 * d0
    return gold, med, P0, d0, kappa, rho0


def test_helix_launch_matches_paper_geometry():
    gold, med, P0, d0, kappa, rho0 = helix_setup()
    assert abs(math.degrees(math.acos(d0[2])) - gold["angle_to_z_deg"]) < 0.005
    assert np.allclose(P0, gold["P0"], atol=5e-4)


def test_helix_rmse_matches_paper(orc):
    gold, med, P0, d0, kappa, rho0 = helix_setup()
    path, res = orc.trace_path(med, P0, d0, P(gold["dL0"], max_steps=2_000_000))
    assert res["status"] == orc.EXITED
    ins = path[path[:, 2] >= 0.0]
    z = ins[:, 2]
    rmse = math.sqrt(np.mean((ins[:, 0] - rho0 * np.cos(kappa * z)) ** 2 +
                             (ins[:, 1] - rho0 * np.sin(kappa * z)) ** 2))
    assert abs(len(ins) - gold["m_points"]) <= 1
    assert abs(rmse / gold["rmse"] - 1.0) < 0.10, rmse
    # the helix stays on its cylinder
    rho = np.hypot(ins[:, 0], ins[:, 1])
    assert np.max(np.abs(rho - rho0)) < 1e-3


# ---------------------------------------------------------------------------
# P5: meridional ray in the fiber: tangential rule and closed-form cosine path
# ---------------------------------------------------------------------------
def test_meridional_ray_tangential_rule_and_cosine_path(orc):
    nc, Dl, R = 1.38, 0.2, 5.0
    med = {"kind": "fiber", "params": np.array([nc, Dl, R, 0.0, 0.0]),
           "boundary": {"kind": "cylinder", "params": np.array([0, 0, R, 0.0, 30.0])},
           "n_amb": 1.0}
    x0 = 2.0
    om = nc * math.sqrt(2 * Dl) / R
    n_x0 = nc * math.sqrt(1 - 2 * Dl * x0 ** 2 / R ** 2)
    P0 = np.array([x0, 0.0, 1.0])
    d0 = np.array([0.0, 0.0, 1.0])
    errs = []
    for dL0 in (4e-4, 2e-4, 1e-4):
        path, res = orc.trace_path(med, P0, d0, P(dL0, max_steps=1_000_000))
        assert res["flags"] & orc.F_TANGENT
        assert np.all(path[:, 1] == 0.0)  # stays in the meridional plane
        # first step turns the ray by half the arc angle: sin(a) ~ Delta K / 2
        # with ray curvature K = |grad n| / n (Eq. (13))
        s = path[1] - path[0]
        ang = math.atan2(-s[0], s[2])
        K = 2 * Dl * nc * nc * x0 / (R * R * n_x0) / n_x0
        assert abs(ang / (0.5 * (dL0 / n_x0) * K) - 1.0) < 1e-3
        pts = path[(path[:, 2] > 1.0) & (path[:, 2] < 29.0)]
        xe = x0 * np.cos(om * (pts[:, 2] - 1.0) / n_x0)
        errs.append(np.sqrt(np.mean((pts[:, 0] - xe) ** 2)))
    errs = np.array(errs)
    assert errs[-1] < 2e-3
    assert 1.6 < errs[0] / errs[1] < 2.5 and 1.6 < errs[1] / errs[2] < 2.5, errs


# ---------------------------------------------------------------------------
# P6: discretized medium (trilinear grid) twins analytic media
# ---------------------------------------------------------------------------
def test_grid_of_linear_field_twins_linear_medium(orc):
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([1.0, 1.2, 1.4])
    nx, ny, nz = 5, 6, 7
    g = np.array([0.1, -0.05, 0.2])
    xs = [np.linspace(lo[a], hi[a], n) for a, n in zip(range(3), (nx, ny, nz))]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    vals = (1.5 + g[0] * X + g[1] * Y + g[2] * Z)
    vals32 = vals.astype(np.float32)
    # use a field whose node values are exact in float32: fit n0, g to the rounded grid
    grid = workloads.grid_medium(vals32, lo, hi)
    lin = {"kind": "linear", "params": np.array([1.5, *g]), "boundary": grid["boundary"],
           "n_amb": 1.0}
    rng = np.random.default_rng(3)
    pts = rng.uniform(lo, hi, (200, 3))
    n_g, g_g = orc.evaluate(grid, pts)
    n_l, g_l = orc.evaluate(lin, pts)
    assert np.allclose(n_g, n_l, atol=2e-7)  # float32 node rounding only
    assert np.allclose(g_g, g_l, atol=2e-6)
    # with node values exactly linear in float64 the twin is exact to rounding
    grid64 = dict(grid)
    grid64["grid"] = vals.astype(np.float32)
    exact = np.abs(vals32.astype(np.float64) - vals).max() == 0.0
    P0, d0 = workloads.face_cone_rays(300, seed=13, cone_deg=25.0)
    P0 = P0 * np.array([1.0, 1.2, 1.0])
    prm = P(2e-3)
    rg = orc.trace(grid, (P0, d0), prm)
    rl = orc.trace(lin, (P0, d0), prm)
    assert np.array_equal(rg["status"], rl["status"])
    tol = 1e-11 if exact else 5e-5
    assert np.allclose(rg["P"], rl["P"], atol=tol)
    assert np.allclose(rg["D"], rl["D"], atol=tol)


def test_grid_of_exactly_linear_nodes_is_bitwise_close(orc):
    """Node values k/8 are exact in float32, so grid and linear twins agree to
    rounding and take identical discrete decisions."""
    lo, hi = np.zeros(3), np.array([1.0, 1.0, 1.0])
    N = 9
    k = np.arange(N) / (N - 1)
    Z, Y, X = np.meshgrid(k, k, k, indexing="ij")
    vals = 1.5 + 0.125 * X - 0.25 * Y + 0.375 * Z  # all multiples of 2^-6
    grid = workloads.grid_medium(vals.astype(np.float32), lo, hi)
    lin = {"kind": "linear", "params": np.array([1.5, 0.125, -0.25, 0.375]),
           "boundary": grid["boundary"], "n_amb": 1.0}
    P0, d0 = workloads.face_cone_rays(300, seed=14, cone_deg=30.0)
    prm = P(1e-3)
    rg, rl = orc.trace(grid, (P0, d0), prm), orc.trace(lin, (P0, d0), prm)
    for key in ("status", "steps", "ntir", "nbtir"):
        assert np.array_equal(rg[key], rl[key]), key
    assert np.allclose(rg["P"], rl["P"], atol=1e-12)
    assert np.allclose(rg["D"], rl["D"], atol=1e-12)


def test_constant_grid_twins_homogeneous(orc):
    grid = workloads.grid_medium(np.full((4, 4, 4), 1.5, dtype=np.float32))
    hom = homogeneous(1.5, grid["boundary"])
    P0, d0 = workloads.face_cone_rays(200, seed=15, cone_deg=20.0)
    prm = P(1e-3)
    rg, rh = orc.trace(grid, (P0, d0), prm), orc.trace(hom, (P0, d0), prm)
    for key in ("status", "steps", "ntir", "nbtir"):
        assert np.array_equal(rg[key], rh[key])
    assert np.allclose(rg["P"], rh["P"], atol=1e-13)
    assert np.all(rg["flags"] & orc.F_STRAIGHT)


def test_one_cell_grid_by_hand(orc):
    """2x2x2 grid: n is the trilinear blend of the 8 corners and the gradient
    the blend of one-sided corner differences."""
    v = np.arange(8, dtype=np.float32).reshape(2, 2, 2) * 0.01 + 1.4  # v[z, y, x]
    grid = workloads.grid_medium(v)
    x, y, z = 0.25, 0.5, 0.75
    n, g = orc.evaluate(grid, np.array([[x, y, z]]))
    vv = v.astype(np.float64)
    lerp = lambda a, b, t: a + (b - a) * t
    c00 = lerp(vv[0, 0, 0], vv[0, 0, 1], x)
    c10 = lerp(vv[0, 1, 0], vv[0, 1, 1], x)
    c01 = lerp(vv[1, 0, 0], vv[1, 0, 1], x)
    c11 = lerp(vv[1, 1, 0], vv[1, 1, 1], x)
    ref = lerp(lerp(c00, c10, y), lerp(c01, c11, y), z)
    assert abs(n[0] - ref) < 1e-15
    # index = 1.4 + 0.01 (4 z + 2 y + x): a linear field -> exact constant gradient
    assert np.allclose(g[0], [0.01, 0.02, 0.04], atol=1e-12)


# ---------------------------------------------------------------------------
# P7: convergence against an independent integration of the ray equation
# ---------------------------------------------------------------------------
def test_first_order_convergence_vs_ray_equation_gaussian_medium(orc):
    from scipy.integrate import solve_ivp

    med = workloads.gaussian_medium(2)
    p = med["params"]
    n0, K = p[0], int(p[1])
    B = p[2:].reshape(K, 5)

    def n_and_grad(r):
        d = r[None, :] - B[:, 2:5]
        e = B[:, 0] * np.exp(-np.sum(d * d, axis=1) / (2 * B[:, 1] ** 2))
        return n0 + e.sum(), -(e / B[:, 1] ** 2) @ d

    def rhs(t, y):  # d2r/dtau2 = n grad n, dtau = ds / n
        n, g = n_and_grad(y[:3])
        return np.concatenate([y[3:], n * g])

    def hit(t, y):
        return y[2] - 1.0
    hit.terminal = True
    hit.direction = 1

    rng = np.random.default_rng(21)
    steps = (2e-3, 1e-3, 5e-4, 2.5e-4)
    clean, kicked = [], []
    for _ in range(80):
        if len(clean) == 8:
            break
        r0 = np.array([rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7), 0.02])
        th, ph = rng.uniform(0, 0.25), rng.uniform(0, 2 * math.pi)
        d0 = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        n_start, _ = n_and_grad(r0)
        sol = solve_ivp(rhs, (0, 10.0), np.concatenate([r0, n_start * d0]), method="DOP853",
                        rtol=1e-12, atol=1e-13, events=hit)
        if sol.status != 1:
            continue
        xe = sol.y_events[0][0][:3]
        if np.any(xe[:2] < 0.01) or np.any(xe[:2] > 0.99):
            continue
        row, tirs = [], 0
        for dL0 in steps:
            r = orc.trace(med, (r0[None], d0[None]), P(dL0))
            assert r["status"][0] == orc.EXITED and r["nbtir"][0] == 0
            row.append(np.linalg.norm(r["P"][0] - xe))
            tirs += int(r["ntir"][0])
        (clean if tirs == 0 else kicked).append(row)
    # Snell-only rays: first order (RMS error proportional to dL0, Sec. III)
    assert len(clean) == 8
    rms = np.sqrt(np.mean(np.array(clean) ** 2, axis=0))
    slope = np.polyfit(np.log(steps), np.log(rms), 1)[0]
    assert 0.85 < slope < 1.15, (rms, slope)
    # a turning-point TIR is an O(dL0) kick too: bounded by the same order
    for row in kicked:
        assert np.all(np.array(row) < 2.0 * np.array(steps)), row


# ---------------------------------------------------------------------------
# statuses, flags, exit plane
# ---------------------------------------------------------------------------
def test_near_critical_flag_at_the_critical_angle(orc):
    """Ray inside an n = 1.5 cube hitting the face z = 1 within / outside 1e-6
    rad of the critical angle asin(1/1.5) (Eq. (19))."""
    med = homogeneous(1.5, box((0, 0, 0), (1, 1, 1)))
    thc = math.asin(1 / 1.5)
    # (offset, TIR, within 1e-6, within the wide window 1e-5)
    cases = [(+3e-7, True, True, True), (-3e-7, False, True, True),
             (+5e-6, True, False, True), (-5e-6, False, False, True),
             (+2e-5, True, False, False), (-2e-5, False, False, False)]
    for dth, tir, flagged, wide in cases:
        th = thc + dth
        d = np.array([[math.sin(th), 0.0, math.cos(th)]])
        P0 = np.array([[0.02, 0.5, 0.95]])
        r = orc.trace(med, (P0, d), P(1e-3))
        assert bool(r["flags"][0] & orc.F_NEAR_CRITICAL) == flagged, dth
        assert bool(r["flags"][0] & orc.F_NEAR_CRITICAL_WIDE) == wide, dth
        assert (r["nbtir"][0] >= 1) == tir, dth


def test_wide_flag_windows_are_the_narrow_ones_scaled(orc):
    """Bits 64/128/256 with windows (crit_rad, tie_eps) equal bits 1/16/32 with
    ten times those windows, on a Gaussian-bump medium with many TIRs."""
    spec, (P0, d0), prm = workloads.gaussian_cube(n_rays=1 << 20)
    P0, d0 = P0[:2048], d0[:2048]
    a = orc.trace(spec, (P0, d0), prm)
    wide = dict(prm, crit_rad=10 * prm["crit_rad"], tie_eps=10 * prm["tie_eps"])
    b = orc.trace(spec, (P0, d0), wide)
    for narrow_bit, wide_bit in ((orc.F_NEAR_CRITICAL, orc.F_NEAR_CRITICAL_WIDE),
                                 (orc.F_NEAR_TIE, orc.F_NEAR_TIE_WIDE),
                                 (orc.F_NEAR_GRAZING, orc.F_NEAR_GRAZING_WIDE)):
        assert np.array_equal((a["flags"] & wide_bit) != 0, (b["flags"] & narrow_bit) != 0)
        # the narrow window lies inside the wide one
        assert not np.any((a["flags"] & narrow_bit) & ~((a["flags"] & wide_bit) // wide_bit * narrow_bit))
        assert ((b["flags"] & narrow_bit) != 0).sum() > 0


def test_statuses(orc):
    med = homogeneous(1.5, sphere(1.0))
    P0 = np.array([[0, 0, -3.0], [3, 3, -3.0], [np.nan, 0, 0], [0, 0, -3.0], [0, 0, 0.0]])
    d0 = np.array([[0, 0, 1.0], [0, 0, 1.0], [0, 0, 1.0], [0, 0, 0.0], [1.0, 0, 0]])
    r = orc.trace(med, (P0, d0), P(1e-3, max_steps=10000))
    assert list(r["status"]) == [orc.EXITED, orc.MISSED, orc.INVALID_INPUT, orc.INVALID_INPUT,
                                 orc.EXITED]
    r = orc.trace(med, (P0[:1], d0[:1]), P(1e-3, max_steps=5))
    assert r["status"][0] == orc.TRUNCATED and r["steps"][0] == 5
    # optically denser surroundings: grazing entry is reflected
    med2 = homogeneous(1.0, sphere(1.0), n_amb=2.0)
    r = orc.trace(med2, (np.array([[0.95, 0, -3.0]]), np.array([[0, 0, 1.0]])), P(1e-3))
    assert r["status"][0] == orc.REFLECTED_AT_ENTRY
    assert np.allclose(np.linalg.norm(r["P"][0]), 1.0)


def test_exit_plane_is_straight_continuation(orc):
    med = homogeneous(1.5, box((0, 0, 0), (1, 1, 1)))
    P0, d0 = workloads.face_cone_rays(50, seed=16, cone_deg=10.0)
    ra = orc.trace(med, (P0, d0), P(1e-3))
    rb = orc.trace(med, (P0, d0), P(1e-3, exit_plane_z=1.2))
    t = 0.2 / ra["D"][:, 2]
    assert np.allclose(rb["P"], ra["P"] + t[:, None] * ra["D"], atol=1e-12)
    assert np.all(rb["P"][:, 2] == 1.2)
    # leaving backwards through z = 0 never reaches the plane
    rc = orc.trace(med, (np.array([[0.5, 0.5, 0.5]]), np.array([[0, 0, -1.0]])),
                   P(1e-3, exit_plane_z=1.2))
    assert rc["status"][0] == orc.NO_PLANE


def test_exit_gain_is_the_derivative_of_snells_law():
    """The parity bar on exit directions is widened by the derivative of the
    exit refraction; check that factor against a finite difference of the
    scalar law n_in sin t_in = n_amb sin t_out, for a box face and a sphere."""
    from parity import exit_gain, surface_normal

    n_in, n_amb = 1.5, 1.0
    t_in = np.array([0.1, 0.4, 0.6, 0.72])  # critical angle asin(1/1.5) = 0.7297
    t_out = np.arcsin(n_in / n_amb * np.sin(t_in))
    h = 1e-7
    fd = (np.arcsin(n_in / n_amb * np.sin(t_in + h)) - np.arcsin(n_in / n_amb * np.sin(t_in - h))) / (2 * h)
    # exits through the face z = 1 of the unit box, direction in the x-z plane
    P = np.column_stack([np.full(4, 0.3), np.full(4, 0.6), np.ones(4)])
    D = np.column_stack([np.sin(t_out), np.zeros(4), np.cos(t_out)])
    spec = {"boundary": {"kind": "box", "params": np.array([0, 0, 0, 1, 1, 1.0])}, "n_amb": n_amb}
    orc = {"status": np.zeros(4, np.uint32), "P": P, "D": D}
    g = exit_gain(spec, orc, lambda Q: np.full(len(Q), n_in))
    assert np.allclose(g, fd, rtol=1e-5), (g, fd)
    # the same exits through a sphere of radius 2 about the origin
    spec_s = {"boundary": {"kind": "sphere", "params": np.array([0, 0, 0, 2.0])}, "n_amb": n_amb}
    N = np.array([0.0, 0.6, 0.8])
    assert np.allclose(surface_normal(spec_s["boundary"], 2.0 * N[None, :]), N[None, :])
    e1 = np.cross(N, [1.0, 0, 0]); e1 /= np.linalg.norm(e1)
    Ds = np.cos(t_out)[:, None] * N[None, :] + np.sin(t_out)[:, None] * e1[None, :]
    orc_s = {"status": np.zeros(4, np.uint32), "P": np.tile(2.0 * N, (4, 1)), "D": Ds}
    assert np.allclose(exit_gain(spec_s, orc_s, lambda Q: np.full(len(Q), n_in)), fd, rtol=1e-5)
    # not on the surface (an exit plane) or not exited: no widening
    orc_p = {"status": np.array([0, 2, 0, 0], np.uint32), "P": P + [0, 0, 0.5], "D": D}
    assert np.all(exit_gain(spec, orc_p, lambda Q: np.full(len(Q), n_in)) == 1.0)


# ---------------------------------------------------------------------------
# the grid's node gradient at interior nodes (discretized-medium reading:
# central differences inside, one-sided at the faces)
# ---------------------------------------------------------------------------
def _quadratic_grid(N=9):
    """Nodes k/(N-1) of the unit cube carrying a full quadratic field whose
    node values are exact in float32 (coefficients and coordinates are short
    dyadic fractions), with its analytic gradient."""
    a, b, c, d, e, f = 0.0625, -0.125, 0.09375, 0.03125, -0.046875, 0.0546875
    gx0, gy0, gz0 = 0.25, -0.1875, 0.125

    def q(X, Y, Z):
        return (1.5 + gx0 * X + gy0 * Y + gz0 * Z + a * X * X + b * Y * Y + c * Z * Z +
                d * X * Y + e * Y * Z + f * X * Z)

    def grad(X, Y, Z):
        return np.stack([gx0 + 2 * a * X + d * Y + f * Z,
                         gy0 + 2 * b * Y + d * X + e * Z,
                         gz0 + 2 * c * Z + e * Y + f * X], axis=-1)

    k = np.arange(N) / (N - 1)
    Z, Y, X = np.meshgrid(k, k, k, indexing="ij")
    vals = q(X, Y, Z)
    assert np.array_equal(vals.astype(np.float32).astype(np.float64), vals)
    return workloads.grid_medium(vals.astype(np.float32)), q, grad, (a, b, c)


def test_grid_gradient_is_exact_for_a_quadratic_field_inside(orc):
    """Central differences are exact for a quadratic, so at every point of a
    cell whose eight corners are interior nodes the gradient (trilinear blend
    of the node differences, each exact and linear in the coordinates) equals
    the analytic one.  A one-sided (forward or backward) stencil is off by
    a h there, which this rules out."""
    N = 9
    grid, q, grad, (a, b, c) = _quadratic_grid(N)
    h = 1.0 / (N - 1)
    rng = np.random.default_rng(31)
    pts = rng.uniform(h, 1.0 - h, (300, 3))
    n, g = orc.evaluate(grid, pts)
    assert np.allclose(g, grad(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=0, atol=1e-13)
    # at the interior nodes themselves, n is the node value
    k = np.arange(1, N - 1) * h
    Z, Y, X = np.meshgrid(k, k, k, indexing="ij")
    nodes = np.column_stack([X.ravel(), Y.ravel(), Z.ravel()])
    nn, gn = orc.evaluate(grid, nodes)
    assert np.allclose(nn, q(nodes[:, 0], nodes[:, 1], nodes[:, 2]), rtol=0, atol=1e-15)
    assert np.allclose(gn, grad(nodes[:, 0], nodes[:, 1], nodes[:, 2]), rtol=0, atol=1e-13)


def test_grid_gradient_is_one_sided_at_the_faces(orc):
    """At a face node the difference runs over the one spacing that exists:
    (q(h) - q(0)) / h = q'(0) + a h for the pure square term, and
    (q(1) - q(1-h)) / h = q'(1) - a h on the opposite face."""
    N = 9
    grid, q, grad, (a, b, c) = _quadratic_grid(N)
    h = 1.0 / (N - 1)
    y, z = 3 * h, 5 * h
    lo_face, hi_face = np.array([[0.0, y, z]]), np.array([[1.0, y, z]])
    _, g_lo = orc.evaluate(grid, lo_face)
    _, g_hi = orc.evaluate(grid, hi_face)
    ex_lo = grad(0.0, y, z)[0] + a * h
    ex_hi = grad(1.0, y, z)[0] - a * h
    assert abs(g_lo[0, 0] - ex_lo) < 1e-13 and abs(g_hi[0, 0] - ex_hi) < 1e-13
    # the other two components at those nodes are interior central differences
    assert np.allclose(g_lo[0, 1:], grad(0.0, y, z)[1:], atol=1e-13)


# ---------------------------------------------------------------------------
# the windows that mark ill-conditioned decisions, placed by hand
# ---------------------------------------------------------------------------
def _tie_case(orc, boundary, E, X, d, cos_t, delta_perp, k=5, dL0=1e-3, n=1.5):
    """Launch a ray inside a homogeneous medium so that the end of its k-th
    constant-OPL step lies at signed distance delta_perp from the surface,
    measured perpendicular to it (> 0: inside).  E is where the step ends, X the
    surface point on the ray.  Returns the oracle's flags after the ray meets
    the surface (the march is truncated right after the surface event)."""
    med = homogeneous(n, boundary)
    Delta = dL0 / n
    P0 = E - k * Delta * d
    r = orc.trace(med, (P0[None], d[None]), P(dL0, max_steps=k + 1))
    return int(r["flags"][0]), r


def test_near_tie_window_is_perpendicular_distance_box(orc):
    """Sec. II case (i): whether a step is cut at the surface or taken in full
    is decided by the step end's side of the surface.  The near-tie flag marks
    a step end within tie_eps of the surface measured perpendicular to it, so
    a ray crossing the face z = 1 at cos t = 1/4 is flagged at a perpendicular
    distance of tie_eps / 2 (two tie_eps along the ray) on either side, and
    not at 2 tie_eps; the ten times wider bit marks 5 tie_eps."""
    tie = workloads.DEFAULT_TIE_EPS
    cos_t = 0.25
    d = np.array([math.sqrt(1.0 - cos_t * cos_t), 0.0, cos_t])
    bnd = box((0, 0, 0), (1, 1, 1))
    for dp, narrow, wide in ((0.5 * tie, True, True), (-0.5 * tie, True, True),
                             (2 * tie, False, True), (-2 * tie, False, True),
                             (5 * tie, False, True), (20 * tie, False, False)):
        X = np.array([0.2, 0.5, 1.0])
        E = X - (dp / cos_t) * d
        flags, r = _tie_case(orc, bnd, E, X, d, cos_t, dp)
        assert bool(flags & orc.F_NEAR_TIE) == narrow, dp
        assert bool(flags & orc.F_NEAR_TIE_WIDE) == wide, dp
        # the geometry is what was built: the ray meets the face after 5 or 6 steps
        assert r["nbtir"][0] == 1 and r["status"][0] == orc.TRUNCATED


def test_near_tie_window_is_perpendicular_distance_sphere(orc):
    """The same construction at the unit sphere: the step end sits at
    perpendicular distance dp from the surface point X where the ray crosses,
    with N(X) . d = 1/4."""
    tie = workloads.DEFAULT_TIE_EPS
    cos_t = 0.25
    N = np.array([0.36, -0.48, 0.8])  # unit
    t = np.cross(N, [0.0, 0.0, 1.0])
    t /= np.linalg.norm(t)
    d = cos_t * N + math.sqrt(1 - cos_t * cos_t) * t
    for dp, narrow in ((0.5 * tie, True), (-0.5 * tie, True), (2 * tie, False),
                       (-2 * tie, False)):
        X = N.copy()
        E = X - (dp / cos_t) * d
        flags, r = _tie_case(orc, sphere(1.0), E, X, d, cos_t, dp)
        assert bool(flags & orc.F_NEAR_TIE) == narrow, dp
        assert r["nbtir"][0] == 1


def test_near_grazing_window_into_higher_index(orc):
    """Eq. (10) takes sgn(N.I): a ray entering higher index (mu < 1) nearly
    along the isoindicial surface is refracted to one side of it or the other
    by the sign of a tiny N.I.  In the stratified medium n = 1.5 + 0.2 z
    (N = z) a ray launched inside with I_z = s takes a first step with mu = 1
    (no bend) and meets its second decision with mu = n(P_0)/n(P_1) < 1 and
    N.I = s exactly.  Flagged for |s| < crit_rad, also at ten times that in
    the wide bit; a ray going down (mu > 1) is a TIR case, never flagged as
    grazing."""
    crit = workloads.DEFAULT_CRIT_RAD
    med = linear_slab(1.5, 0.2)
    for s, narrow, wide in ((0.5 * crit, True, True), (2 * crit, False, True),
                            (5 * crit, False, True), (20 * crit, False, False),
                            (-0.5 * crit, False, False)):
        d = np.array([[math.sqrt(1.0 - s * s), 0.0, s]])
        P0 = np.array([[0.3, 0.5, 0.5]])
        r = orc.trace(med, (P0, d), P(1e-3, max_steps=2))
        f = int(r["flags"][0])
        assert bool(f & orc.F_NEAR_GRAZING) == narrow, s
        assert bool(f & orc.F_NEAR_GRAZING_WIDE) == wide, s
        if s < 0:
            assert r["ntir"][0] == 1  # mu > 1 at grazing: reflected, Eq. (19)
        else:
            assert r["ntir"][0] == 0
