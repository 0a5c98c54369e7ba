"""Pins of the oracle's freeform cylindrical lens of Sec. V: an index made of
Fringe Zernike polynomials across the lens times Legendre polynomials along
it, n = n0 + dn sum c Z_j(x', y') V_l(z').

The oracle evaluates Z_j from the general radial formula in polar form and
V_l by the three-term recursion; the checks below use other things: the
Cartesian forms of the sixteen Fringe terms, numpy's Legendre series,
orthogonality on the unit disc and on [-1, 1], finite differences, the
bound the paper's coefficients put on the index, and exact discrete
invariants of the vectorial law under the symmetries a term keeps.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre

import workloads

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def cartesian_fringe(j, u, v):
    """The sixteen unnormalised Fringe Zernike polynomials written out in x, y."""
    r2 = u * u + v * v
    return {1: np.ones_like(u), 2: u, 3: v, 4: 2 * r2 - 1, 5: u * u - v * v, 6: 2 * u * v,
            7: (3 * r2 - 2) * u, 8: (3 * r2 - 2) * v, 9: 6 * r2 * r2 - 6 * r2 + 1,
            10: u ** 3 - 3 * u * v * v, 11: 3 * u * u * v - v ** 3,
            12: (4 * r2 - 3) * (u * u - v * v), 13: (4 * r2 - 3) * 2 * u * v,
            14: (10 * r2 * r2 - 12 * r2 + 3) * u, 15: (10 * r2 * r2 - 12 * r2 + 3) * v,
            16: 20 * r2 ** 3 - 30 * r2 * r2 + 12 * r2 - 1}[j]


# (radial order, azimuthal order) of the Fringe terms, for their norms
FRINGE_NM = {1: (0, 0), 2: (1, 1), 3: (1, 1), 4: (2, 0), 5: (2, 2), 6: (2, 2), 7: (3, 1),
             8: (3, 1), 9: (4, 0), 10: (3, 3), 11: (3, 3), 12: (4, 2), 13: (4, 2), 14: (5, 1),
             15: (5, 1), 16: (6, 0)}


def single(j, l, rho_max=2.0, z_max=3.0, c=1.0):
    """One term with n0 = 0 and dn = 1, so that n is the term itself."""
    return workloads.zernike_lens(-1.0, 1.0, rho_max, z_max, terms=((j, l, c),))


def lens_points(n, rho_max, z_max, seed):
    rng = np.random.default_rng(seed)
    r = rho_max * np.sqrt(rng.random(n))
    a = 2 * math.pi * rng.random(n)
    P = np.column_stack([r * np.cos(a), r * np.sin(a), z_max * rng.random(n)])
    P[:4, :2] = 0.0  # on the axis, where the polar angle is undefined
    return P


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_fringe_terms_match_cartesian_and_legendre_forms(orc, l):
    P = lens_points(300, 2.0, 3.0, seed=50 + l)
    u, v, w = P[:, 0] / 2.0, P[:, 1] / 2.0, 2 * P[:, 2] / 3.0 - 1
    Vl = legendre.legval(w, [0] * l + [1])
    for j in range(1, 17):
        n, _ = orc.evaluate(single(j, l), P)
        assert np.allclose(n, cartesian_fringe(j, u, v) * Vl, rtol=0, atol=1e-13), (j, l)


def test_zernike_gradient_matches_finite_difference(orc):
    h = 1e-6
    for j in range(1, 17):
        for l in (0, 3):
            med = single(j, l)
            P = lens_points(60, 2.0, 3.0, seed=60 + j)
            _, g = orc.evaluate(med, P)
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                fd = (orc.evaluate(med, P + e)[0] - orc.evaluate(med, P - e)[0]) / (2 * h)
                assert np.allclose(g[:, a], fd, rtol=1e-6, atol=1e-7), (j, l, a)


def test_fringe_terms_are_orthogonal_on_the_unit_disc(orc):
    """int_disc Z_i Z_j dA = 0 for i != j and pi / (n + 1) (m = 0) or
    pi / (2 (n + 1)) (m > 0) for i = j -- Gauss-Legendre in rho (weight rho)
    times the trapezoidal rule in theta, both exact at these degrees."""
    x, wx = legendre.leggauss(12)
    rho, wr = (x + 1) / 2, wx / 2 * (x + 1) / 2
    th = 2 * math.pi * np.arange(32) / 32
    R, T = np.meshgrid(rho, th, indexing="ij")
    W = (wr[:, None] * np.full(32, 2 * math.pi / 32)[None, :]).ravel()
    P = np.column_stack([R.ravel() * np.cos(T.ravel()), R.ravel() * np.sin(T.ravel()),
                         np.full(R.size, 1.5)])  # rho_max = 1, z' = 0
    Z = np.stack([orc.evaluate(single(j, 0, rho_max=1.0), P)[0] for j in range(1, 17)])
    G = (Z * W) @ Z.T
    want = np.diag([math.pi / ((FRINGE_NM[j][0] + 1) * (1 if FRINGE_NM[j][1] == 0 else 2))
                    for j in range(1, 17)])
    assert np.allclose(G, want, rtol=0, atol=1e-12)


def test_legendre_factor_is_orthogonal_on_the_lens_thickness(orc):
    """int_{-1}^{1} V_k V_l dz' = 2 / (2 l + 1) delta_kl along the axis."""
    x, wx = legendre.leggauss(8)
    P = np.column_stack([np.zeros(8), np.zeros(8), (x + 1) / 2 * 3.0])  # z_max = 3
    V = np.stack([orc.evaluate(single(1, l), P)[0] for l in range(4)])
    assert np.allclose((V * wx) @ V.T, np.diag([2 / (2 * l + 1) for l in range(4)]), atol=1e-13)


@pytest.mark.parametrize("n_lo,n_hi", [(1.5148, 1.5162), (1.5261, 1.5608)])
def test_paper_lens_stays_between_its_parent_indices(orc, n_lo, n_hi):
    """The paper's coefficients sum to 0.9998 in absolute value and every
    |Z_j| <= 1 on the disc, |V_l| <= 1 on [-1, 1]: a binary composition of
    the two parent materials never leaves [n_lo, n_hi]."""
    assert sum(abs(c) for _, _, c in workloads.ZERNIKE_TERMS) == pytest.approx(0.9998)
    spec = workloads.zernike_lens(n_lo, n_hi)
    n, _ = orc.evaluate(spec, lens_points(20000, 4.2, 2.5, seed=70))
    assert n.min() >= n_lo and n.max() <= n_hi
    assert n.max() - n.min() > 0.5 * (n_hi - n_lo)


def segments(path, dL0):
    """Interior segments of a path (entry point on): start points, unit
    directions, and the index that sized each full step (n = dL0 / length,
    Eq. (4)); the last segment, cut at the surface, is dropped."""
    pts = path[1:]
    seg = pts[1:] - pts[:-1]
    ln = np.linalg.norm(seg, axis=1)
    return pts[:-2], seg[:-1] / ln[:-1, None], dL0 / ln[:-1]


@pytest.mark.parametrize("case", ["axisymmetric", "z_invariant", "mirror"])
def test_symmetric_lenses_keep_their_exact_discrete_invariants(orc, case):
    """Rotationally symmetric terms (Z4, Z9, Z16) -> n (P x R)_z is conserved
    at every Snell step; terms without z dependence (l = 0) -> n R_z; cosine
    terms (even in y) -> a ray launched in the plane y = 0 stays in it.  Rays
    without TIR (the march's literal n_{i-1} = n(P_{i-1}) rescales the
    momentum at a TIR step) and without boundary reflection."""
    terms = {"axisymmetric": ((4, 1, 0.3), (9, 0, -0.2), (16, 2, 0.1), (9, 3, 0.2)),
             "z_invariant": ((5, 0, -0.2368), (8, 0, 0.3), (11, 0, -0.17), (12, 0, 0.1)),
             "mirror": ((5, 0, -0.2368), (12, 1, 0.2), (9, 2, 0.1), (2, 1, 0.3))}[case]
    med = workloads.zernike_lens(1.5261, 1.5608, terms=terms)
    P0, d0 = workloads.zernike_rays(40, seed=71)
    if case == "mirror":
        P0[:, 1] = 0.0
        d0[:, 1] = 0.0
        d0 /= np.linalg.norm(d0, axis=1)[:, None]
    prm = workloads.trace_params(2e-3, 100000)
    checked = 0
    for i in range(40):
        path, res = orc.trace_path(med, P0[i], d0[i], prm)
        if res["status"] != orc.EXITED or res["nbtir"] or res["ntir"] or len(path) < 20:
            continue
        if case == "mirror":
            assert np.abs(path[:, 1]).max() < 1e-11, i
        else:
            p, R, n = segments(path, prm["dL0"])
            inv = n * np.cross(p, R)[:, 2] if case == "axisymmetric" else n * R[:, 2]
            assert np.abs(inv - inv[0]).max() < 1e-11 * max(1.0, abs(inv[0])), (i, case)
        checked += 1
    assert checked >= 10


def test_figure_ray_enters_reflects_and_leaves(orc):
    """The ray of Fig. 3(a) -- from (1, -5, -1.5) at theta = 80 deg, phi = 110
    deg -- enters through the lens face z = 0, is totally reflected at the
    lens wall and leaves the lens, as the figure's caption describes."""
    P0, d0 = workloads.zernike_rays(1, seed=0)
    path, res = orc.trace_path(workloads.zernike_lens(), P0[0], d0[0],
                               workloads.trace_params(1e-3, 100000))
    assert res["status"] == orc.EXITED
    assert path[1][2] == pytest.approx(0.0, abs=1e-12) and np.hypot(*path[1][:2]) < 4.2
    assert res["nbtir"] >= 1 and res["ntir"] == 0
