"""Seeded synthetic inputs for the constant-OPL ray march.

This module only *draws data*: medium parameters, index grids and ray launch
states.  It contains none of the ray-tracing arithmetic (no index evaluation,
no refraction, no stepping), so that the FP64 CPU oracle and the HIP path can
both consume exactly the same bits without sharing any of the method's code.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in
the order written in its docstring.  Inputs meant for the FP32 path are rounded
to float32 here and handed to both sides as the same values (the oracle reads
them as float64).

Media are plain dicts::

    {"kind": "luneburg" | "gaussian" | "linear" | "homogeneous" | "fiber" | "grid" |
             "spherical" | "n2p" | "zernike",
     "params": float64 array (layout per kind, see ``MEDIUM_PARAM_LAYOUT``),
     "boundary": {"kind": "box" | "sphere" | "cylinder", "params": float64 array},
     "n_amb": float,
     # grid media only:
     "grid": float32 array of shape (nz, ny, nx), x fastest,
     "grid_lo": (3,) float64, "grid_hi": (3,) float64}

Rays are ``(P0, d0)``: two (n, 3) float64 arrays (launch point, launch
direction).  Trace settings are a dict ``{"dL0", "max_steps", "eps_tan",
"crit_rad", "tie_eps", "exit_plane_z"}``.
"""
from __future__ import annotations

import math

import numpy as np

# Parameter layouts (documentation of the data format shared by both sides).
MEDIUM_PARAM_LAYOUT = {
    "homogeneous": "[n_h]",
    "linear": "[n0, gx, gy, gz]            n = n0 + g.P",
    "luneburg": "[R, cx, cy, cz]             n = sqrt(2 - |P-C|^2/R^2)",
    "fiber": "[n_c, Delta, R, cx, cy]       parabolic core about the z axis through (cx, cy)",
    "gaussian": "[n0, K, (A, sigma, cx, cy, cz) x K]",
    "grid": "[] (values in 'grid', nodes spanning grid_lo..grid_hi)",
    "spherical": "[a0, a1, a2, a3, cx, cy, cz]  Sec. V, Eq. (26) about (cx, cy, cz)",
    "n2p": "[R, F, beta, gamma]          Sec. VI, Eq. (27), axis z; lens = cylinder boundary",
    "zernike": "[n_lo, n_hi, rho_max, z_max, K, (j, l, c) x K]  Sec. V, Fringe Zernike j <= 16, "
               "Legendre l <= 3",
}
BOUNDARY_PARAM_LAYOUT = {
    "box": "[lox, loy, loz, hix, hiy, hiz]",
    "sphere": "[cx, cy, cz, r]",
    "cylinder": "[cx, cy, r, z0, z1]   axis along z",
}

DEFAULT_CRIT_RAD = 1e-6
DEFAULT_TIE_EPS = 1e-7


def trace_params(dL0, max_steps, eps_tan=0.0, crit_rad=DEFAULT_CRIT_RAD, exit_plane_z=None,
                 tie_eps=DEFAULT_TIE_EPS):
    return {"dL0": float(dL0), "max_steps": int(max_steps), "eps_tan": float(eps_tan),
            "crit_rad": float(crit_rad), "tie_eps": float(tie_eps),
            "exit_plane_z": None if exit_plane_z is None else float(exit_plane_z)}


def _f32(a):
    """Round to float32 and return float64 holding exactly those values."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def unit_box(n_amb=1.0):
    return {"kind": "box", "params": np.array([0, 0, 0, 1, 1, 1], dtype=np.float64)}


# ---------------------------------------------------------------------------
# Luneburg sphere, parallel beam (accuracy configuration, FP64)
# ---------------------------------------------------------------------------
def luneburg_beam(n_side=64, R=1.0, z0=-1.5, dL0=1e-3, max_steps=20000):
    """Luneburg sphere of radius R centred at the origin, n_amb = 1, beam along +z.

    Launch grid: cell-centred ``x, y = -R + (k + 1/2) * 2R/n_side`` on the plane
    z = z0; every ray has direction (0, 0, 1).  No random draws.
    """
    k = (np.arange(n_side, dtype=np.float64) + 0.5) * (2.0 * R / n_side) - R
    X, Y = np.meshgrid(k, k, indexing="xy")
    n = n_side * n_side
    P0 = np.stack([X.ravel(), Y.ravel(), np.full(n, z0)], axis=1)
    d0 = np.zeros((n, 3))
    d0[:, 2] = 1.0
    medium = {"kind": "luneburg", "params": np.array([R, 0.0, 0.0, 0.0]),
              "boundary": {"kind": "sphere", "params": np.array([0.0, 0.0, 0.0, R])},
              "n_amb": 1.0}
    return medium, (P0, d0), trace_params(dL0, max_steps)


def helix_fiber(n_c=1.38, Delta=0.2, R=5.0, rho0=4.0, L=55.0):
    """The helical ray of Sec. IV (Eq. (21), Fig. 2): a parabolic-index fiber
    of core index n_c and radius R along z in 0 <= z <= L, surrounded by the
    cladding index n_c sqrt(1 - 2 Delta) (also before the fiber face), and one
    ray launched so that it enters at P_I = (rho0, 0, 0) and winds on the
    cylinder of radius rho0.  With n^2 = n_c^2 - w^2 rho^2, w = n_c sqrt(2
    Delta) / R, a helix of radius rho0 needs tangential momentum w rho0 (seen
    in the cladding) and axial invariant b = sqrt(n_c^2 - 2 w^2 rho0^2); its
    closed form is (rho0 cos kz, rho0 sin kz, z) with k = w / b.  Returns
    (medium, (P0, d0) of shape (1, 3), {"rho0", "kappa"}).  No random draws."""
    ncl = n_c * math.sqrt(1.0 - 2.0 * Delta)
    w = n_c * math.sqrt(2.0 * Delta) / R
    b = math.sqrt(n_c ** 2 - 2.0 * w ** 2 * rho0 ** 2)
    s = w * rho0 / ncl
    d0 = np.array([[0.0, s, math.sqrt(1.0 - s * s)]])
    P0 = np.array([[rho0, 0.0, 0.0]]) - rho0 * d0
    medium = {"kind": "fiber", "params": np.array([n_c, Delta, R, 0.0, 0.0]),
              "boundary": {"kind": "cylinder", "params": np.array([0.0, 0.0, R, 0.0, L])},
              "n_amb": ncl}
    return medium, (P0, d0), {"rho0": rho0, "kappa": w / b}


# ---------------------------------------------------------------------------
# Launch states on the z = 0 face of the unit cube
# ---------------------------------------------------------------------------
def face_cone_rays(n_rays, seed, cone_deg):
    """Rays launched on the face z = 0 of the unit cube into a cone about +z.

    One draw u ~ U[0,1) of shape (n_rays, 4); row i belongs to ray i, so the
    first m rays are the same for every n_rays >= m.  Per ray:
    kx = floor(u0 2^23), ky = floor(u1 2^23), cos(theta) = 1 - u2 (1 - cos(cone)),
    phi = 2 pi u3.  Positions are x = (2k+1)/2^24, exactly representable in
    float32 and strictly inside (0, 1), so no ray starts on a cube edge.
    Directions are uniform in solid angle inside the cone (in the ambient
    medium) and rounded to float32.
    """
    rng = np.random.default_rng(seed)
    u = rng.random((n_rays, 4))
    kx = np.floor(u[:, 0] * (1 << 23))
    ky = np.floor(u[:, 1] * (1 << 23))
    ct = 1.0 - u[:, 2] * (1.0 - math.cos(math.radians(cone_deg)))
    ph = 2.0 * math.pi * u[:, 3]
    P0 = np.zeros((n_rays, 3))
    P0[:, 0] = (2.0 * kx + 1.0) / float(1 << 24)
    P0[:, 1] = (2.0 * ky + 1.0) / float(1 << 24)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    d0 = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    return _f32(P0), _f32(d0)


# ---------------------------------------------------------------------------
# Freeform analytic medium: unit cube, 1.5 + sum of Gaussian bumps
# ---------------------------------------------------------------------------
def gaussian_medium(seed=2, K=16, n0=1.5, amp=0.1, wmin=0.05, wmax=0.3, n_amb=1.0):
    """n = n0 + sum_k A_k exp(-|P - c_k|^2 / (2 sigma_k^2)) in the unit cube.

    Draw order: A ~ U(-amp, amp) [K]; sigma ~ U(wmin, wmax) [K]; c ~ U(0,1) [K x 3].
    All parameters rounded to float32.
    """
    rng = np.random.default_rng(seed)
    A = rng.uniform(-amp, amp, K)
    s = rng.uniform(wmin, wmax, K)
    c = rng.uniform(0.0, 1.0, (K, 3))
    p = [n0, float(K)]
    for k in range(K):
        p += [A[k], s[k], c[k, 0], c[k, 1], c[k, 2]]
    return {"kind": "gaussian", "params": _f32(np.array(p)),
            "boundary": unit_box(), "n_amb": float(n_amb)}


def gaussian_cube(n_rays=1 << 20, seed_medium=2, seed_rays=102, cone_deg=20.0,
                  dL0=5e-4, max_steps=60000):
    """Freeform analytic configuration: 16 seeded Gaussian bumps, 1M rays, 20 deg cone."""
    medium = gaussian_medium(seed_medium)
    rays = face_cone_rays(n_rays, seed_rays, cone_deg)
    return medium, rays, trace_params(dL0, max_steps)


# ---------------------------------------------------------------------------
# Discretized isoindicial medium: quantized smoothed-noise grid
# ---------------------------------------------------------------------------
def noise_grid(N=256, seed=3, sigma_vox=8.0, nmin=1.4, nmax=1.8, levels=32):
    """N^3 float32 index grid from periodic Gaussian-smoothed white noise.

    Draw order: w ~ N(0,1) [N, N, N] (axis order z, y, x).  Smoothing is exact
    periodic Gaussian filtering (multiplication of the FFT by
    exp(-2 pi^2 sigma^2 f^2), f in cycles per voxel).  The result is mapped
    affinely onto [nmin, nmax] and quantized to ``levels`` equally spaced values
    n = nmin + q (nmax - nmin)/(levels - 1), q = round(...).
    """
    import scipy.fft as sfft

    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N, N))
    W = sfft.rfftn(w, workers=-1)
    del w
    f = np.fft.fftfreq(N)
    fr = np.fft.rfftfreq(N)
    T = np.exp(-2.0 * math.pi ** 2 * sigma_vox ** 2 *
               (f[:, None, None] ** 2 + f[None, :, None] ** 2 + fr[None, None, :] ** 2))
    W *= T
    v = sfft.irfftn(W, s=(N, N, N), workers=-1)
    del W
    lo, hi = v.min(), v.max()
    v = (v - lo) / (hi - lo)
    q = np.rint(v * (levels - 1))
    n = nmin + q * ((nmax - nmin) / (levels - 1))
    return n.astype(np.float32)


def grid_medium(values, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), n_amb=1.0):
    values = np.ascontiguousarray(values, dtype=np.float32)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return {"kind": "grid", "params": np.zeros(0), "grid": values,
            "grid_lo": lo, "grid_hi": hi,
            "boundary": {"kind": "box", "params": np.concatenate([lo, hi])},
            "n_amb": float(n_amb)}


def quantized_grid_cube(n_rays=1 << 22, N=256, seed_grid=3, seed_rays=103,
                        cone_deg=30.0, dL0=5e-4, max_steps=60000):
    """Discretized configuration: 256^3 quantized grid, 4M rays, 30 deg cone."""
    medium = grid_medium(noise_grid(N, seed_grid))
    rays = face_cone_rays(n_rays, seed_rays, cone_deg)
    return medium, rays, trace_params(dL0, max_steps)


# ---------------------------------------------------------------------------
# Differentiable design configuration (index-grid parameters + target ring)
# ---------------------------------------------------------------------------
def design_problem(N=64, n_side=512, seed_grid=4, seed_target=204, n0=1.5, jitter=0.01,
                   ring_r=0.2, plane_z=1.2, dL0=5e-4, max_steps=60000):
    """N^3 grid 1.5 + 0.01 N(0,1) (seed 4), n_side^2 parallel rays along +z from
    cell centres of z = 0, exit plane z = plane_z, target points on a ring.

    Draw orders: grid w ~ N(0,1) [N,N,N]; target phi ~ U[0, 2pi) [n_side^2].
    """
    rng = np.random.default_rng(seed_grid)
    g = (n0 + jitter * rng.standard_normal((N, N, N))).astype(np.float32)
    medium = grid_medium(g)
    k = (np.arange(n_side, dtype=np.float64) + 0.5) / n_side
    X, Y = np.meshgrid(k, k, indexing="xy")
    n = n_side * n_side
    P0 = _f32(np.stack([X.ravel(), Y.ravel(), np.zeros(n)], axis=1))
    d0 = np.zeros((n, 3))
    d0[:, 2] = 1.0
    rt = np.random.default_rng(seed_target)
    phi = rt.uniform(0.0, 2.0 * math.pi, n)
    target = np.stack([0.5 + ring_r * np.cos(phi), 0.5 + ring_r * np.sin(phi)], axis=1)
    return medium, (P0, d0), trace_params(dL0, max_steps, exit_plane_z=plane_z), target


# ---------------------------------------------------------------------------
# Served mix: a Poisson stream of trace jobs against resident media
# ---------------------------------------------------------------------------
# ---------------------------------------------------------------------------
# Spherical freeform medium (Sec. V, Eq. (26)) and the N2P lens (Sec. VI)
# ---------------------------------------------------------------------------
def spherical_medium(a=(1.5, 1.0, -0.2, 0.3), center=(0.0, 0.0, 0.0)):
    """n = a0 + a1 G1 + a2 G2 + a3 G3 inside the unit sphere about `center`
    (r_max = 1), surroundings n = 1.  Default coefficients are the paper's."""
    c = np.asarray(center, dtype=np.float64)
    return {"kind": "spherical", "params": np.concatenate([np.asarray(a, dtype=np.float64), c]),
            "boundary": {"kind": "sphere", "params": np.concatenate([c, [1.0]])},
            "n_amb": 1.0}


def sphere_aimed_rays(n_rays, seed, r_launch=1.5, r_target=0.8):
    """Rays launched from the sphere of radius r_launch about the origin
    towards a point drawn uniformly in the ball of radius r_target.

    One draw u ~ U[0,1) of shape (n_rays, 5); row i belongs to ray i:
    launch direction (cos t = 1 - 2 u0, phi = 2 pi u1), target radius
    r_target u2^(1/3), target direction (1 - 2 u3, 2 pi u4).  Rounded to
    float32.
    """
    rng = np.random.default_rng(seed)
    u = rng.random((n_rays, 5))

    def unit(ct, ph):
        st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
        return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)

    P0 = r_launch * unit(1.0 - 2.0 * u[:, 0], 2.0 * math.pi * u[:, 1])
    T = (r_target * np.cbrt(u[:, 2]))[:, None] * unit(1.0 - 2.0 * u[:, 3], 2.0 * math.pi * u[:, 4])
    d0 = T - P0
    d0 /= np.linalg.norm(d0, axis=1)[:, None]
    return _f32(P0), _f32(d0)


# Sec. V: the corrective freeform cylindrical lens, Fringe Zernike x Legendre
ZERNIKE_TERMS = ((5, 0, -0.2368), (8, 0, 0.0249), (9, 0, 0.0011), (11, 0, -0.0078),
                 (12, 0, -0.0013), (8, 1, 0.5548), (11, 1, -0.1731))


def zernike_lens(n_lo=1.5261, n_hi=1.5608, rho_max=4.2, z_max=2.5, terms=ZERNIKE_TERMS):
    """n = n0 + dn sum c Z_j(x/rho_max, y/rho_max) V_l(2z/z_max - 1) in the
    cylinder rho <= rho_max, 0 <= z <= z_max, in air (the paper's coefficients
    and geometry)."""
    t = np.asarray(terms, dtype=np.float64).ravel()
    return {"kind": "zernike",
            "params": np.concatenate([[n_lo, n_hi, rho_max, z_max, len(terms)], t]),
            "boundary": {"kind": "cylinder", "params": np.array([0.0, 0.0, rho_max, 0.0, z_max])},
            "n_amb": 1.0}


def zernike_rays(n_rays, seed, rho_max=4.2, z_max=2.5):
    """The paper's launch of Fig. 3(a) -- P0 = (1, -5, -1.5), theta0 = 80 deg,
    phi0 = 110 deg -- followed by n_rays - 1 rays from the plane z = -0.5
    (uniform in the disc of radius rho_max) to points uniform in the lens
    volume.  One draw u ~ U[0,1) of shape (n_rays, 5).  Rounded to float32."""
    rng = np.random.default_rng(seed)
    u = rng.random((n_rays, 5))
    r0 = rho_max * np.sqrt(u[:, 0])
    a0 = 2 * math.pi * u[:, 1]
    P0 = np.stack([r0 * np.cos(a0), r0 * np.sin(a0), np.full(n_rays, -0.5)], axis=1)
    r1 = 0.95 * rho_max * np.sqrt(u[:, 2])
    a1 = 2 * math.pi * u[:, 3]
    T = np.stack([r1 * np.cos(a1), r1 * np.sin(a1), z_max * u[:, 4]], axis=1)
    d0 = T - P0
    d0 /= np.linalg.norm(d0, axis=1)[:, None]
    th, ph = math.radians(80.0), math.radians(110.0)
    P0[0] = (1.0, -5.0, -1.5)
    d0[0] = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
    return _f32(P0), _f32(d0)


def n2p_lens(beta, gamma, L, R=1.0, F=2.0):
    """Cylindrical N2P-GRIN lens of radius R, focal distance F and thickness L
    occupying 0 <= rho <= R, -L <= z <= 0, in air."""
    return {"kind": "n2p", "params": np.array([R, F, beta, gamma], dtype=np.float64),
            "boundary": {"kind": "cylinder", "params": np.array([0.0, 0.0, R, -L, 0.0])},
            "n_amb": 1.0}


def n2p_heights(N=10, R=1.0, h_max=0.995):
    """Ray heights of the design: N rays on the y axis, uniformly spaced,
    excluding y = 0, the highest at h_max R:  y_i = h_max R i / N, i = 1..N."""
    return h_max * R * np.arange(1, N + 1, dtype=np.float64) / N


def n2p_rays(L, N=10, R=1.0, h_max=0.995, gap=0.1):
    """Launch states of the design rays: parallel to the axis (+z), from
    (0, y_i, -L - gap R) in the air before the lens."""
    y = n2p_heights(N, R, h_max)
    P0 = np.stack([np.zeros(N), y, np.full(N, -L - gap * R)], axis=1)
    d0 = np.tile([0.0, 0.0, 1.0], (N, 1))
    return P0, d0


def served_media(grid_sizes=(128, 160, 192, 256)):
    """Eight media: four Gaussian-bump cubes (seeds 500..503) and four quantized
    grids (seeds 504..507) with the given edge sizes."""
    media = [gaussian_medium(500 + i) for i in range(4)]
    for i, N in enumerate(grid_sizes):
        media.append(grid_medium(noise_grid(N, 504 + i)))
    return media


def served_jobs(n_jobs=10000, seed_arrival=5, seed_sizes=105, rate_hz=100.0,
                min_rays=1000, max_rays=4_000_000, n_media=8):
    """Job stream: Poisson arrivals (exponential gaps, seed 5), ray counts
    log-uniform in [min_rays, max_rays] (seed 105, draw order: log-size [n],
    medium id [n], ray seed [n])."""
    ra = np.random.default_rng(seed_arrival)
    gaps = ra.exponential(1.0 / rate_hz, n_jobs)
    t = np.cumsum(gaps)
    rs = np.random.default_rng(seed_sizes)
    size = np.exp(rs.uniform(math.log(min_rays), math.log(max_rays), n_jobs)).astype(np.int64)
    med = rs.integers(0, n_media, n_jobs)
    rseed = rs.integers(0, 2 ** 31 - 1, n_jobs)
    return [{"t_arrival": float(t[j]), "n_rays": int(size[j]), "medium": int(med[j]),
             "ray_seed": int(rseed[j])} for j in range(n_jobs)]
