"""Oracle of the paper's first design example (Sec. VI): the cylindrical
N2P-GRIN lens, its aberration score and the successive-refinement search.

TEST INFRASTRUCTURE ONLY: the independent reference the GPU design sweep is
checked against.  Only ``tests/``, the smoke check, the CPU-baseline leg of
the benchmark and the script that writes ``tests/golden/n2p_design.json``
may use it.  It shares no code with the GPU library; the lens and the launch
states come from ``workloads.py`` like every other input.

Every ray is traced by the FP64 C oracle (``oracle.trace``); the rest is plain
numpy written from the equations:
  - z_Int: where the straight line the ray follows after leaving the lens
    crosses the optical axis (the paper's definition under Eq. (29)); only
    the forward part of the line counts;
  - LSA_i = F - z_Int,i (Eq. (29)); RMSE_LSA = sqrt(mean LSA_i^2) (Eq. (28));
  - the search: sample a grid of (beta, gamma) over a box, keep the best,
    shrink the box around it, repeat (the strategy stated in Sec. VI).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import workloads


def axis_crossing(P, D):
    """z where the exit line P + s D (s >= 0) meets the z axis, for rays in
    the yz-plane; +inf when it never does (the ray heads away from the axis
    or runs parallel to it)."""
    P = np.asarray(P, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    z = np.full(P.shape[0], np.inf)
    for i in range(P.shape[0]):
        y, dy = P[i, 1], D[i, 1]
        if dy != 0.0:
            s = -y / dy  # y + s dy = 0
            if s > 0.0:
                z[i] = P[i, 2] + s * D[i, 2]
    return z


def rmse_lsa(beta, gamma, L, R=1.0, F=2.0, N=10, h_max=0.995, dL0=1e-4, max_steps=10 ** 7,
             want_z=False):
    """RMSE of the longitudinal spherical aberration of the N design rays
    (Eqs. (28)-(29)); +inf if a ray does not exit or never crosses the axis."""
    lens = workloads.n2p_lens(beta, gamma, L, R, F)
    rays = workloads.n2p_rays(L, N, R, h_max)
    res = oracle.trace(lens, rays, {"dL0": dL0, "max_steps": max_steps}, n_threads=1)
    z = axis_crossing(res["P"], res["D"])
    z[res["status"] != oracle.EXITED] = np.inf
    lsa = F - z
    e = float(np.sqrt(np.mean(lsa ** 2))) if np.all(np.isfinite(z)) else np.inf
    return (e, z) if want_z else e


def sweep(bg, L, threads=8, **kw):
    """rmse_lsa for each (beta, gamma) row of bg, candidates spread over threads
    (the C oracle releases the interpreter lock while it traces)."""
    bg = np.asarray(bg, dtype=np.float64).reshape(-1, 2)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return np.array(list(ex.map(lambda p: rmse_lsa(p[0], p[1], L, **kw), bg)))


def design(L, beta=(0.2, 2.5), gamma=(0.5, 8.0), grid=33, window=3, levels=12, tol=1e-5,
           threads=8, **kw):
    """Successive refinement: a grid x grid sample of the box, the best point,
    the next box +-window grid spacings around it (clipped at > 0), until the
    box is narrower than tol in both parameters or `levels` samples ran.
    Returns (beta, gamma, rmse, list of per-level bests)."""
    b0, b1 = beta
    g0, g1 = gamma
    best = (np.nan, np.nan, np.inf)
    levels_out = []
    for _ in range(levels):
        bs = [b0 + (b1 - b0) * i / (grid - 1) for i in range(grid)]
        gs = [g0 + (g1 - g0) * j / (grid - 1) for j in range(grid)]
        cand = [(b, g) for b in bs for g in gs]
        e = sweep(cand, L, threads=threads, **kw)
        k = int(np.argmin(e))
        if e[k] < best[2]:
            best = (cand[k][0], cand[k][1], float(e[k]))
        levels_out.append(best)
        if b1 - b0 < tol and g1 - g0 < tol:
            break
        db = (b1 - b0) / (grid - 1)
        dg = (g1 - g0) / (grid - 1)
        b0, b1 = max(1e-6, best[0] - window * db), best[0] + window * db
        g0, g1 = max(1e-6, best[1] - window * dg), best[1] + window * dg
    return best[0], best[1], best[2], levels_out
