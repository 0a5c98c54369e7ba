"""Design loop of the cylindrical N2P-GRIN lens (Sec. VI of the paper).

The lens index is Eq. (27); a candidate (beta, gamma) is scored by the RMSE of
the longitudinal spherical aberration of N design rays (Eqs. (28)-(29)).  The
search is the paper's successive refinement: sample a grid of candidates over
the current (beta, gamma) box, keep the best, shrink the box around it, and
repeat.  Each refinement level is one GPU launch (``vrt_n2p_sweep``: one wave
per candidate, the plain FP64 march in every lane).

The paper states the strategy but not its grid, box or stopping rule; the
defaults below are this library's reading: a 33 x 33 grid over
beta in [0.2, 2.5], gamma in [0.5, 8], the next box spanning +-3 grid
spacings around the best candidate, until the box is narrower than 1e-5 in
both parameters or 12 levels have run.
"""
from __future__ import annotations

import numpy as np

import paper_2606_22655_amd as vrt


def refine(score, beta=(0.2, 2.5), gamma=(0.5, 8.0), grid=33, window=3, levels=12, tol=1e-5):
    """Successive refinement of a two-parameter score (lower is better).

    ``score(bg)`` maps an (m, 2) array of (beta, gamma) candidates to m
    scores.  Returns (beta, gamma, score, history) with one history row
    (beta, gamma, score, box width in beta, in gamma) per level."""
    blo, bhi = beta
    glo, ghi = gamma
    best = (np.nan, np.nan, np.inf)
    hist = []
    for _ in range(levels):
        bs = np.linspace(blo, bhi, grid)
        gs = np.linspace(glo, ghi, grid)
        B, G = np.meshgrid(bs, gs, indexing="ij")
        e = np.asarray(score(np.stack([B.ravel(), G.ravel()], axis=1)))
        k = int(np.argmin(e))
        if e[k] < best[2]:
            best = (float(B.ravel()[k]), float(G.ravel()[k]), float(e[k]))
        db, dg = bs[1] - bs[0], gs[1] - gs[0]
        hist.append((best[0], best[1], best[2], bhi - blo, ghi - glo))
        if bhi - blo < tol and ghi - glo < tol:
            break
        blo, bhi = max(1e-6, best[0] - window * db), best[0] + window * db
        glo, ghi = max(1e-6, best[1] - window * dg), best[1] + window * dg
    return best[0], best[1], best[2], np.array(hist)


def design_n2p(ctx, L, R=1.0, F=2.0, n_rays=10, h_max=0.995, dL0=None, max_steps=200000,
               stream=0, **search):
    """Optimise (beta, gamma) of the N2P lens of thickness L for focal
    distance F.  dL0 defaults to 1e-4 R (the paper's step).  A ray still in
    the lens after max_steps steps (trapped by TIR at the faces, as strong
    candidates are) makes its candidate invalid; the default is ~8x the
    steps a ray needs through the thickest lens of the paper (L = R).
    Returns a dict with beta, gamma, rmse_lsa, the refinement history, the
    candidates and ray-steps evaluated and the wall time."""
    import time

    import workloads

    lens_spec = workloads.n2p_lens(1.0, 1.0, L, R, F)
    y = workloads.n2p_heights(n_rays, R, h_max)
    P0, _ = workloads.n2p_rays(L, n_rays, R, h_max)
    z_launch = float(P0[0, 2])
    prm = vrt.make_params({"dL0": 1e-4 * R if dL0 is None else dL0, "max_steps": max_steps},
                          "fp64")
    lens = vrt.Medium(ctx, lens_spec)
    evals, steps = [0], [0]
    t0 = time.perf_counter()
    try:
        def score(bg):
            rm, st = vrt.vrt_n2p_sweep(lens.handle, bg, y, z_launch, prm, stream, want_steps=True)
            evals[0] += len(bg)
            steps[0] += int(st.sum())
            return rm

        b, g, e, hist = refine(score, **search)
    finally:
        lens.close()
    return {"beta": b, "gamma": g, "rmse_lsa": e, "history": hist, "evaluations": evals[0],
            "ray_steps": steps[0], "seconds": time.perf_counter() - t0}
