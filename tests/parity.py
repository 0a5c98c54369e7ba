"""Element-by-element comparison of GPU results with the FP64 oracle.

The bar, per ray, on the same seeded inputs (the pass rule):
  - status, interior TIR count and surface TIR count identical;
  - exit position within pos_tol * aperture;
  - exit direction, as it leaves the medium, within dir_tol rad;
except
  - rays the oracle flags near-critical: some refraction/TIR decision within
    crit_rad (1e-6 rad) of the critical angle (counted, exempt);
  - rays the oracle flags near-grazing: a refraction into higher index with
    |N.I| < crit_rad, where the sgn(N.I) of Eq. (10) alone decides on which
    side of the isoindicial surface the ray continues (counted, exempt; the
    window is pinned on the oracle).
Nothing else is set aside: near-tie rays (a step of the oracle ended within
tie_eps of the enclosing surface, so "full step or cut" was decided by the
last bits) meet every check; only their step count may differ.  Step counts
are reported, not part of the bar.

Diagnostics, reported beside the pass/fail counts: the exit direction error
measured inside the medium (the final refraction's gain n_in cos t_in /
(n_amb cos t_out), Snell's law differentiated, divided out), and how many of
the failing rays the oracle marks in its ten times wider windows.
"""
from __future__ import annotations

import math

import numpy as np

F_NEAR_CRITICAL = 1
F_NEAR_TIE = 16
F_NEAR_GRAZING = 32
EXEMPT = F_NEAR_CRITICAL | F_NEAR_TIE | F_NEAR_GRAZING
WIDE = 64 | 128 | 256  # the same windows ten times wider


def angle_between(a, b):
    a = a / np.maximum(np.linalg.norm(a, axis=1, keepdims=True), 1e-300)
    b = b / np.maximum(np.linalg.norm(b, axis=1, keepdims=True), 1e-300)
    return 2.0 * np.arcsin(np.clip(np.linalg.norm(a - b, axis=1) / 2.0, 0.0, 1.0))


def surface_normal(boundary, P, tol=1e-7):
    """Outward unit normal of the enclosing surface at points P (m,3) lying on
    it; NaN rows where a point is not on the surface within tol."""
    kind, q = boundary["kind"], np.asarray(boundary["params"], dtype=np.float64)
    N = np.full(P.shape, np.nan)
    if kind == "sphere":
        o = P - q[:3]
        r = np.linalg.norm(o, axis=1)
        on = np.abs(r - q[3]) < tol
        N[on] = o[on] / r[on, None]
    elif kind == "box":
        lo, hi = q[:3], q[3:6]
        for a in range(3):
            for side, val in ((-1.0, lo[a]), (1.0, hi[a])):
                on = np.abs(P[:, a] - val) < tol
                N[on] = 0.0
                N[on, a] = side
    elif kind == "cylinder":
        cx, cy, r0, z0, z1 = q[:5]
        o = P[:, :2] - np.array([cx, cy])
        r = np.linalg.norm(o, axis=1)
        side = np.abs(r - r0) < tol
        N[side, :2] = o[side] / r[side, None]
        N[side, 2] = 0.0
        for sgn, zz in ((-1.0, z0), (1.0, z1)):
            cap = np.abs(P[:, 2] - zz) < tol
            N[cap] = np.array([0.0, 0.0, sgn])
    return N


def exit_gain(spec, orc, n_index):
    """How much the final refraction out of the medium magnifies an error of
    the direction inside.  Snell's law n_in sin t_in = n_amb sin t_out (the
    scalar form of Eqs. (9)-(10)) differentiates to
    d t_out / d t_in = n_in cos t_in / (n_amb cos t_out); near the critical
    angle cos t_out -> 0 and a direction that is 1e-6 rad off inside leaves
    the surface 1e-4 rad off.  n_index(P) gives n at the exit points.
    Returns the factor (>= 1) per ray, 1 where the exit point is not on the
    enclosing surface (an exit plane) or the ray did not leave."""
    gain = np.ones(len(orc["status"]))
    ex = orc["status"] == 0
    if not ex.any():
        return gain
    P, D = orc["P"][ex], orc["D"][ex]
    N = surface_normal(spec["boundary"], P)
    ok = np.isfinite(N).all(axis=1)
    if not ok.any():
        return gain
    cos_out = np.abs(np.einsum("ij,ij->i", D[ok], N[ok]) /
                     np.linalg.norm(D[ok], axis=1))
    mu = n_index(P[ok]) / spec["n_amb"]
    sin2_out = 1.0 - cos_out ** 2
    mu_cos_in = np.sqrt(np.maximum(mu ** 2 - sin2_out, 0.0))
    g = mu_cos_in / np.maximum(cos_out, 1e-12)
    idx = np.nonzero(ex)[0][ok]
    gain[idx] = np.maximum(1.0, g)
    return gain


def compare(orc, gpu, aperture, pos_tol=1e-4, dir_tol=1e-4, spec=None):
    """Per-ray comparison under the pass rule of this module.  spec (the
    medium) given: also the inside-the-medium direction error (diagnostic)."""
    n = len(orc["status"])
    gain = np.ones(n)
    if spec is not None:
        import oracle

        gain = np.asarray(exit_gain(spec, orc, lambda P: oracle.evaluate(spec, P)[0]))
    fo, fg = orc["flags"], gpu["flags"]
    crit = (fo & F_NEAR_CRITICAL) != 0
    graze = (fo & F_NEAR_GRAZING) != 0
    tie = (fo & F_NEAR_TIE) != 0
    dsteps = orc["steps"].astype(np.int64) - gpu["steps"].astype(np.int64)
    checked = ~crit & ~graze
    st = orc["status"] == gpu["status"]
    tir = orc["ntir"] == gpu["ntir"]
    btir = orc["nbtir"] == gpu["nbtir"]
    pe = np.linalg.norm(orc["P"] - gpu["P"], axis=1)
    de = angle_between(orc["D"], gpu["D"])
    de_in = de / gain
    same = checked & st
    bad_pos = same & (pe > pos_tol * aperture)
    bad_dir = same & (de > dir_tol)
    fail = checked & (~st | ~tir | ~btir | bad_pos | bad_dir)
    wide = (fo & WIDE) != 0

    def mx(v, m):
        return float(v[m].max()) if m.any() else 0.0

    def pct(v, m, q):
        return float(np.percentile(v[m], q)) if m.any() else 0.0

    rep = {
        "n": n,
        "checked": int(checked.sum()),
        "fail": int(fail.sum()),
        "exempt_critical": int(crit.sum()),
        "exempt_grazing": int((graze & ~crit).sum()),
        "tie_checked": int((tie & checked).sum()),
        "tie_steps_differ": int((tie & checked & (dsteps != 0)).sum()),
        "flagged_oracle_critical": int(crit.sum()),
        "flagged_oracle_tie": int(tie.sum()),
        "flagged_oracle_grazing": int(graze.sum()),
        "flagged_gpu_critical": int(((fg & F_NEAR_CRITICAL) != 0).sum()),
        "flagged_gpu_tie": int(((fg & F_NEAR_TIE) != 0).sum()),
        "flagged_gpu_grazing": int(((fg & F_NEAR_GRAZING) != 0).sum()),
        "status_mismatch": int((checked & ~st).sum()),
        "tir_mismatch": int((checked & ~tir).sum()),
        "btir_mismatch": int((checked & ~btir).sum()),
        "pos_fail": int(bad_pos.sum()),
        "dir_fail": int(bad_dir.sum()),
        "fail_in_wide_window": int((fail & wide).sum()),
        "steps_mismatch": int((checked & (dsteps != 0)).sum()),
        "steps_absmax": int(np.abs(dsteps[checked]).max()) if checked.any() else 0,
        "pos_err_max": mx(pe, same),
        "pos_err_p99": pct(pe, same, 99),
        "pos_err_p50": pct(pe, same, 50),
        "dir_err_max": mx(de, same),
        "dir_err_p99": pct(de, same, 99),
        "dir_err_inside_max": mx(de_in, same),
        "exempt_pos_err_max": mx(pe, ~checked),
        "tir_total_oracle": int(orc["ntir"].sum()),
        "btir_total_oracle": int(orc["nbtir"].sum()),
    }
    rep["bad_rays"] = np.nonzero(fail)[0][:20].tolist()
    return rep


def assert_parity(rep):
    """The pass rule: no checked ray fails."""
    msg = {k: v for k, v in rep.items()}
    assert rep["fail"] == 0, msg
    assert rep["status_mismatch"] == 0 and rep["tir_mismatch"] == 0, msg
    assert rep["btir_mismatch"] == 0 and rep["pos_fail"] == 0 and rep["dir_fail"] == 0, msg


def stat_compare(orc, gpu, n_bins=8, face_axis=2):
    """Distribution-level agreement for media where single rays are chaotic:
    the oracle's own exits move under 1e-11 launch perturbations, so only the
    statistics of the exit state are reproducible.  Two-sample comparisons:
    status counts, mean event counts and steps (in units of their standard
    error), mean exit direction, and a chi-square of the exit points over an
    n_bins x n_bins histogram of the exit face z = 1."""
    n = len(orc["status"])
    rep = {"n": n}
    for s in range(6):
        a, b = int((orc["status"] == s).sum()), int((gpu["status"] == s).sum())
        rep[f"status{s}"] = (a, b)
    z = {}
    for k in ("ntir", "nbtir", "steps"):
        a, b = orc[k].astype(float), gpu[k].astype(float)
        se = math.sqrt(a.var() / n + b.var() / n) + 1e-300
        z[k] = (b.mean() - a.mean()) / se
        rep[f"mean_{k}"] = (float(a.mean()), float(b.mean()))
    for i, c in enumerate("xyz"):
        a, b = orc["D"][:, i], gpu["D"][:, i]
        se = math.sqrt(a.var() / n + b.var() / n) + 1e-300
        z[f"dir_{c}"] = (b.mean() - a.mean()) / se
    rep["z"] = {k: round(float(v), 3) for k, v in z.items()}

    def hist(r):
        m = (r["status"] == 0) & (np.abs(r["P"][:, face_axis] - 1.0) < 1e-9)
        h, _, _ = np.histogram2d(r["P"][m, 0], r["P"][m, 1], bins=n_bins, range=[[0, 1], [0, 1]])
        return h.ravel()

    ha, hb = hist(orc), hist(gpu)
    keep = (ha + hb) > 0
    chi2 = float((((ha - hb) ** 2)[keep] / (ha + hb)[keep]).sum())
    dof = int(keep.sum()) - 1
    rep["chi2"], rep["chi2_dof"] = round(chi2, 2), dof
    return rep


def assert_stats(rep, z_max=4.5):
    for s in range(6):
        a, b = rep[f"status{s}"]
        assert abs(a - b) <= 4.0 * math.sqrt(a + b + 1) + 2, rep
    for k, v in rep["z"].items():
        assert abs(v) <= z_max, (k, rep)
    # chi-square two-sample test: a 5-sigma bound on the statistic
    dof = max(rep["chi2_dof"], 1)
    assert rep["chi2"] <= dof + 5.0 * math.sqrt(2.0 * dof), rep


def ill_conditioned(orc_trace, spec, rays, params, delta=1e-9, tol=1e-5, turn=0.0):
    """Rays whose oracle result is itself unstable: shifting the launch point
    by delta (x and y) -- or, with turn > 0, turning the launch direction by
    turn radians -- changes the event counts or moves the exit state by more
    than tol.  Returns a boolean mask."""
    o = orc_trace(spec, rays, params)

    def unstable(o2):
        return ((o["status"] != o2["status"]) | (o["ntir"] != o2["ntir"]) |
                (o["nbtir"] != o2["nbtir"]) |
                (np.linalg.norm(o["P"] - o2["P"], axis=1) > tol) |
                (angle_between(o["D"], o2["D"]) > tol))

    P = rays[0].copy()
    P[:, 0] += delta
    P[:, 1] -= delta
    bad = unstable(orc_trace(spec, (P, rays[1]), params))
    if turn > 0.0:
        # a unit vector across each direction (a fixed oblique axis crossed with D)
        D = rays[1]
        t = np.cross(D, np.array([0.3, 0.5, 0.81]))
        ln = np.linalg.norm(t, axis=1)
        t[ln < 1e-3] = np.cross(D[ln < 1e-3], np.array([1.0, 0.0, 0.0]))
        t /= np.linalg.norm(t, axis=1)[:, None]
        D2 = D + turn * t
        D2 /= np.linalg.norm(D2, axis=1)[:, None]
        bad |= unstable(orc_trace(spec, (rays[0], D2), params))
    return bad


def exempt(rep_input, mask):
    """Drop the rays of mask from a result dict (both sides)."""
    return {k: (v[~mask] if hasattr(v, "__len__") and len(v) == len(mask) else v)
            for k, v in rep_input.items()}
