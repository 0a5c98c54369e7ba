"""GPU: gradient of the exit-plane loss with respect to the node values of a
grid medium (vrt_grid_loss_grad, the differentiable design configuration:
64^3 grid 1.5 + 0.01 N(0,1), parallel rays along +z, exit plane z = 1.2,
targets on a ring).

The march is piecewise smooth in the node values: the gradient is that of the
discrete march with its branch pattern fixed.  Finite differences are
compared per ray, only on rays whose difference quotient is in its linear
regime -- same status and TIR counts at v +- h and v +- h/2, and the two
quotients agreeing -- since near-critical refraction makes the derivative
grow as 1/sqrt(D) and a quotient across it measures nothing."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vrt():
    import torch

    import paper_2606_22655_amd as vrt

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    vrt.load_library()
    return vrt


@pytest.fixture(scope="module")
def ctx(vrt):
    c = vrt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def problem():
    med, (P0, d0), prm, tgt = workloads.design_problem(n_side=128, max_steps=10000)
    return med, P0, d0, prm, tgt


def trace_fp64(vrt, ctx, values, P0, d0, prm):
    """Per-ray exit-plane points and events from the plain FP64 trace."""
    import torch

    spec = workloads.grid_medium(values)
    med = vrt.Medium(ctx, spec)
    try:
        b = vrt.RayBatch(P0, d0, "fp64")
        vrt.trace(med, b, prm, "fp64")
        torch.cuda.synchronize()
        return b.results()
    finally:
        med.close()


def ray_loss(res, tgt):
    ok = res["status"] == 0  # EXITED (to the plane)
    d = res["P"][:, :2] - tgt
    return np.where(ok, (d * d).sum(axis=1), 0.0), ok


def adjoint(vrt, ctx, values, P0, d0, prm, tgt, scale, K=64):
    import torch

    f = vrt.ExitPlaneLoss(ctx, P0, d0, tgt, prm, scale=scale, checkpoint_every=K)
    v = torch.as_tensor(values, device="cuda")
    g = torch.empty(v.shape, dtype=torch.float64, device="cuda")
    L = f.evaluate(v, g)
    torch.cuda.synchronize()
    return L, g.cpu().numpy(), f.loss_ray.cpu().numpy(), f.end.cpu().numpy()


def test_forward_loss_equals_the_plain_trace(vrt, ctx, problem):
    med, P0, d0, prm, tgt = problem
    L, _, lr, end = adjoint(vrt, ctx, med["grid"], P0, d0, prm, tgt, 1.0 / len(P0))
    res = trace_fp64(vrt, ctx, med["grid"], P0, d0, prm)
    l0, ok = ray_loss(res, tgt)
    assert np.array_equal(end == 1, ok)
    assert np.abs(lr - l0).max() < 1e-15
    assert L == pytest.approx(l0.sum() / len(P0), rel=1e-13)


def test_full_size_forward_matches_the_plain_trace_and_the_oracle(vrt, ctx, orc):
    """The 512 x 512-ray design configuration the benchmark times: per-ray
    loss and exit events of the adjoint's forward march equal the plain FP64
    trace's on every ray, and a seeded sample of 512 rays' exit points equals
    the oracle's to 1e-12; the gradient is finite, zero only where no ray
    passes, and its sum of |g| is reproducible from call to call."""
    med, (P0, d0), prm, tgt = workloads.design_problem(max_steps=10000)
    scale = 1.0 / len(P0)
    L, g, lr, end = adjoint(vrt, ctx, med["grid"], P0, d0, prm, tgt, scale)
    res = trace_fp64(vrt, ctx, med["grid"], P0, d0, prm)
    l0, ok = ray_loss(res, tgt)
    assert np.array_equal(end == 1, ok)
    assert np.abs(lr - l0).max() < 1e-15
    assert L == pytest.approx(l0.sum() * scale, rel=1e-13)
    idx = np.sort(np.random.default_rng(2026).choice(len(P0), 512, replace=False))
    o = orc.trace(med, (P0[idx], d0[idx]), prm)
    assert np.array_equal(o["status"], res["status"][idx])
    assert np.abs(o["P"] - res["P"][idx]).max() < 1e-12
    assert np.all(np.isfinite(g)) and np.abs(g).sum() > 0
    L2, g2, _, _ = adjoint(vrt, ctx, med["grid"], P0, d0, prm, tgt, scale)
    assert L2 == L
    # atomics make the order of additions vary: the sums agree to rounding
    assert np.abs(g2 - g).max() <= 1e-9 * np.abs(g).max()


def fd_rays(vrt, ctx, values, flat, h, P0, d0, prm, tgt):
    """Per-ray central difference quotient of the loss at node `flat` with step
    h (float32 values, the step actually taken), and the branch signature."""
    vp = values.copy().ravel()
    vm = values.copy().ravel()
    vp[flat] += np.float32(h)
    vm[flat] -= np.float32(h)
    hh = float(vp[flat]) - float(vm[flat])
    rp = trace_fp64(vrt, ctx, vp.reshape(values.shape), P0, d0, prm)
    rm = trace_fp64(vrt, ctx, vm.reshape(values.shape), P0, d0, prm)
    lp, _ = ray_loss(rp, tgt)
    lm, _ = ray_loss(rm, tgt)
    sig = [(r["status"], r["ntir"], r["nbtir"], r["steps"]) for r in (rp, rm)]
    return (lp - lm) / hh, sig


def linear_rays(q1, q2, sigs, base):
    same = np.ones(len(q1), dtype=bool)
    for s in sigs:
        for a, b in zip(s, base):
            same &= a == b
    tol = 1e-3 * np.maximum(np.abs(q2), 1e-9)
    return same & (np.abs(q1 - q2) <= tol)


def test_gradient_matches_finite_differences(vrt, ctx, problem):
    """32 seeded nodes (seed 304), central differences with h = 1e-4 and
    h / 2 on the plain FP64 trace; Richardson-extrapolated quotients of the
    linear rays against the adjoint of the same rays."""
    med, P0, d0, prm, tgt = problem
    values = med["grid"]
    n = len(P0)
    base_res = trace_fp64(vrt, ctx, values, P0, d0, prm)
    base = (base_res["status"], base_res["ntir"], base_res["nbtir"], base_res["steps"])
    nodes = np.random.default_rng(304).choice(values.size, 32, replace=False)
    checked = worst = 0.0
    set_aside = []
    for flat in nodes:
        q1, s1 = fd_rays(vrt, ctx, values, flat, 1e-4, P0, d0, prm, tgt)
        q2, s2 = fd_rays(vrt, ctx, values, flat, 5e-5, P0, d0, prm, tgt)
        lin = linear_rays(q1, q2, s1 + s2, base)
        set_aside.append(int((~lin & ((q1 != 0) | (q2 != 0))).sum()))
        qr = ((4 * q2 - q1) / 3)[lin]
        fd = qr.sum() / n
        _, g, _, _ = adjoint(vrt, ctx, values, P0[lin], d0[lin], prm, tgt[lin], 1.0 / n)
        err = abs(g.ravel()[flat] - fd)
        scale = max(np.abs(qr).sum() / n, 1e-9)  # the size of the rays' contributions
        print(f"[adjoint] node {flat}: adjoint {g.ravel()[flat]:.6e} fd {fd:.6e} "
              f"(sum |per ray| {scale:.3e}, {set_aside[-1]} rays set aside)", flush=True)
        worst = max(worst, err / scale)
        checked += 1
    print(f"[adjoint] worst error / contribution size: {worst:.3e}", flush=True)
    assert worst < 1e-3
    assert np.mean(set_aside) < 0.05 * n


def test_gradient_matches_the_oracle(vrt, ctx, orc, problem):
    """The FP64 oracle's own difference quotients against the adjoint at 32
    nodes, on 8,192 of the rays.

    In this medium (1 % white noise on 64^3 nodes) a parallel ray meets ~50
    TIR decisions at near-grazing incidence, so even a small change of one
    node value flips the branch pattern (status, TIR counts, step count) of
    most rays crossing the node's cells; a difference quotient is meaningful
    only on the rays whose pattern is unchanged at v +- h and v +- h/2 and
    whose two quotients agree to 1e-3 (linear rays).  Steps h = 8 and 4 float
    ulps of the node value keep the most rays linear.  Rays that move the
    loss lie within 5 cells of the node across the beam (lateral drift over
    the unit path stays below one cell), so the oracle retraces only those
    (the adjoint of the footprint rays equals the adjoint of all rays at the
    node, checked).  Nodes are taken in a seeded order among those the rays
    depend on, keeping the first 32 with at least one linear ray.  Each
    node's error is bounded against its net gradient (1e-3 of it, with a
    floor of 1e-6 of the summed size of the rays' contributions for nodes
    where they cancel) and against that summed size (1e-3)."""
    med, P0, d0, prm, tgt = problem
    values = med["grid"]
    N = values.shape[0]
    sel = np.arange(0, len(P0), 2)
    P0s, d0s, tgs = P0[sel], d0[sel], tgt[sel]
    n = len(sel)
    _, g_all, _, _ = adjoint(vrt, ctx, values, P0s, d0s, prm, tgs, 1.0 / n)
    o = orc.trace(workloads.grid_medium(values), (P0s, d0s), prm)
    base = (o["status"], o["ntir"], o["nbtir"], o["steps"])

    def oracle_q(flat, h, idx):
        vp = values.copy().ravel()
        vm = values.copy().ravel()
        vp[flat] += np.float32(h)
        vm[flat] -= np.float32(h)
        hh = float(vp[flat]) - float(vm[flat])
        rp = orc.trace(workloads.grid_medium(vp.reshape(values.shape)), (P0s[idx], d0s[idx]), prm)
        rm = orc.trace(workloads.grid_medium(vm.reshape(values.shape)), (P0s[idx], d0s[idx]), prm)
        lp, _ = ray_loss(rp, tgs[idx])
        lm, _ = ray_loss(rm, tgs[idx])
        return (lp - lm) / hh, [(r["status"], r["ntir"], r["nbtir"], r["steps"]) for r in (rp, rm)]

    order = np.random.default_rng(305).permutation(np.nonzero(g_all.ravel())[0])
    h = 8 * 1.1920929e-07
    compared, tried = 0, 0
    worst_net = worst_sum = 0.0
    for flat in order[:600]:
        if compared == 32:
            break
        tried += 1
        k, j, i = np.unravel_index(flat, values.shape)
        near = ((np.abs(P0s[:, 0] - i / (N - 1)) < 5.0 / (N - 1)) &
                (np.abs(P0s[:, 1] - j / (N - 1)) < 5.0 / (N - 1)))
        idx = np.nonzero(near)[0]
        q1, s1 = oracle_q(flat, h, idx)
        q2, s2 = oracle_q(flat, h / 2, idx)
        lin = linear_rays(q1, q2, s1 + s2, tuple(b[idx] for b in base))
        dep = (q1 != 0) | (q2 != 0)
        if not (lin & dep).any():
            continue
        if compared < 4:  # the footprint holds every ray that reaches the node
            _, gf, _, _ = adjoint(vrt, ctx, values, P0s[idx], d0s[idx], prm, tgs[idx], 1.0 / n)
            assert abs(gf.ravel()[flat] - g_all.ravel()[flat]) <= 1e-12 * np.abs(g_all).max()
        qr = ((4 * q2 - q1) / 3)[lin]
        fd = qr.sum() / n
        li = idx[lin]
        _, g, _, _ = adjoint(vrt, ctx, values, P0s[li], d0s[li], prm, tgs[li], 1.0 / n)
        scale = max(np.abs(qr).sum() / n, 1e-300)
        err = abs(g.ravel()[flat] - fd)
        rel_net = err / max(abs(fd), 1e-300)
        print(f"[adjoint] oracle node {flat}: adjoint {g.ravel()[flat]:.9e} oracle fd {fd:.9e} "
              f"error / net {rel_net:.2e}, / sum |per ray| {err / scale:.2e} "
              f"({int((lin & dep).sum())} linear of {int(dep.sum())} dependent rays)", flush=True)
        assert err <= 1e-3 * scale
        assert err <= 1e-3 * abs(fd) + 1e-6 * scale
        worst_sum = max(worst_sum, err / scale)
        if abs(fd) > 1e-3 * scale:
            worst_net = max(worst_net, rel_net)
        compared += 1
    print(f"[adjoint] oracle: {compared} nodes compared ({tried} tried); worst error / net "
          f"gradient {worst_net:.3e}, worst error / sum |per ray| {worst_sum:.3e}", flush=True)
    assert compared == 32


def test_checkpoint_interval_does_not_change_the_gradient(vrt, ctx, problem):
    med, P0, d0, prm, tgt = problem
    sel = np.arange(0, len(P0), 4)
    ref = None
    for K in (1, 16, 64, 4096):
        L, g, _, _ = adjoint(vrt, ctx, med["grid"], P0[sel], d0[sel], prm, tgt[sel],
                             1.0 / len(sel), K=K)
        if ref is None:
            ref = (L, g)
        else:
            assert L == ref[0]
            assert np.abs(g - ref[1]).max() <= 1e-10 * np.abs(ref[1]).max()


def test_autograd_backward_and_a_descent_step(vrt, ctx):
    """Through torch.autograd: the gradient equals the direct call, and a
    small step against it lowers the loss.  The medium is graded along z with
    a weak transverse ripple (32^3 nodes, n = 1.5 + 0.05 z + 0.002
    sin(2 pi x) cos(2 pi y)) and the rays are tilted 10 deg, so every
    refraction is far from critical and the loss is smooth."""
    import math

    import torch

    N = 32
    k = np.linspace(0.0, 1.0, N)
    Z, Y, X = np.meshgrid(k, k, k, indexing="ij")
    values = (1.5 + 0.05 * Z + 0.002 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)).astype(
        np.float32)
    n_side = 64
    c = (np.arange(n_side) + 0.5) / n_side
    XX, YY = np.meshgrid(c, c, indexing="xy")
    P0 = np.stack([XX.ravel() * 0.8, YY.ravel(), np.zeros(XX.size)], axis=1)
    a = math.radians(10.0)
    d0 = np.tile([math.sin(a), 0.0, math.cos(a)], (len(P0), 1))
    tgt = np.full((len(P0), 2), 0.5)
    prm = workloads.trace_params(5e-4, 10000, exit_plane_z=1.2)
    f = vrt.ExitPlaneLoss(ctx, P0, d0, tgt, prm)
    v = torch.tensor(values, device="cuda", requires_grad=True)
    L = f(v)
    L.backward()
    g = torch.empty(v.shape, dtype=torch.float64, device="cuda")
    L2 = f.evaluate(v, g)
    assert L.item() == L2
    assert torch.equal(v.grad, g.float())
    assert int(f.end.eq(1).sum()) == len(P0)
    gn = float((g * g).sum())
    eta = 1e-3 * L.item() / gn  # predicted decrease: 1e-3 L
    with torch.no_grad():
        v2 = (v.double() - eta * g).float()
    L3 = f.evaluate(v2)
    print(f"\n[adjoint] descent: L {L.item():.8e} -> {L3:.8e} (predicted "
          f"{L.item() - eta * gn:.8e})", flush=True)
    assert L3 < L.item()
    assert (L.item() - L3) == pytest.approx(eta * gn, rel=0.1)


def test_adjoint_refusals(vrt, ctx, problem):
    import torch

    med, P0, d0, prm, tgt = problem
    f = vrt.ExitPlaneLoss(ctx, P0[:64], d0[:64], tgt[:64], prm)
    v = torch.tensor(med["grid"], device="cuda")
    for bad in ({"eps_tan": 1e-3}, {"exit_plane_z": None}):
        g = vrt.ExitPlaneLoss(ctx, P0[:64], d0[:64], tgt[:64], dict(prm, **bad))
        with pytest.raises(vrt.VrtError):
            g.evaluate(v)
    other = vrt.Medium(ctx, workloads.spherical_medium())
    try:
        with pytest.raises(vrt.VrtError):  # not a grid medium
            vrt.vrt_grid_loss_grad(other.handle, f.params, f.rays, 64, 1.0, 64, 0, 0)
        with pytest.raises(vrt.VrtError):  # checkpoint interval out of range
            f.checkpoint_every = 0
            f.evaluate(v)
    finally:
        other.close()


def test_gradient_on_an_anisotropic_grid(vrt, ctx):
    """The adjoint on a grid with unequal node counts and spacings (11 x 19 x
    21 nodes) in a box off the origin, surroundings of index 1.33 (the seeded
    random grid 2 of the random-media tests): parallel rays along +z from
    below the box, exit plane 0.2 above it, targets scattered about the launch
    points.  Against central differences of the plain FP64 trace at 8 nodes
    the rays depend on (seeded order), with steps of 8 and 4 float ulps of
    the node value (larger steps straddle kinks of rays that pass near a
    critical decision: one-sided quotients of such a ray converge to the
    adjoint as the step shrinks), Richardson-extrapolated on the linear rays
    as above; each error bounded by 1e-3 of the summed size of the rays'
    contributions."""
    import torch

    from test_random_media_gpu import grid_case

    spec, _, shape = grid_case(2)
    values, lo, hi, n_amb = spec["grid"], spec["grid_lo"], spec["grid_hi"], spec["n_amb"]
    rng = np.random.default_rng(410)
    n = 4096
    P0 = np.stack([rng.uniform(lo[0] + 0.05, hi[0] - 0.05, n),
                   rng.uniform(lo[1] + 0.05, hi[1] - 0.05, n), np.full(n, lo[2] - 0.1)], axis=1)
    d0 = np.tile([0.0, 0.0, 1.0], (n, 1))
    tgt = P0[:, :2] + rng.normal(0.0, 0.05, (n, 2))
    prm = workloads.trace_params(2e-3, 20000, exit_plane_z=float(hi[2] + 0.2))

    def trace(vals, idx=slice(None)):
        med = vrt.Medium(ctx, workloads.grid_medium(vals, lo, hi, n_amb))
        try:
            b = vrt.RayBatch(P0[idx], d0[idx], "fp64")
            vrt.trace(med, b, prm, "fp64")
            torch.cuda.synchronize()
            return b.results()
        finally:
            med.close()

    def adj(idx):
        f = vrt.ExitPlaneLoss(ctx, P0[idx], d0[idx], tgt[idx], prm, lo=tuple(lo), hi=tuple(hi),
                              n_amb=n_amb, scale=1.0 / n, checkpoint_every=64)
        v = torch.as_tensor(values, device="cuda")
        g = torch.empty(v.shape, dtype=torch.float64, device="cuda")
        L = f.evaluate(v, g)
        torch.cuda.synchronize()
        return L, g.cpu().numpy()

    def quotient(flat, h):
        vp = values.copy().ravel()
        vm = values.copy().ravel()
        vp[flat] += np.float32(h)
        vm[flat] -= np.float32(h)
        hh = float(vp[flat]) - float(vm[flat])
        rp, rm = trace(vp.reshape(values.shape)), trace(vm.reshape(values.shape))
        lp, _ = ray_loss(rp, tgt)
        lm, _ = ray_loss(rm, tgt)
        return (lp - lm) / hh, [(r["status"], r["ntir"], r["nbtir"], r["steps"]) for r in (rp, rm)]

    res = trace(values)
    l0, ok = ray_loss(res, tgt)
    assert ok.sum() > 0.9 * n and int(res["ntir"].sum()) > 0
    L, g_all = adj(slice(None))
    assert L == pytest.approx(l0.sum() / n, rel=1e-13)
    base = (res["status"], res["ntir"], res["nbtir"], res["steps"])
    order = np.random.default_rng(411).permutation(np.nonzero(g_all.ravel())[0])
    compared = 0
    for flat in order[:200]:
        if compared == 8:
            break
        h = 8 * 1.1920929e-07
        q1, s1 = quotient(flat, h)
        q2, s2 = quotient(flat, h / 2)
        lin = linear_rays(q1, q2, s1 + s2, base)
        dep = (q1 != 0) | (q2 != 0)
        if not (lin & dep).any():
            continue
        qr = ((4 * q2 - q1) / 3)[lin]
        fd = qr.sum() / n
        _, g = adj(np.nonzero(lin)[0])
        scale = max(np.abs(qr).sum() / n, 1e-300)
        err = abs(g.ravel()[flat] - fd)
        print(f"[adjoint] {shape} node {flat}: adjoint {g.ravel()[flat]:.9e} fd {fd:.9e} "
              f"error / sum |per ray| {err / scale:.2e} "
              f"({int((lin & dep).sum())} linear of {int(dep.sum())} dependent rays)", flush=True)
        assert err <= 1e-3 * scale
        compared += 1
    assert compared == 8
