"""GPU: vrt_trace on the caller's streams -- two traces running concurrently
on two streams give the results of the same traces run one after the other,
and a single-precision trace captured in a HIP graph (through torch's
CUDAGraph) gives, on every replay, the result of the eager call."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

KEYS = ("P", "D", "status", "steps", "ntir", "nbtir", "flags")


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


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in KEYS)


def test_concurrent_streams_equal_serial(vrt, ctx):
    import torch

    cases = [(workloads.gaussian_medium(510), workloads.face_cone_rays(20000, 511, 20.0), "fp32c"),
             (workloads.grid_medium(workloads.noise_grid(32, 512)),
              workloads.face_cone_rays(15000, 513, 30.0), "fp32c"),
             (workloads.gaussian_medium(514), workloads.face_cone_rays(3000, 515, 20.0), "fp64")]
    prm = workloads.trace_params(1e-3, 20000)
    meds = [vrt.Medium(ctx, c[0]) for c in cases]
    try:
        serial = []
        for m, (_, rays, prec) in zip(meds, cases):
            b = vrt.RayBatch(rays[0], rays[1], prec)
            vrt.trace(m, b, prm, prec)
            torch.cuda.synchronize()
            serial.append(b.results())
        streams = [torch.cuda.Stream() for _ in cases]  # default priority
        batches = [vrt.RayBatch(rays[0], rays[1], prec) for (_, rays, prec) in cases]
        torch.cuda.synchronize()
        for s, m, b, (_, _, prec) in zip(streams, meds, batches, cases):
            vrt.trace(m, b, prm, prec, stream=s.cuda_stream)
        torch.cuda.synchronize()
        for k, b in enumerate(batches):
            assert same(serial[k], b.results()), k
    finally:
        for m in meds:
            m.close()


def test_trace_batches_two_in_flight_equal_serial(vrt, ctx):
    """A stream of ragged batches traced two at a time on two streams
    (trace_batches) gives every batch the result of a serial trace, and the
    results are in order on torch's current stream: read with no device-wide
    synchronisation in between."""
    import torch

    cases = [(workloads.grid_medium(workloads.noise_grid(32, 516)), 30.0, "fp32c"),
             (workloads.zernike_lens(), None, "fp32c"),
             (workloads.gaussian_medium(517), 20.0, "fp64")]
    sizes = (3001, 700, 4096, 257, 1999)
    for spec, cone, prec in cases:
        prm = workloads.trace_params(1e-3, 20000)
        med = vrt.Medium(ctx, spec)
        try:
            rays = [workloads.zernike_rays(n, seed=520 + k) if cone is None
                    else workloads.face_cone_rays(n, 520 + k, cone) for k, n in enumerate(sizes)]
            serial = []
            for r in rays:
                b = vrt.RayBatch(r[0], r[1], prec)
                vrt.trace(med, b, prm, prec)
                serial.append(b.results())
            batches = [vrt.RayBatch(r[0], r[1], prec) for r in rays]
            vrt.trace_batches(med, batches, prm, prec)
            for k, b in enumerate(batches):
                assert same(serial[k], b.results()), (spec["kind"], k)
        finally:
            med.close()
        torch.cuda.synchronize()


def test_trace_captured_in_a_graph_replays_the_eager_result(vrt, ctx):
    import torch

    spec, rays, prm = workloads.gaussian_cube(n_rays=8192)
    med = vrt.Medium(ctx, spec)
    try:
        b = vrt.RayBatch(rays[0], rays[1], "fp32c")
        vrt.trace(med, b, prm, "fp32c")  # eager (also settles the launch shape)
        torch.cuda.synchronize()
        eager = b.results()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                vrt.trace(med, b, prm, "fp32c", stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        for k in range(4):
            b.out.fill_(float("nan"))  # eager work between replays
            b.u32.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert same(eager, b.results()), k
        del g
    finally:
        med.close()


def test_grid_trace_captured_in_a_graph_equals_the_eager_one(vrt, ctx):
    """An eager single-precision trace on a grid medium enters its rays in a
    kernel of its own (states in stream-ordered memory); the same trace
    captured in a graph enters them inside the march.  Both give the same
    results bit for bit, on every replay."""
    import torch

    spec = workloads.grid_medium(workloads.noise_grid(48, 531))
    rays = workloads.face_cone_rays(6000, 532, 30.0)
    prm = workloads.trace_params(5e-4, 60000)
    med = vrt.Medium(ctx, spec)
    try:
        b = vrt.RayBatch(rays[0], rays[1], "fp32c")
        vrt.trace(med, b, prm, "fp32c")
        torch.cuda.synchronize()
        eager = b.results()
        assert (eager["status"] == 0).mean() > 0.9
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                vrt.trace(med, b, prm, "fp32c", stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        for k in range(3):
            b.out.fill_(float("nan"))
            b.u32.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert same(eager, b.results()), k
        del g
    finally:
        med.close()


def test_graph_replays_beside_more_than_1024_eager_traces(vrt, ctx):
    """A single-precision trace captured in a graph keeps a ray-queue counter
    of its own: replayed while 1,100 eager traces (more than the context's
    1,024 counters) run on another stream, every replay still equals the eager
    result bitwise, and so do the eager traces."""
    import torch

    spec, rays, prm = workloads.gaussian_cube(n_rays=16384)
    eager_rays = workloads.face_cone_rays(2048, 517, 20.0)
    prm_short = dict(prm, max_steps=400)
    med = vrt.Medium(ctx, spec)
    try:
        a = vrt.RayBatch(rays[0], rays[1], "fp32c")
        vrt.trace(med, a, prm, "fp32c")
        bref = vrt.RayBatch(eager_rays[0], eager_rays[1], "fp32c")
        vrt.trace(med, bref, prm_short, "fp32c")
        torch.cuda.synchronize()
        want_a, want_b = a.results(), bref.results()
        g = torch.cuda.CUDAGraph()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()  # default priority
        s1.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s1):
            with torch.cuda.graph(g, stream=s1):
                vrt.trace(med, a, prm, "fp32c", stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        outs = [vrt.RayBatch(eager_rays[0], eager_rays[1], "fp32c") for _ in range(4)]
        torch.cuda.synchronize()
        n_eager, replays = 1100, 0
        for k in range(n_eager):
            vrt.trace(med, outs[k % 4], prm_short, "fp32c", stream=s2.cuda_stream)
            if k % 100 == 50:
                a.out.fill_(float("nan"))
                a.u32.fill_(-1)
                torch.cuda.synchronize()
                with torch.cuda.stream(s1):
                    g.replay()
                replays += 1
                s1.synchronize()
                assert same(want_a, a.results()), k
        torch.cuda.synchronize()
        assert replays == 11
        for b in outs:
            assert same(want_b, b.results())
        del g
    finally:
        med.close()


def test_medium_destroy_defers_the_free_behind_a_running_trace(vrt, ctx):
    """vrt_medium_destroy returns without waiting for a trace still running on
    the medium; the memory is freed behind it, so the trace's results are
    intact, and a medium created right after works."""
    import time

    import torch

    spec, rays, prm = workloads.gaussian_cube(n_rays=1 << 19)
    med = vrt.Medium(ctx, spec)
    b = vrt.RayBatch(rays[0], rays[1], "fp32c")
    vrt.trace(med, b, prm, "fp32c")
    torch.cuda.synchronize()
    want = b.results()
    s = torch.cuda.Stream()
    b2 = vrt.RayBatch(rays[0], rays[1], "fp32c")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vrt.trace(med, b2, prm, "fp32c", stream=s.cuda_stream)
    t1 = time.perf_counter()
    med.close()  # the trace is still running
    t2 = time.perf_counter()
    s.synchronize()
    t3 = time.perf_counter()
    print(f"\n[destroy] launch {1e3 * (t1 - t0):.3f} ms, destroy {1e3 * (t2 - t1):.3f} ms, "
          f"trace done after {1e3 * (t3 - t0):.1f} ms", flush=True)
    assert (t3 - t0) > 0.01 and (t2 - t1) < 0.25 * (t3 - t0)
    assert same(want, b2.results())
    # a new medium (its memory may be the freed one) traces correctly
    med2 = vrt.Medium(ctx, spec)
    try:
        b3 = vrt.RayBatch(rays[0][:4096], rays[1][:4096], "fp32c")
        vrt.trace(med2, b3, prm, "fp32c")
        torch.cuda.synchronize()
        got = b3.results()
        assert all(np.array_equal(got[k], want[k][:4096]) for k in KEYS)
    finally:
        med2.close()
