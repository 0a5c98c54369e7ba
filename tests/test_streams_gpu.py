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
