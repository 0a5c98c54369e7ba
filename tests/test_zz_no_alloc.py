"""GPU: vrt_n2p_sweep_noalloc (the design sweep with its device buffers in the
library's fixed scratch array) gives the results of vrt_n2p_sweep bitwise,
on two calls in a row -- the second smaller, so that stale contents of the
shared array from the first would show -- and refuses a sweep whose buffers
do not fit the array."""
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


def test_noalloc_sweep_equals_the_allocating_sweep(vrt):
    ctx = vrt.Context(0)
    try:
        L = 0.3
        lens = vrt.Medium(ctx, workloads.n2p_lens(1.0, 1.0, L))
        try:
            rng = np.random.default_rng(41)
            prm = vrt.make_params({"dL0": 2e-4, "max_steps": 10 ** 7}, "fp64")
            for n_cand, n_rays in ((300, 10), (37, 7)):
                bg = np.column_stack([rng.uniform(0.5, 1.2, n_cand), rng.uniform(2.5, 6.0, n_cand)])
                bg[3] = (1.0, -1.0)  # diverging: +inf
                P0, _ = workloads.n2p_rays(L, n_rays)
                y = workloads.n2p_heights(n_rays)
                print(f"\n[noalloc] {n_cand} candidates x {n_rays} rays", flush=True)
                want = vrt.vrt_n2p_sweep(lens.handle, bg, y, P0[0, 2], prm, want_z=True,
                                         want_steps=True)
                got = vrt.vrt_n2p_sweep_noalloc(lens.handle, bg, y, P0[0, 2], prm, want_z=True,
                                                want_steps=True)
                for a, b in zip(want, got):
                    assert a.shape == b.shape and np.array_equal(a, b)
                assert np.isinf(got[0][3]) and np.isfinite(got[0]).sum() > n_cand // 2
                # RMSE alone (no z, no steps): the layout without the optional buffers
                r = vrt.vrt_n2p_sweep_noalloc(lens.handle, bg, y, P0[0, 2], prm)
                assert np.array_equal(r, want[0])
            # a sweep whose buffers exceed the fixed array is refused before any launch
            big = np.tile([[0.8, 4.0]], (200000, 1))
            with pytest.raises(vrt.VrtError, match="scratch"):
                vrt.vrt_n2p_sweep_noalloc(lens.handle, big, workloads.n2p_heights(10), -0.5,
                                          prm, want_z=True)
        finally:
            lens.close()
    finally:
        ctx.close()
