"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, and the roofline bookkeeping is consistent."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_flop_and_traffic_tables():
    sys.path.insert(0, ROOT)
    import bench

    for w in ("freeform", "grid", "luneburg", "zernike", "spherical"):
        assert bench.algo_flops_per_step(w) >= 50
    assert bench.algo_flops_per_step("freeform") == 19 * 16 + 50
    assert set(bench.FP64_FLOPS_PER_STEP) == {"zernike", "spherical"}
    for w, (fetch, write, sha) in bench.TRAFFIC_KIB.items():
        assert fetch > 0 and write > 0 and len(sha) == 64
    # traffic is reported only for the kernel sources it was measured on
    t = bench.traffic_bytes("freeform")
    assert t is None or t == int((bench.TRAFFIC_KIB["freeform"][0] * bench.FETCH_SCALE +
                                  bench.TRAFFIC_KIB["freeform"][1] * bench.WRITE_SCALE) * 1024)
    assert bench.traffic_bytes("luneburg") is None
