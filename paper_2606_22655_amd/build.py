"""Build libvrt.so (the gfx950 HIP library behind include/vrt.h) in-tree.

    python -m paper_2606_22655_amd.build

Compiles every source under csrc/ with hipcc for gfx950 into
paper_2606_22655_amd/libvrt.so.  Packed FP32 instructions are disabled: the
march's single-precision arithmetic is scalar per lane.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvrt.so")
SOURCES = ["vrt_api.hip", "march_fp64.hip", "march_fp32c.hip", "serve.hip", "design.hip",
           "adjoint.hip"]
ARCH = os.environ.get("VRT_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc_command(out, extra=()):
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Wall", "-Wno-unused-function", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(HERE, "..", "include"), "-o", out] +
            [os.path.join(CSRC, s) for s in SOURCES] +
            # the serving copies run on the SDMA engines through the HSA runtime
            ["-L", os.path.join(ROCM, "lib"), "-lhsa-runtime64"] + list(extra))


def build(verbose=False):
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    if verbose and errs:
        print("\n".join(errs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
