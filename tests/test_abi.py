"""The C-ABI library loads and exports every entry point include/vrt.h
declares, and the binding's struct layouts match the header (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrt.h")


@pytest.fixture(scope="module")
def vrt():
    import paper_2606_22655_amd as vrt

    if not os.path.exists(vrt.LIB_PATH):
        from paper_2606_22655_amd import build

        build.build()
    return vrt


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vrt_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("vrt_context_create", "vrt_medium_create_analytic", "vrt_medium_create_grid",
                     "vrt_medium_destroy", "vrt_trace", "vrt_reduce_counters", "vrt_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(vrt):
    lib = vrt.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(vrt.EXPORTED) == declared_functions()


def test_abi_version_and_empty_error(vrt):
    assert vrt.vrt_abi_version() == 1
    assert vrt.vrt_last_error() == ""


def test_struct_layouts_match_header(vrt, tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "vrt.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(vrt_boundary),
         sizeof(vrt_trace_params), sizeof(vrt_rays), sizeof(vrt_counters),
         offsetof(vrt_trace_params, precision), offsetof(vrt_rays, status),
         offsetof(vrt_boundary, params), sizeof(vrt_job_info), offsetof(vrt_job_info, t_done),
         sizeof(vrt_server_stats), offsetof(vrt_server_stats, lanes));
  return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(vrt.vrt_boundary), C.sizeof(vrt.vrt_trace_params), C.sizeof(vrt.vrt_rays),
            C.sizeof(vrt.vrt_counters), vrt.vrt_trace_params.precision.offset,
            vrt.vrt_rays.status.offset, vrt.vrt_boundary.params.offset,
            C.sizeof(vrt.vrt_job_info), vrt.vrt_job_info.t_done.offset,
            C.sizeof(vrt.vrt_server_stats), vrt.vrt_server_stats.lanes.offset]
    assert got == want


def test_enums_match_header(vrt):
    src = open(HEADER).read()

    def val(name):
        return int(re.search(rf"\b{name}\s*=\s*(-?\d+)", src).group(1))

    for k, v in vrt.MEDIUM_KINDS.items():
        assert val("VRT_MEDIUM_" + k.upper()) == v
    for k, v in vrt.BOUNDARY_KINDS.items():
        assert val("VRT_BOUNDARY_" + k.upper()) == v
    for k, v in vrt.STATUS.items():
        assert val("VRT_RAY_" + k) == v
    assert val("VRT_FP64") == vrt.VRT_FP64 and val("VRT_FP32_COMP") == vrt.VRT_FP32_COMP
    assert val("VRT_EINVAL") == vrt.VRT_EINVAL and val("VRT_ETIMEOUT") == vrt.VRT_ETIMEOUT
    for k, v in vrt.JOB_STATES.items():
        assert val("VRT_JOB_" + v) == k


def test_product_path_does_not_reference_the_oracle():
    """The GPU package and its sources never import, link or load the oracle."""
    pkg = os.path.join(ROOT, "paper_2606_22655_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "liboracle" not in text and "import oracle" not in text, f
                assert "from oracle" not in text and "vrt_oracle" not in text, f


def test_missing_library_fails_loudly():
    """Without libvrt.so the binding raises; there is no CPU fallback."""
    import subprocess
    import sys

    code = ("import paper_2606_22655_amd as v\n"
            "try:\n    v.load_library('/nonexistent/libvrt.so')\n"
            "except ImportError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "raised" in r.stdout and "not built" in r.stdout, r.stderr


def test_trace_batches_wants_two_streams(vrt):
    """The binding's two-in-flight helper refuses a stream list of another
    length before it touches the GPU."""
    with pytest.raises(ValueError):
        vrt.trace_batches(None, [], {}, "fp32c", streams=(None,))
