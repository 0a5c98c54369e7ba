"""Host logic on the CPU: the serving pool's first-fit allocator
(paper_2606_22655_amd/csrc/pool.h), built with g++ in libstdc++'s checked
mode and driven by a seeded random sequence of allocations and releases.

Checked after every operation, against an independent model of the live
blocks: blocks lie inside the pool and do not overlap; an allocation takes
the lowest offset where the rounded size fits (and fails only when no gap
fits); used() is the sum of the live rounded sizes and peak() its maximum;
after everything is released the whole pool is one free range again.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_22655_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>
#include "pool.h"

using vrt::serve::Pool;

static size_t round_up(size_t b) { return (b + 255) & ~(size_t)255; }

// lowest offset in [0, size) where `need` bytes fit between live blocks
static bool first_gap(const std::map<size_t, size_t> &live, size_t size, size_t need, size_t *off) {
    size_t at = 0;
    for (const auto &kv : live) {
        if (kv.first >= at && kv.first - at >= need) { *off = at; return true; }
        at = kv.first + kv.second;
    }
    if (size >= at && size - at >= need) { *off = at; return true; }
    return false;
}

int main(int argc, char **argv) {
    const unsigned seed = (unsigned)atoi(argv[1]);
    const size_t size = (size_t)1 << 20;
    std::mt19937_64 rng(seed);
    Pool p;
    p.reset(size);
    std::map<size_t, size_t> live;  // offset -> rounded size
    size_t peak = 0, fails = 0, allocs = 0;
    for (int op = 0; op < 20000; ++op) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t bytes = 1 + rng() % (48 << 10);
            size_t off = 0, want = 0;
            const bool fits = first_gap(live, size, round_up(bytes), &want);
            const bool ok = p.alloc(bytes, &off);
            if (ok != fits) { printf("FAIL alloc result %d expected %d at op %d\n", ok, fits, op); return 1; }
            if (ok) {
                if (off != want) { printf("FAIL first fit: %zu expected %zu at op %d\n", off, want, op); return 1; }
                if (off % 256 || off + round_up(bytes) > size) { printf("FAIL range at op %d\n", op); return 1; }
                live[off] = round_up(bytes);
                ++allocs;
            } else {
                ++fails;
            }
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            // release with the caller's unrounded size, as the server does
            p.release(it->first, it->second - (rng() % 256));
            live.erase(it);
        }
        size_t used = 0, end = 0;
        for (const auto &kv : live) {
            if (kv.first < end) { printf("FAIL overlap at op %d\n", op); return 1; }
            end = kv.first + kv.second;
            used += kv.second;
        }
        peak = used > peak ? used : peak;
        if (p.used() != used || p.peak() != peak) {
            printf("FAIL accounting at op %d: used %zu/%zu peak %zu/%zu\n", op, p.used(), used, p.peak(), peak);
            return 1;
        }
    }
    for (const auto &kv : live) p.release(kv.first, kv.second);
    size_t off = 1;
    if (p.used() != 0 || !p.alloc(size, &off) || off != 0) { printf("FAIL merge after release\n"); return 1; }
    printf("OK allocs %zu fails %zu peak %zu\n", allocs, fails, peak);
    return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("pool")
    src = d / "pool_harness.cpp"
    src.write_text(HARNESS)
    exe = d / "pool_harness"
    subprocess.run([gxx, "-std=c++17", "-O1", "-D_GLIBCXX_DEBUG", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True, capture_output=True, text=True)
    return str(exe)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pool_first_fit_and_merging(harness, seed):
    r = subprocess.run([harness, str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")
    allocs, fails = int(r.stdout.split()[2]), int(r.stdout.split()[4])
    assert allocs > 1000 and fails > 100  # the pool both fills up and recovers
