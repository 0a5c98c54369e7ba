// march_fp64.hip -- plain double-precision VRT march: one lane per ray, one
// launch per batch, no compaction.  Every step follows Sec. II literally in
// IEEE double: medium evaluation, normal (Eq. (5)), straight / tangential /
// TIR / Snell dispatch (cases (ii)-(v), Eqs. (9)-(20)), constant-OPL move
// (Eqs. (3)-(4)), and refraction or reflection at the enclosing surface
// (case (i)).
//
// The formulas are evaluated as written, each operation correctly rounded:
// no FMA contraction in this file, divisions kept as divisions.  Where no
// transcendental function is involved (homogeneous, linear, Luneburg, fiber
// and grid media) the march is therefore the exact IEEE-double evaluation of
// the method, step for step.
#pragma clang fp contract(off)
#include "lane64.h"

namespace vrt {

template <int MK>
__global__ __launch_bounds__(256) void march_fp64_kernel(MediumDev m, BoundaryDev b, TraceDev t,
                                                         RaysDev<double> io, uint32_t n) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    Out64 o;
    trace_ray64<MK>(m, b, t, mk(io.px[r], io.py[r], io.pz[r]), mk(io.dx[r], io.dy[r], io.dz[r]), o);
    io.ox[r] = o.P.x;
    io.oy[r] = o.P.y;
    io.oz[r] = o.P.z;
    io.odx[r] = o.D.x;
    io.ody[r] = o.D.y;
    io.odz[r] = o.D.z;
    io.status[r] = o.status;
    io.steps[r] = o.steps;
    io.n_tir[r] = o.ntir;
    io.n_btir[r] = o.nbtir;
    io.flags[r] = o.flags;
}

// The same march with its polyline recorded: point k of ray r at
// path[(k * n + r) * 3 .. + 2] for k < cap (point-major, so the lanes of a wave
// write neighbouring points), the number of points of ray r in n_points[r].
template <int MK>
__global__ __launch_bounds__(256) void record_paths_kernel(MediumDev m, BoundaryDev b, TraceDev t,
                                                           RaysDev<double> io, uint32_t n,
                                                           double *path, uint64_t cap,
                                                           uint64_t *n_points) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    Out64 o;
    PathRec rec{path + (size_t)r * 3, cap, 0, (size_t)n * 3};
    trace_ray64<MK>(m, b, t, mk(io.px[r], io.py[r], io.pz[r]), mk(io.dx[r], io.dy[r], io.dz[r]), o,
                    rec);
    io.ox[r] = o.P.x;
    io.oy[r] = o.P.y;
    io.oz[r] = o.P.z;
    io.odx[r] = o.D.x;
    io.ody[r] = o.D.y;
    io.odz[r] = o.D.z;
    io.status[r] = o.status;
    io.steps[r] = o.steps;
    io.n_tir[r] = o.ntir;
    io.n_btir[r] = o.nbtir;
    io.flags[r] = o.flags;
    n_points[r] = rec.n;
}

template <int MK>
static hipError_t launch_rec(const LaunchArgs &a, double *path, uint64_t cap, uint64_t *n_points) {
    const uint32_t blocks = (a.n + 255u) / 256u;
    hipLaunchKernelGGL(record_paths_kernel<MK>, dim3(blocks), dim3(256), 0, a.stream, a.m, a.b,
                       a.t, a.io64, a.n, path, cap, n_points);
    return hipGetLastError();
}

template <int MK>
static hipError_t launch64(const LaunchArgs &a) {
    const uint32_t blocks = (a.n + 255u) / 256u;
    hipLaunchKernelGGL(march_fp64_kernel<MK>, dim3(blocks), dim3(256), 0, a.stream, a.m, a.b, a.t,
                       a.io64, a.n);
    return hipGetLastError();
}

hipError_t launch_march_fp64(const LaunchArgs &a) {
    if (a.n == 0) return hipSuccess;
    switch (a.m.kind) {
    case VRT_MEDIUM_HOMOGENEOUS: return launch64<VRT_MEDIUM_HOMOGENEOUS>(a);
    case VRT_MEDIUM_LINEAR: return launch64<VRT_MEDIUM_LINEAR>(a);
    case VRT_MEDIUM_LUNEBURG: return launch64<VRT_MEDIUM_LUNEBURG>(a);
    case VRT_MEDIUM_FIBER: return launch64<VRT_MEDIUM_FIBER>(a);
    case VRT_MEDIUM_GAUSSIAN: return launch64<VRT_MEDIUM_GAUSSIAN>(a);
    case VRT_MEDIUM_GRID: return launch64<VRT_MEDIUM_GRID>(a);
    case VRT_MEDIUM_SPHERICAL: return launch64<VRT_MEDIUM_SPHERICAL>(a);
    case VRT_MEDIUM_N2P: return launch64<VRT_MEDIUM_N2P>(a);
    case VRT_MEDIUM_ZERNIKE: return launch64<VRT_MEDIUM_ZERNIKE>(a);
    }
    return hipErrorInvalidValue;
}


hipError_t launch_paths_fp64(const LaunchArgs &a, double *path, uint64_t cap, uint64_t *n_points) {
    if (a.n == 0) return hipSuccess;
    switch (a.m.kind) {
    case VRT_MEDIUM_HOMOGENEOUS: return launch_rec<VRT_MEDIUM_HOMOGENEOUS>(a, path, cap, n_points);
    case VRT_MEDIUM_LINEAR: return launch_rec<VRT_MEDIUM_LINEAR>(a, path, cap, n_points);
    case VRT_MEDIUM_LUNEBURG: return launch_rec<VRT_MEDIUM_LUNEBURG>(a, path, cap, n_points);
    case VRT_MEDIUM_FIBER: return launch_rec<VRT_MEDIUM_FIBER>(a, path, cap, n_points);
    case VRT_MEDIUM_GAUSSIAN: return launch_rec<VRT_MEDIUM_GAUSSIAN>(a, path, cap, n_points);
    case VRT_MEDIUM_GRID: return launch_rec<VRT_MEDIUM_GRID>(a, path, cap, n_points);
    case VRT_MEDIUM_SPHERICAL: return launch_rec<VRT_MEDIUM_SPHERICAL>(a, path, cap, n_points);
    case VRT_MEDIUM_N2P: return launch_rec<VRT_MEDIUM_N2P>(a, path, cap, n_points);
    case VRT_MEDIUM_ZERNIKE: return launch_rec<VRT_MEDIUM_ZERNIKE>(a, path, cap, n_points);
    }
    return hipErrorInvalidValue;
}

}  // namespace vrt
