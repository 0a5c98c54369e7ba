// design.hip -- the paper's first design example (Sec. VI): a sweep of the
// cylindrical N2P-GRIN lens (Eq. (27)) over (beta, gamma) candidates, each
// scored by the RMSE of its longitudinal spherical aberration (Eqs. (28)-(29)).
//
// One lane per (candidate, ray): a wave holds floor(64 / N) candidates of N
// rays (or, for N > 64, one candidate whose rays its lanes stride over).
// Each lane marches its ray through its candidate's lens with the plain
// double-precision march (lane64.h) and turns the exit state into the axial
// coordinate where the ray's exit line crosses the optical axis; the squared
// aberrations of a candidate are then summed in ray order.  A refinement
// step of the design loop is one launch.
#pragma clang fp contract(off)
#include <vector>

#include "api_internal.h"
#include "lane64.h"

namespace vrt {

__global__ __launch_bounds__(64) void n2p_sweep_kernel(const MediumDev *__restrict__ meds,
                                                       uint32_t n_cand, BoundaryDev b,
                                                       TraceDev t, const double *__restrict__ y,
                                                       uint32_t n_rays, double z_launch,
                                                       double F, double *__restrict__ z_int,
                                                       double *__restrict__ rmse,
                                                       unsigned long long *__restrict__ steps) {
    // up to 64 rays: floor(64 / n_rays) candidates per wave, one ray per lane;
    // more rays: one candidate per wave, lanes striding over its rays
    __shared__ double sq_l[64];
    __shared__ int bad_l[64];
    __shared__ unsigned long long st_l[64];
    const uint32_t lane = threadIdx.x;
    const uint32_t per = n_rays <= 64 ? 64 / n_rays : 1;
    const uint32_t c0 = blockIdx.x * per;
    const uint32_t c = n_rays <= 64 ? c0 + lane / n_rays : c0;
    const uint32_t first = n_rays <= 64 ? lane % n_rays : lane;
    const uint32_t stride = n_rays <= 64 ? n_rays : 64;
    const bool mine = c < n_cand && (n_rays <= 64 ? lane < per * n_rays : true);
    double sq = 0.0;
    int bad = 0;
    unsigned long long nst = 0;
    if (mine) {
        const MediumDev &m = meds[c];
        for (uint32_t i = first; i < n_rays; i += stride) {
            Out64 o;
            trace_ray64<VRT_MEDIUM_N2P>(m, b, t, mk(0.0, y[i], z_launch), mk(0.0, 0.0, 1.0), o);
            // the exit line P + s D meets the axis (y = 0) at s = -P_y / D_y, ahead of
            // the exit point only if the ray heads towards the axis
            double zi = INFINITY;
            if (o.status == VRT_RAY_EXITED && o.P.y * o.D.y < 0.0)
                zi = o.P.z - o.P.y * o.D.z / o.D.y;
            else
                bad = 1;
            if (z_int) z_int[(size_t)c * n_rays + i] = zi;
            nst += o.steps;
            const double lsa = F - zi;  // Eq. (29)
            sq += lsa * lsa;
        }
    }
    sq_l[lane] = sq;
    bad_l[lane] = bad;
    st_l[lane] = nst;
    __syncthreads();
    // Eq. (28), the squared aberrations of a candidate summed in lane order
    if (n_rays <= 64) {
        if (lane < per && c0 + lane < n_cand) {
            double s2 = 0.0;
            int any = 0;
            unsigned long long ns = 0;
            for (uint32_t k = 0; k < n_rays; ++k) {
                s2 += sq_l[lane * n_rays + k];
                any |= bad_l[lane * n_rays + k];
                ns += st_l[lane * n_rays + k];
            }
            rmse[c0 + lane] = any ? INFINITY : sqrt(s2 / (double)n_rays);
            if (steps) steps[c0 + lane] = ns;
        }
    } else if (lane == 0) {
        double s2 = 0.0;
        int any = 0;
        unsigned long long ns = 0;
        for (uint32_t k = 0; k < 64; ++k) {
            s2 += sq_l[k];
            any |= bad_l[k];
            ns += st_l[k];
        }
        rmse[c0] = any ? INFINITY : sqrt(s2 / (double)n_rays);
        if (steps) steps[c0] = ns;
    }
}

}  // namespace vrt

using namespace vrt;

extern "C" int vrt_n2p_sweep(vrt_medium_t lens, const double *beta_gamma, size_t n_cand,
                             const double *y, size_t n_rays, double z_launch,
                             const vrt_trace_params *p, double *rmse, double *z_int,
                             uint64_t *steps, void *stream) {
    if (!lens || !beta_gamma || !y || !p || !rmse)
        return fail(VRT_EINVAL, "vrt_n2p_sweep: NULL argument");
    if (lens->dev.kind != VRT_MEDIUM_N2P)
        return fail(VRT_EINVAL, "vrt_n2p_sweep: the medium must be VRT_MEDIUM_N2P");
    if (lens->bnd.kind != VRT_BOUNDARY_CYLINDER || lens->bnd.p[0] != 0.0 || lens->bnd.p[1] != 0.0)
        return fail(VRT_EINVAL, "vrt_n2p_sweep: the lens boundary must be a cylinder on the z axis");
    if (n_cand == 0 || n_cand > (1u << 20) || n_rays == 0 || n_rays > 4096)
        return fail(VRT_EINVAL, "vrt_n2p_sweep: n_cand in [1, 2^20], n_rays in [1, 4096]");
    if (p->precision != VRT_FP64 || p->max_lanes != 0 || !isnan(p->exit_plane_z))
        return fail(VRT_EINVAL, "vrt_n2p_sweep: VRT_FP64, max_lanes 0 and no exit plane");
    if (!(p->dL0 > 0.0) || !isfinite(p->dL0) || p->max_steps <= 0 ||
        p->max_steps > 0xFFFFFFFFll || !(p->eps_tan >= 0.0) || !(p->crit_rad >= 0.0) ||
        !(p->tie_eps >= 0.0) || !(p->tie_eps <= 1e-6))
        return fail(VRT_EINVAL, "vrt_n2p_sweep: trace parameters out of range");
    if (!(z_launch < lens->bnd.p[3]) || !isfinite(z_launch))
        return fail(VRT_EINVAL, "vrt_n2p_sweep: z_launch must lie before the lens (z < z0)");
    for (size_t i = 0; i < n_rays; ++i)
        if (!isfinite(y[i])) return fail(VRT_EINVAL, "vrt_n2p_sweep: non-finite ray height");
    std::vector<MediumDev> meds(n_cand, lens->dev);
    for (size_t c = 0; c < n_cand; ++c) {
        const double be = beta_gamma[2 * c], ga = beta_gamma[2 * c + 1];
        if (!isfinite(be) || !isfinite(ga))
            return fail(VRT_EINVAL, "vrt_n2p_sweep: non-finite candidate %zu", c);
        meds[c].q[2] = be;
        meds[c].q[3] = ga;
    }
    int rc = set_device(lens->ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    MediumDev *d_meds = nullptr;
    double *d_y = nullptr, *d_rmse = nullptr, *d_z = nullptr;
    unsigned long long *d_st = nullptr;
    hipError_t e = hipMalloc((void **)&d_meds, sizeof(MediumDev) * n_cand);
    if (e == hipSuccess) e = hipMalloc((void **)&d_y, sizeof(double) * n_rays);
    if (e == hipSuccess) e = hipMalloc((void **)&d_rmse, sizeof(double) * n_cand);
    if (e == hipSuccess && z_int) e = hipMalloc((void **)&d_z, sizeof(double) * n_cand * n_rays);
    if (e == hipSuccess && steps) e = hipMalloc((void **)&d_st, sizeof(unsigned long long) * n_cand);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_meds, meds.data(), sizeof(MediumDev) * n_cand, hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_y, y, sizeof(double) * n_rays, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        TraceDev t{};
        t.dL0 = p->dL0;
        t.max_steps = p->max_steps;
        t.eps_tan = p->eps_tan;
        t.crit_rad = p->crit_rad;
        t.tie_eps = p->tie_eps;
        t.has_plane = 0;
        const uint32_t per = n_rays <= 64 ? 64u / (uint32_t)n_rays : 1u;
        const uint32_t blocks = (uint32_t)((n_cand + per - 1) / per);
        hipLaunchKernelGGL(n2p_sweep_kernel, dim3(blocks), dim3(64), 0, st, d_meds,
                           (uint32_t)n_cand, lens->bnd, t, d_y, (uint32_t)n_rays, z_launch,
                           lens->dev.q[1], d_z, d_rmse, d_st);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(rmse, d_rmse, sizeof(double) * n_cand, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && z_int)
        e = hipMemcpyAsync(z_int, d_z, sizeof(double) * n_cand * n_rays, hipMemcpyDeviceToHost,
                           st);
    if (e == hipSuccess && steps)
        e = hipMemcpyAsync(steps, d_st, sizeof(unsigned long long) * n_cand, hipMemcpyDeviceToHost,
                           st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_meds);
    (void)hipFree(d_y);
    (void)hipFree(d_rmse);
    (void)hipFree(d_z);
    (void)hipFree(d_st);
    if (e != hipSuccess) return fail_hip(e, "vrt_n2p_sweep");
    return VRT_OK;
}
