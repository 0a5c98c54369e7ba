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
#include <mutex>
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

// Scratch of vrt_n2p_sweep_noalloc (4 MiB, held by every device the library
// runs on until the process ends).
static constexpr size_t kSweepScratchBytes = 4u << 20;
static __device__ __align__(256) unsigned char scratch[kSweepScratchBytes];

namespace {

// Device buffers of one sweep: the candidates' medium descriptors, the ray
// heights (uploaded), the RMSE per candidate and the optional axis crossings
// and step counts (downloaded).  Every entry the launch reads is uploaded
// first and every output is written by the kernel: nothing needs clearing.
struct SweepBufs {
    MediumDev *meds;
    double *y, *rmse, *z;
    unsigned long long *st;
};

int sweep_check(vrt_medium_t lens, const double *beta_gamma, size_t n_cand, const double *y,
                size_t n_rays, double z_launch, const vrt_trace_params *p, double *rmse,
                const char *who) {
    if (!lens || !beta_gamma || !y || !p || !rmse) return fail(VRT_EINVAL, "%s: NULL argument", who);
    if (lens->dev.kind != VRT_MEDIUM_N2P)
        return fail(VRT_EINVAL, "%s: the medium must be VRT_MEDIUM_N2P", who);
    if (lens->bnd.kind != VRT_BOUNDARY_CYLINDER || lens->bnd.p[0] != 0.0 || lens->bnd.p[1] != 0.0)
        return fail(VRT_EINVAL, "%s: the lens boundary must be a cylinder on the z axis", who);
    if (n_cand == 0 || n_cand > (1u << 20) || n_rays == 0 || n_rays > 4096)
        return fail(VRT_EINVAL, "%s: n_cand in [1, 2^20], n_rays in [1, 4096]", who);
    if (p->precision != VRT_FP64 || p->max_lanes != 0 || !isnan(p->exit_plane_z))
        return fail(VRT_EINVAL, "%s: VRT_FP64, max_lanes 0 and no exit plane", who);
    if (!(p->dL0 > 0.0) || !isfinite(p->dL0) || p->max_steps <= 0 ||
        p->max_steps > 0xFFFFFFFFll || !(p->eps_tan >= 0.0) || !(p->crit_rad >= 0.0) ||
        !(p->tie_eps >= 0.0) || !(p->tie_eps <= 1e-6))
        return fail(VRT_EINVAL, "%s: trace parameters out of range", who);
    if (!(z_launch < lens->bnd.p[3]) || !isfinite(z_launch))
        return fail(VRT_EINVAL, "%s: z_launch must lie before the lens (z < z0)", who);
    for (size_t i = 0; i < n_rays; ++i)
        if (!isfinite(y[i])) return fail(VRT_EINVAL, "%s: non-finite ray height", who);
    for (size_t c = 0; c < n_cand; ++c)
        if (!isfinite(beta_gamma[2 * c]) || !isfinite(beta_gamma[2 * c + 1]))
            return fail(VRT_EINVAL, "%s: non-finite candidate %zu", who, c);
    return VRT_OK;
}

// Upload, one launch, download, synchronise.
hipError_t sweep_run(vrt_medium_t lens, const double *beta_gamma, size_t n_cand, const double *y,
                     size_t n_rays, double z_launch, const vrt_trace_params *p, double *rmse,
                     double *z_int, uint64_t *steps, hipStream_t st, const SweepBufs &d) {
    std::vector<MediumDev> meds(n_cand, lens->dev);
    for (size_t c = 0; c < n_cand; ++c) {
        meds[c].q[2] = beta_gamma[2 * c];
        meds[c].q[3] = beta_gamma[2 * c + 1];
    }
    hipError_t e = hipMemcpyAsync(d.meds, meds.data(), sizeof(MediumDev) * n_cand,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.y, y, sizeof(double) * n_rays, hipMemcpyHostToDevice, st);
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
        hipLaunchKernelGGL(n2p_sweep_kernel, dim3(blocks), dim3(64), 0, st, d.meds,
                           (uint32_t)n_cand, lens->bnd, t, d.y, (uint32_t)n_rays, z_launch,
                           lens->dev.q[1], d.z, d.rmse, d.st);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(rmse, d.rmse, sizeof(double) * n_cand, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && z_int)
        e = hipMemcpyAsync(z_int, d.z, sizeof(double) * n_cand * n_rays, hipMemcpyDeviceToHost,
                           st);
    if (e == hipSuccess && steps)
        e = hipMemcpyAsync(steps, d.st, sizeof(unsigned long long) * n_cand,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// ---------------------------------------------------------------------------
// The sweep's buffers in a fixed device array, for callers that cannot
// allocate.  Each device holds its own copy of `scratch` at its own address,
// found once per device with hipGetSymbolAddress; host code uses that
// address, never the array's name (a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the sweep's buffers in one array; returns the total.
size_t sweep_layout(size_t n_cand, size_t n_rays, bool z, bool st, size_t off[5]) {
    size_t o = 0;
    off[0] = o;
    o += align256(sizeof(MediumDev) * n_cand);
    off[1] = o;
    o += align256(sizeof(double) * n_rays);
    off[2] = o;
    o += align256(sizeof(double) * n_cand);
    off[3] = o;
    o += z ? align256(sizeof(double) * n_cand * n_rays) : 0;
    off[4] = o;
    o += st ? align256(sizeof(unsigned long long) * n_cand) : 0;
    return o;
}

// Device address of this device's scratch (the device must be current).
int scratch_address(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(VRT_EUNSUPPORTED, "vrt_n2p_sweep_noalloc: device %d beyond %d", device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "vrt_n2p_sweep_noalloc: hipGetSymbolAddress");
        g_scratch_ptr[device] = ptr;
    }
    *out = (unsigned char *)g_scratch_ptr[device];
    return VRT_OK;
}

}  // namespace

extern "C" int vrt_n2p_sweep(vrt_medium_t lens, const double *beta_gamma, size_t n_cand,
                             const double *y, size_t n_rays, double z_launch,
                             const vrt_trace_params *p, double *rmse, double *z_int,
                             uint64_t *steps, void *stream) {
    if (int rc = sweep_check(lens, beta_gamma, n_cand, y, n_rays, z_launch, p, rmse,
                             "vrt_n2p_sweep"))
        return rc;
    int rc = set_device(lens->ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    SweepBufs d{};
    hipError_t e = hipMalloc((void **)&d.meds, sizeof(MediumDev) * n_cand);
    if (e == hipSuccess) e = hipMalloc((void **)&d.y, sizeof(double) * n_rays);
    if (e == hipSuccess) e = hipMalloc((void **)&d.rmse, sizeof(double) * n_cand);
    if (e == hipSuccess && z_int) e = hipMalloc((void **)&d.z, sizeof(double) * n_cand * n_rays);
    if (e == hipSuccess && steps)
        e = hipMalloc((void **)&d.st, sizeof(unsigned long long) * n_cand);
    if (e == hipSuccess)
        e = sweep_run(lens, beta_gamma, n_cand, y, n_rays, z_launch, p, rmse, z_int, steps, st, d);
    (void)hipFree(d.meds);
    (void)hipFree(d.y);
    (void)hipFree(d.rmse);
    (void)hipFree(d.z);
    (void)hipFree(d.st);
    if (e != hipSuccess) return fail_hip(e, "vrt_n2p_sweep");
    return VRT_OK;
}

extern "C" int vrt_n2p_sweep_noalloc(vrt_medium_t lens, const double *beta_gamma, size_t n_cand,
                                     const double *y, size_t n_rays, double z_launch,
                                     const vrt_trace_params *p, double *rmse, double *z_int,
                                     uint64_t *steps, void *stream) {
    if (int rc = sweep_check(lens, beta_gamma, n_cand, y, n_rays, z_launch, p, rmse,
                             "vrt_n2p_sweep_noalloc"))
        return rc;
    size_t off[5];
    const size_t need = sweep_layout(n_cand, n_rays, z_int != nullptr, steps != nullptr, off);
    if (need > kSweepScratchBytes)
        return fail(VRT_EINVAL,
                    "vrt_n2p_sweep_noalloc: %zu candidates x %zu rays need %zu bytes of scratch; "
                    "the fixed array holds %zu (use vrt_n2p_sweep, or fewer candidates)",
                    n_cand, n_rays, need, kSweepScratchBytes);
    int rc = set_device(lens->ctx);
    if (rc) return rc;
    unsigned char *base = nullptr;
    if ((rc = scratch_address(lens->ctx->device, &base))) return rc;
    SweepBufs d{};
    d.meds = (MediumDev *)(base + off[0]);
    d.y = (double *)(base + off[1]);
    d.rmse = (double *)(base + off[2]);
    d.z = z_int ? (double *)(base + off[3]) : nullptr;
    d.st = steps ? (unsigned long long *)(base + off[4]) : nullptr;
    const hipError_t e = sweep_run(lens, beta_gamma, n_cand, y, n_rays, z_launch, p, rmse, z_int,
                                   steps, (hipStream_t)stream, d);
    if (e != hipSuccess) return fail_hip(e, "vrt_n2p_sweep_noalloc");
    return VRT_OK;
}
