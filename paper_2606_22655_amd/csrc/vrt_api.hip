// vrt_api.hip -- host side of libvrt: the extern "C" entry points declared
// in include/vrt.h (contexts, device-resident media, trace dispatch, counter
// reduction, error reporting).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace vrt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int vrt::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
int vrt::fail_hip(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? VRT_ENOMEM : VRT_EHIP, "%s: %s", what,
                hipGetErrorString(e));
}

// A kernel may read or write this pointer: device, managed or pinned host
// memory.  Pageable host memory is refused (a kernel touching it would take a
// memory fault).
bool vrt::gpu_accessible(const void *p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type != hipMemoryTypeUnregistered;
}

// Medium memory comes from the stream-ordered allocator on the context's
// library stream, so that a medium can be freed in stream order behind the
// launches that read it, without blocking the host (a plain hipFree waits for
// the device, which may hold a resident serving kernel).
static int dev_alloc(vrt_medium_t m, void **p, size_t bytes) {
    hipError_t e = m->async_allocs ? hipMallocAsync(p, bytes, m->ctx->aux) : hipMalloc(p, bytes);
    if (e != hipSuccess) return fail_hip(e, "device allocation (medium)");
    m->allocs.push_back(*p);
    m->bytes += bytes;
    return VRT_OK;
}

// Wait for the medium's uploads on the library stream.
static hipError_t medium_ready(vrt_medium_t m) { return hipStreamSynchronize(m->ctx->aux); }

// Free a medium after every eager launch recorded on it: the library stream
// waits for their events, then returns the memory in stream order.  The host
// does not wait.  (Without the stream-ordered allocator: wait, then free.)
static void free_medium(vrt_medium_t m) {
    vrt_context_t ctx = m->ctx;
    {
        std::lock_guard<std::mutex> lk(m->use_mu);
        for (const MediumUse &u : m->uses) {
            if (m->async_allocs)
                (void)hipStreamWaitEvent(ctx->aux, u.ev, 0);
            else
                (void)hipEventSynchronize(u.ev);
            (void)hipEventDestroy(u.ev);
        }
        m->uses.clear();
    }
    for (void *p : m->allocs) (void)(m->async_allocs ? hipFreeAsync(p, ctx->aux) : hipFree(p));
    m->allocs.clear();
    delete m;
}

// Record that a launch on `stream` reads the medium (one event per stream:
// recording again on the same stream supersedes the earlier launch, which
// completes first).  A launch captured in a graph is not recorded: the caller
// who owns the graph keeps the medium alive while the graph may replay.
static int note_use(vrt_medium_t m, hipStream_t stream, bool captured) {
    if (captured) return VRT_OK;
    std::lock_guard<std::mutex> lk(m->use_mu);
    for (MediumUse &u : m->uses)
        if (u.stream == stream) {
            HIP_TRY(hipEventRecord(u.ev, stream), "hipEventRecord (medium use)");
            return VRT_OK;
        }
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate (medium use)");
    hipError_t e = hipEventRecord(ev, stream);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ev);
        return fail_hip(e, "hipEventRecord (medium use)");
    }
    m->uses.push_back(MediumUse{stream, ev});
    return VRT_OK;
}

static int stream_captured(hipStream_t stream, bool &captured) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cs), "hipStreamIsCapturing");
    captured = cs != hipStreamCaptureStatusNone;
    return VRT_OK;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// Node records of a discretized medium: value and, per axis, the central
// difference of the node values divided by the number of spacings it spans
// (2; 1 at the first and last node) -- exact in float for nearby values;
// grad n = record * (1/h).  Flags non-positive or non-finite values.
__global__ void grid_records_kernel(const float *__restrict__ v, float4 *__restrict__ rec, int nx,
                                    int ny, int nz, unsigned int *bad) {
    const size_t total = (size_t)nx * ny * nz;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nx);
        const int j = (int)((idx / nx) % ny);
        const int k = (int)(idx / ((size_t)nx * ny));
        const float c = v[idx];
        if (!(c > 0.0f) || !isfinite(c)) atomicOr(bad, 1u);
        const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
        const int il = i > 0 ? i - 1 : 0, ih = i < nx - 1 ? i + 1 : nx - 1;
        const int jl = j > 0 ? j - 1 : 0, jh = j < ny - 1 ? j + 1 : ny - 1;
        const int kl = k > 0 ? k - 1 : 0, kh = k < nz - 1 ? k + 1 : nz - 1;
        const size_t row = (size_t)k * sz + (size_t)j * sy;
        const float hx = (v[row + ih] - v[row + il]) / (float)(ih - il);
        const float hy = (v[(size_t)k * sz + (size_t)jh * sy + i] -
                          v[(size_t)k * sz + (size_t)jl * sy + i]) / (float)(jh - jl);
        const float hz = (v[(size_t)kh * sz + (size_t)j * sy + i] -
                          v[(size_t)kl * sz + (size_t)j * sy + i]) / (float)(kh - kl);
        rec[idx] = make_float4(c, hx, hy, hz);
        // flag differences that float does not hold exactly (neighbouring
        // values more than a factor 2 apart): the double-precision march then
        // forms them from the node values instead of reading the records
        const double ex = (double)v[row + ih] - (double)v[row + il];
        const double ey = (double)v[(size_t)k * sz + (size_t)jh * sy + i] -
                          (double)v[(size_t)k * sz + (size_t)jl * sy + i];
        const double ez = (double)v[(size_t)kh * sz + (size_t)j * sy + i] -
                          (double)v[(size_t)kl * sz + (size_t)j * sy + i];
        if ((double)hx * (double)(ih - il) != ex || (double)hy * (double)(jh - jl) != ey ||
            (double)hz * (double)(kh - kl) != ez)
            atomicOr(bad, 2u);
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void reduce_counters_kernel(const uint32_t *__restrict__ status,
                                       const uint32_t *__restrict__ steps,
                                       const uint32_t *__restrict__ ntir,
                                       const uint32_t *__restrict__ nbtir,
                                       const uint32_t *__restrict__ flags, size_t n,
                                       unsigned long long *out) {
    unsigned long long acc[kNumCounters] = {0};
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (size_t)gridDim.x * blockDim.x) {
        const uint32_t s = status[r], f = flags[r];
        acc[0] += 1;
        acc[1] += steps[r];
        acc[2] += s == VRT_RAY_EXITED;
        acc[3] += s == VRT_RAY_MISSED;
        acc[4] += s == VRT_RAY_TRUNCATED;
        acc[5] += s == VRT_RAY_NO_PLANE;
        acc[6] += s == VRT_RAY_INVALID_INPUT;
        acc[7] += s == VRT_RAY_REFLECTED_AT_ENTRY;
        acc[8] += ntir[r];
        acc[9] += nbtir[r];
        acc[10] += (f & VRT_FLAG_NEAR_CRITICAL) != 0;
        acc[11] += (f & VRT_FLAG_TANGENT) != 0;
        acc[12] += (f & VRT_FLAG_STRAIGHT) != 0;
        acc[13] += (f & VRT_FLAG_NEAR_TIE) != 0;
        acc[14] += (f & VRT_FLAG_NEAR_GRAZING) != 0;
    }
#pragma unroll
    for (int k = 0; k < kNumCounters; ++k) {
        unsigned long long v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (__lane_id() == 0 && v) atomicAdd(out + k, v);
    }
}

// ---------------------------------------------------------------------------
// API
// ---------------------------------------------------------------------------
extern "C" {

int vrt_abi_version(void) { return VRT_ABI_VERSION; }

const char *vrt_last_error(void) { return g_err.c_str(); }

int vrt_context_create(int hip_device, vrt_context_t *out) {
    if (!out) return fail(VRT_EINVAL, "vrt_context_create: out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= n)
        return fail(VRT_EINVAL, "vrt_context_create: device %d of %d", hip_device, n);
    HIP_TRY(hipSetDevice(hip_device), "hipSetDevice");
    auto *c = new vrt_context_s();
    c->device = hip_device;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, hip_device) ==
            hipSuccess &&
        cu > 0)
        c->num_cu = cu;
    hipError_t e = hipMalloc((void **)&c->queues, sizeof(uint32_t) * kQueueSlots * kQueueStride);
    if (e == hipSuccess)
        e = hipMalloc((void **)&c->counters, sizeof(unsigned long long) * kNumCounters);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    for (int i = 0; i < kEagerSlots && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&c->slot_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) {
        int pools = 0;
        if (hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, hip_device) !=
                hipSuccess)
            pools = 0;
        c->async_pools = pools != 0;
    }
    if (e != hipSuccess) {
        for (int i = 0; i < kEagerSlots; ++i)
            if (c->slot_ev[i]) (void)hipEventDestroy(c->slot_ev[i]);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        if (c->counters) (void)hipFree(c->counters);
        if (c->queues) (void)hipFree(c->queues);
        delete c;
        return fail_hip(e, "vrt_context_create");
    }
    *out = c;
    return VRT_OK;
}

int vrt_context_destroy(vrt_context_t ctx) {
    if (!ctx) return fail(VRT_EINVAL, "vrt_context_destroy: NULL context");
    if (ctx->n_media.load() != 0)
        return fail(VRT_EINVAL, "vrt_context_destroy: %d media still alive", ctx->n_media.load());
    if (ctx->n_servers.load() != 0)
        return fail(VRT_EINVAL, "vrt_context_destroy: %d servers still alive",
                    ctx->n_servers.load());
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->aux);  // deferred medium frees
    (void)hipDeviceSynchronize();
    for (int i = 0; i < kEagerSlots; ++i) (void)hipEventDestroy(ctx->slot_ev[i]);
    (void)hipStreamDestroy(ctx->aux);
    (void)hipFree(ctx->queues);
    (void)hipFree(ctx->counters);
    delete ctx;
    return VRT_OK;
}

static bool finite_all(const double *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i])) return false;
    return true;
}

static int check_boundary(const vrt_boundary *b, BoundaryDev &out) {
    if (!b) return fail(VRT_EINVAL, "boundary is NULL");
    if (b->reserved != 0) return fail(VRT_EINVAL, "boundary.reserved must be 0");
    const double *p = b->params;
    switch (b->kind) {
    case VRT_BOUNDARY_BOX:
        if (!finite_all(p, 6) || !(p[0] < p[3]) || !(p[1] < p[4]) || !(p[2] < p[5]))
            return fail(VRT_EINVAL, "box boundary needs finite lo < hi");
        break;
    case VRT_BOUNDARY_SPHERE:
        if (!finite_all(p, 4) || !(p[3] > 0.0)) return fail(VRT_EINVAL, "sphere radius must be > 0");
        break;
    case VRT_BOUNDARY_CYLINDER:
        if (!finite_all(p, 5) || !(p[2] > 0.0) || !(p[3] < p[4]))
            return fail(VRT_EINVAL, "cylinder needs r > 0 and z0 < z1");
        break;
    default:
        return fail(VRT_EINVAL, "unknown boundary kind %d", b->kind);
    }
    out.kind = b->kind;
    for (int i = 0; i < 6; ++i) {
        out.p[i] = p[i];
        out.pf[i] = (float)p[i];
    }
    return VRT_OK;
}

int vrt_medium_create_analytic(vrt_context_t ctx, int kind, const double *params, int n_params,
                               const vrt_boundary *bnd, double n_ambient, vrt_medium_t *out) {
    if (!ctx || !out) return fail(VRT_EINVAL, "vrt_medium_create_analytic: NULL argument");
    if (!params || n_params <= 0 || !finite_all(params, n_params))
        return fail(VRT_EINVAL, "vrt_medium_create_analytic: params missing or non-finite");
    if (!(n_ambient > 0.0) || !isfinite(n_ambient))
        return fail(VRT_EINVAL, "n_ambient must be finite and > 0");
    static const int need[] = {1, 4, 4, 5, -1, -1, 7, 4, -1};
    if (kind < VRT_MEDIUM_HOMOGENEOUS || kind > VRT_MEDIUM_ZERNIKE || kind == VRT_MEDIUM_GRID)
        return fail(VRT_EINVAL, "analytic medium kind %d unknown (grids use vrt_medium_create_grid)",
                    kind);
    if (need[kind] >= 0 && n_params != need[kind])
        return fail(VRT_EINVAL, "medium kind %d needs %d params, got %d", kind, need[kind], n_params);
    BoundaryDev b;
    if (int rc = check_boundary(bnd, b)) return rc;
    int rc = set_device(ctx);
    if (rc) return rc;
    auto *m = new vrt_medium_s();
    m->ctx = ctx;
    m->async_allocs = ctx->async_pools;
    m->bnd = b;
    MediumDev &d = m->dev;
    d.kind = kind;
    d.n_amb = n_ambient;
    const double *p = params;
    MedF &f = m->mf;
    switch (kind) {
    case VRT_MEDIUM_HOMOGENEOUS:
        if (!(p[0] > 0.0)) {
            delete m;
            return fail(VRT_EINVAL, "homogeneous index must be > 0");
        }
        d.q[0] = p[0];
        f.q[0] = (float)p[0];
        f.q[1] = (float)(p[0] - (double)f.q[0]);  // low part of the step's index
        break;
    case VRT_MEDIUM_LINEAR:
        for (int i = 0; i < 4; ++i) {
            d.q[i] = p[i];
            f.q[i] = (float)p[i];
        }
        f.q[4] = (float)(p[0] - (double)f.q[0]);
        break;
    case VRT_MEDIUM_LUNEBURG:
        if (!(p[0] > 0.0)) {
            delete m;
            return fail(VRT_EINVAL, "Luneburg radius must be > 0");
        }
        for (int i = 0; i < 4; ++i) {
            d.q[i] = p[i];
            f.q[i] = (float)p[i];
        }
        f.q[4] = (float)(1.0 / (p[0] * p[0]));
        break;
    case VRT_MEDIUM_FIBER: {
        const double nc = p[0], Dl = p[1], R = p[2];
        if (!(nc > 0.0) || !(R > 0.0) || !(Dl >= 0.0) || !(2.0 * Dl < 1.0)) {
            delete m;
            return fail(VRT_EINVAL, "fiber needs n_c > 0, R > 0, 0 <= Delta < 1/2");
        }
        for (int i = 0; i < 5; ++i) {
            d.q[i] = p[i];
            f.q[i] = (float)p[i];
        }
        f.q[5] = (float)(2.0 * Dl * nc * nc / (R * R));
        f.q[6] = (float)(nc * sqrt(1.0 - 2.0 * Dl));
        f.q[7] = (float)(R * R);
        break;
    }
    case VRT_MEDIUM_SPHERICAL:
        // Sec. V, Eq. (26); evaluated in double on both paths (media.h)
        for (int i = 0; i < 7; ++i) d.q[i] = p[i];
        break;
    case VRT_MEDIUM_N2P:
        // Sec. VI, Eq. (27); w = (R^2 - rho^2/4)/F^2 > 0 for rho < 2R, which the lens
        // (rho <= R) keeps
        if (!(p[0] > 0.0) || !(p[1] > 0.0)) {
            delete m;
            return fail(VRT_EINVAL, "N2P lens needs R > 0 and F > 0");
        }
        for (int i = 0; i < 4; ++i) d.q[i] = p[i];
        break;
    case VRT_MEDIUM_ZERNIKE: {
        // Sec. V; the terms are folded into a 16 x 4 table c[j - 1][l] (media.h)
        const int K = n_params >= 5 ? (int)p[4] : -1;
        if (n_params < 5 || (double)K != p[4] || K < 0 || K > 64 || n_params != 5 + 3 * K) {
            delete m;
            return fail(VRT_EINVAL, "zernike medium: [n_lo, n_hi, rho_max, z_max, K, (j, l, c) x K], "
                                    "K in [0, 64]");
        }
        if (!(p[2] > 0.0) || !(p[3] > 0.0)) {
            delete m;
            return fail(VRT_EINVAL, "zernike medium: rho_max and z_max must be > 0");
        }
        std::vector<double> tab(64, 0.0);
        int mask = 0;
        for (int k = 0; k < K; ++k) {
            const double *t = p + 5 + 3 * k;
            const int j = (int)t[0], l = (int)t[1];
            if ((double)j != t[0] || (double)l != t[1] || j < 1 || j > 16 || l < 0 || l > 3) {
                delete m;
                return fail(VRT_EINVAL, "zernike term %d: Fringe index j in [1, 16] and Legendre "
                                        "order l in [0, 3]", k);
            }
            tab[4 * (j - 1) + l] += t[2];
        }
        for (int j = 0; j < 16; ++j)
            if (tab[4 * j] != 0.0 || tab[4 * j + 1] != 0.0 || tab[4 * j + 2] != 0.0 ||
                tab[4 * j + 3] != 0.0)
                mask |= 1 << j;
        d.q[0] = 0.5 * (p[1] + p[0]);
        d.q[1] = 0.5 * (p[1] - p[0]);
        d.q[2] = p[2];
        d.q[3] = p[3];
        d.K = mask;
        void *pd = nullptr;
        if ((rc = dev_alloc(m, &pd, tab.size() * sizeof(double)))) {
            free_medium(m);
            return rc;
        }
        hipError_t e = hipMemcpyAsync(pd, tab.data(), tab.size() * sizeof(double),
                                      hipMemcpyHostToDevice, ctx->aux);
        if (e == hipSuccess) e = medium_ready(m);
        if (e != hipSuccess) {
            free_medium(m);
            return fail_hip(e, "hipMemcpy (zernike coefficients)");
        }
        d.bumps_d = (const double *)pd;
        break;
    }
    case VRT_MEDIUM_GAUSSIAN: {
        if (n_params < 2) {
            delete m;
            return fail(VRT_EINVAL, "gaussian medium needs [n0, K, ...]");
        }
        const int K = (int)p[1];
        if ((double)K != p[1] || K < 0 || K > VRT_MAX_BUMPS || n_params != 2 + 5 * K) {
            delete m;
            return fail(VRT_EINVAL, "gaussian medium: K=%g invalid or n_params %d != 2+5K", p[1],
                        n_params);
        }
        d.q[0] = p[0];
        f.q[0] = (float)p[0];
        d.K = K;
        std::vector<double> bd((size_t)kBumpD * (K > 0 ? K : 1), 0.0);
        std::vector<float> bf((size_t)kBumpF * (K > 0 ? K : 1), 0.0f);
        double amp = 0.0, sig_min = INFINITY;
        for (int k = 0; k < K; ++k) {
            const double *q = p + 2 + 5 * k;
            if (!(q[1] > 0.0)) {
                delete m;
                return fail(VRT_EINVAL, "gaussian bump %d: sigma must be > 0", k);
            }
            amp += fabs(q[0]);
            sig_min = fmin(sig_min, q[1]);
            for (int i = 0; i < 5; ++i) bd[(size_t)kBumpD * k + i] = q[i];
            fill_bump_f(q, bf.data() + (size_t)kBumpF * k);
        }
        if (!(p[0] - amp > 0.0)) {
            delete m;
            return fail(VRT_EINVAL, "gaussian medium: n0 - sum|A| must be > 0");
        }
        // step bounds of the single-precision index difference (media.h)
        const double nmin_sig = (p[0] - amp) * sig_min;
        f.q[1] = (float)(kGaussRho3 * nmin_sig);
        f.q[2] = (float)(p[0] - (double)f.q[0]);
        m->fp32_max_dL0 = kGaussRhoMax * nmin_sig;
        void *pd = nullptr, *pf = nullptr;
        if ((rc = dev_alloc(m, &pd, bd.size() * sizeof(double))) ||
            (rc = dev_alloc(m, &pf, bf.size() * sizeof(float)))) {
            free_medium(m);
            return rc;
        }
        hipError_t e = hipMemcpyAsync(pd, bd.data(), bd.size() * sizeof(double),
                                      hipMemcpyHostToDevice, ctx->aux);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pf, bf.data(), bf.size() * sizeof(float), hipMemcpyHostToDevice,
                               ctx->aux);
        if (e == hipSuccess) e = medium_ready(m);
        if (e != hipSuccess) {
            free_medium(m);
            return fail_hip(e, "hipMemcpy (gaussian params)");
        }
        d.bumps_d = (const double *)pd;
        d.bumps_f = (const float *)pf;
        break;
    }
    }
    ctx->n_media++;
    *out = m;
    return VRT_OK;
}

int vrt_medium_create_grid(vrt_context_t ctx, const float *values, int nx, int ny, int nz,
                           const double lo[3], const double hi[3], double n_ambient,
                           int values_on_device, vrt_medium_t *out) {
    if (!ctx || !out || !values || !lo || !hi)
        return fail(VRT_EINVAL, "vrt_medium_create_grid: NULL argument");
    if (nx < 2 || ny < 2 || nz < 2 || nx > 4096 || ny > 4096 || nz > 4096)
        return fail(VRT_EINVAL, "grid dimensions must be in [2, 4096], got %d x %d x %d", nx, ny, nz);
    if (!finite_all(lo, 3) || !finite_all(hi, 3) || !(lo[0] < hi[0]) || !(lo[1] < hi[1]) ||
        !(lo[2] < hi[2]))
        return fail(VRT_EINVAL, "grid extent needs finite lo < hi");
    if (!(n_ambient > 0.0) || !isfinite(n_ambient))
        return fail(VRT_EINVAL, "n_ambient must be finite and > 0");
    if (values_on_device && !gpu_accessible(values))
        return fail(VRT_EINVAL, "vrt_medium_create_grid: values_on_device set for pageable host "
                                "memory");
    int rc = set_device(ctx);
    if (rc) return rc;
    auto *m = new vrt_medium_s();
    m->ctx = ctx;
    m->async_allocs = ctx->async_pools;
    m->bnd.kind = VRT_BOUNDARY_BOX;
    for (int a = 0; a < 3; ++a) {
        m->bnd.p[a] = lo[a];
        m->bnd.p[a + 3] = hi[a];
    }
    for (int i = 0; i < 6; ++i) m->bnd.pf[i] = (float)m->bnd.p[i];
    MediumDev &d = m->dev;
    d.kind = VRT_MEDIUM_GRID;
    d.n_amb = n_ambient;
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    const int nn[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = lo[a];
        d.hi[a] = hi[a];
        d.h[a] = (hi[a] - lo[a]) / (double)(nn[a] - 1);
        d.inv_h[a] = 1.0 / d.h[a];
        d.flo[a] = (float)lo[a];
        d.fhi[a] = (float)hi[a];
        d.finv_h[a] = (float)d.inv_h[a];
    }
    const size_t total = (size_t)nx * ny * nz;
    void *g = nullptr, *r = nullptr, *bad = nullptr;
    if ((rc = dev_alloc(m, &g, total * sizeof(float))) ||
        (rc = dev_alloc(m, &r, total * sizeof(float4)))) {
        free_medium(m);
        return rc;
    }
    // uploads and the record kernel run on the library stream (a device-side
    // `values` array must be complete when this is called)
    hipStream_t st = ctx->aux;
    hipError_t e = hipMemcpyAsync(g, values, total * sizeof(float),
                                  values_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  st);
    if (e == hipSuccess)
        e = m->async_allocs ? hipMallocAsync(&bad, sizeof(unsigned int), st)
                            : hipMalloc(&bad, sizeof(unsigned int));
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(unsigned int), st);
    if (e != hipSuccess) {
        if (bad) (void)(m->async_allocs ? hipFreeAsync(bad, st) : hipFree(bad));
        free_medium(m);
        return fail_hip(e, "vrt_medium_create_grid: copy");
    }
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(grid_records_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const float *)g, (float4 *)r, nx, ny, nz, (unsigned int *)bad);
    unsigned int hbad = 0;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = medium_ready(m);
    (void)(m->async_allocs ? hipFreeAsync(bad, st) : hipFree(bad));
    if (e != hipSuccess) {
        free_medium(m);
        return fail_hip(e, "vrt_medium_create_grid: records");
    }
    if (hbad & 1u) {
        free_medium(m);
        return fail(VRT_EINVAL, "grid values must be finite and > 0");
    }
    d.grid = (const float *)g;
    d.rec = (const float4 *)r;
    d.rec_exact = (hbad & 2u) ? 0 : 1;
    ctx->n_media++;
    *out = m;
    return VRT_OK;
}

int vrt_medium_destroy(vrt_medium_t m) {
    if (!m) return fail(VRT_EINVAL, "vrt_medium_destroy: NULL medium");
    if (m->jobs.load() != 0)
        return fail(VRT_EINVAL, "vrt_medium_destroy: %d server jobs on it are not done",
                    m->jobs.load());
    vrt_context_t ctx = m->ctx;
    int rc = set_device(ctx);
    if (rc) return rc;
    free_medium(m);  // deferred behind the launches that read it; the host does not wait
    ctx->n_media--;
    return VRT_OK;
}

int vrt_medium_device_bytes(vrt_medium_t m, size_t *out) {
    if (!m || !out) return fail(VRT_EINVAL, "vrt_medium_device_bytes: NULL argument");
    *out = m->bytes;
    return VRT_OK;
}

static bool aligned(const void *p, size_t a) { return p && ((uintptr_t)p % a) == 0; }


// Argument checks shared by vrt_trace and vrt_trace_paths.
static int check_trace_args(vrt_medium_t m, const vrt_trace_params *p, const vrt_rays *rays,
                            size_t n_rays, const char *who) {
    if (!m || !p || !rays) return fail(VRT_EINVAL, "%s: NULL argument", who);
    if (!(p->dL0 > 0.0) || !isfinite(p->dL0)) return fail(VRT_EINVAL, "%s: dL0 must be > 0", who);
    if (p->max_steps <= 0 || p->max_steps > 0xFFFFFFFFll)
        return fail(VRT_EINVAL, "%s: max_steps must be in [1, 2^32)", who);
    if (p->max_lanes < 0 || (p->precision == VRT_FP64 && p->max_lanes != 0))
        return fail(VRT_EINVAL, "%s: max_lanes must be >= 0 (and 0 for VRT_FP64)", who);
    if (!(p->eps_tan >= 0.0) || !(p->crit_rad >= 0.0) || !(p->tie_eps >= 0.0) ||
        !(p->tie_eps <= 1e-6))
        return fail(VRT_EINVAL, "%s: eps_tan, crit_rad >= 0 and tie_eps in [0, 1e-6]", who);
    if (p->precision != VRT_FP64 && p->precision != VRT_FP32_COMP)
        return fail(VRT_EINVAL, "%s: unknown precision %d", who, p->precision);
    if (n_rays >= (1ull << 31)) return fail(VRT_EINVAL, "%s: n_rays must be < 2^31", who);
    if (p->precision == VRT_FP32_COMP && p->dL0 > m->fp32_max_dL0)
        return fail(VRT_EINVAL,
                    "%s: dL0 = %g exceeds %g, the longest step the single-precision path "
                    "keeps accurate in this medium (0.05 n_min sigma_min); use VRT_FP64",
                    who, p->dL0, m->fp32_max_dL0);
    if (n_rays == 0) return VRT_OK;
    const size_t es = p->precision == VRT_FP64 ? 8 : 4;
    const void *ptrs[] = {rays->px, rays->py, rays->pz, rays->dx, rays->dy, rays->dz,
                          rays->ox, rays->oy, rays->oz, rays->odx, rays->ody, rays->odz};
    for (const void *q : ptrs)
        if (!aligned(q, es)) return fail(VRT_EINVAL, "%s: ray array NULL or misaligned", who);
    const void *uptrs[] = {rays->status, rays->steps, rays->n_tir, rays->n_btir, rays->flags};
    for (const void *q : uptrs)
        if (!aligned(q, 4)) return fail(VRT_EINVAL, "%s: result array NULL or misaligned", who);
    for (const void *q : ptrs)
        if (!gpu_accessible(q))
            return fail(VRT_EINVAL, "%s: a ray array is pageable host memory (not GPU-accessible)",
                        who);
    for (const void *q : uptrs)
        if (!gpu_accessible(q))
            return fail(VRT_EINVAL,
                        "%s: a result array is pageable host memory (not GPU-accessible)", who);
    return VRT_OK;
}

static void fill_launch(vrt_medium_t m, const vrt_trace_params *p, size_t n_rays, void *stream,
                        LaunchArgs &a) {
    a.m = m->dev;
    a.mf = m->mf;
    a.b = m->bnd;
    a.t.dL0 = p->dL0;
    a.t.max_steps = p->max_steps;
    a.t.eps_tan = p->eps_tan;
    a.t.crit_rad = p->crit_rad;
    a.t.tie_eps = p->tie_eps;
    a.t.has_plane = isnan(p->exit_plane_z) ? 0 : 1;
    a.t.plane_z = a.t.has_plane ? p->exit_plane_z : 0.0;
    a.n = (uint32_t)n_rays;
    a.stream = (hipStream_t)stream;
    a.num_cu = m->ctx->num_cu;
    a.blocks_per_cu = 0;
    a.max_blocks = p->max_lanes > 0 ? (uint32_t)((p->max_lanes + 255) / 256) : 0u;
}

static RaysDev<double> rays64(const vrt_rays *rays) {
    return RaysDev<double>{(const double *)rays->px, (const double *)rays->py,
                           (const double *)rays->pz, (const double *)rays->dx,
                           (const double *)rays->dy, (const double *)rays->dz,
                           (double *)rays->ox, (double *)rays->oy, (double *)rays->oz,
                           (double *)rays->odx, (double *)rays->ody, (double *)rays->odz,
                           rays->status, rays->steps, rays->n_tir, rays->n_btir, rays->flags};
}

int vrt_trace(vrt_medium_t m, const vrt_trace_params *p, const vrt_rays *rays, size_t n_rays,
              void *stream) {
    if (int rc = check_trace_args(m, p, rays, n_rays, "vrt_trace")) return rc;
    if (n_rays == 0) return VRT_OK;
    vrt_context_t ctx = m->ctx;
    int rc = set_device(ctx);
    if (rc) return rc;
    bool captured = false;
    if ((rc = stream_captured((hipStream_t)stream, captured))) return rc;
    LaunchArgs a{};
    fill_launch(m, p, n_rays, stream, a);
    hipError_t e;
    if (p->precision == VRT_FP64) {
        a.io64 = rays64(rays);
        e = launch_march_fp64(a);
    } else {
        a.io32 = RaysDev<float>{(const float *)rays->px, (const float *)rays->py,
                                (const float *)rays->pz, (const float *)rays->dx,
                                (const float *)rays->dy, (const float *)rays->dz,
                                (float *)rays->ox, (float *)rays->oy, (float *)rays->oz,
                                (float *)rays->odx, (float *)rays->ody, (float *)rays->odz,
                                rays->status, rays->steps, rays->n_tir, rays->n_btir, rays->flags};
        std::lock_guard<std::mutex> lk(ctx->slot_mu);
        uint32_t slot;
        if (captured) {
            if (ctx->n_captured >= (uint32_t)(kQueueSlots - kEagerSlots))
                return fail(VRT_ENOMEM, "vrt_trace: %d single-precision traces captured in graphs "
                                        "on this context already (each keeps its queue slot)",
                            kQueueSlots - kEagerSlots);
            slot = kEagerSlots + ctx->n_captured++;
        } else {
            slot = ctx->next_eager++ % kEagerSlots;
            if (ctx->slot_recorded[slot])  // the slot's previous launch ends first
                HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, ctx->slot_ev[slot], 0),
                        "vrt_trace: hipStreamWaitEvent");
        }
        a.queue = ctx->queues + (size_t)slot * kQueueStride;
        // media marched from stored entry states get room for them from the
        // stream-ordered pool, freed behind the march on the same stream; a
        // captured launch, or one the pool cannot serve, enters rays inline
        a.entry = nullptr;
        if (!captured && ctx->async_pools && fp32c_pre_entry(m->dev.kind)) {
            void *buf = nullptr;
            if (hipMallocAsync(&buf, (size_t)n_rays * 80u, (hipStream_t)stream) == hipSuccess)
                a.entry = (EntryState *)buf;
            else
                (void)hipGetLastError();  // not sticky: the launch goes on without the states
        }
        e = launch_march_fp32c(a);
        if (a.entry) {
            const hipError_t ef = hipFreeAsync(a.entry, (hipStream_t)stream);
            if (e == hipSuccess) e = ef;
        }
        if (e == hipSuccess && !captured) {
            e = hipEventRecord(ctx->slot_ev[slot], (hipStream_t)stream);
            if (e == hipSuccess) ctx->slot_recorded[slot] = true;
        }
    }
    if (e != hipSuccess) return fail_hip(e, "vrt_trace: launch");
    return note_use(m, (hipStream_t)stream, captured);
}

int vrt_trace_paths(vrt_medium_t m, const vrt_trace_params *p, const vrt_rays *rays,
                    size_t n_rays, double *path, uint64_t cap, uint64_t *n_points, void *stream) {
    if (int rc = check_trace_args(m, p, rays, n_rays, "vrt_trace_paths")) return rc;
    if (p->precision != VRT_FP64)
        return fail(VRT_EINVAL, "vrt_trace_paths: paths are recorded by the VRT_FP64 march");
    if (cap == 0 || cap > (1ull << 40) || (n_rays > 0 && cap > SIZE_MAX / 24 / n_rays))
        return fail(VRT_EINVAL, "vrt_trace_paths: cap must be in [1, 2^40] with n_rays * cap * 24 "
                                "bytes addressable");
    if (n_rays == 0) return VRT_OK;
    if (!aligned(path, 8) || !aligned(n_points, 8))
        return fail(VRT_EINVAL, "vrt_trace_paths: path or n_points NULL or misaligned");
    if (!gpu_accessible(path) || !gpu_accessible(n_points))
        return fail(VRT_EINVAL, "vrt_trace_paths: path or n_points is pageable host memory");
    int rc = set_device(m->ctx);
    if (rc) return rc;
    bool captured = false;
    if ((rc = stream_captured((hipStream_t)stream, captured))) return rc;
    LaunchArgs a{};
    fill_launch(m, p, n_rays, stream, a);
    a.io64 = rays64(rays);
    hipError_t e = launch_paths_fp64(a, path, cap, n_points);
    if (e != hipSuccess) return fail_hip(e, "vrt_trace_paths: launch");
    return note_use(m, (hipStream_t)stream, captured);
}

int vrt_reduce_counters(vrt_context_t ctx, const vrt_rays *rays, size_t n_rays, vrt_counters *out,
                        void *stream) {
    if (!ctx || !rays || !out) return fail(VRT_EINVAL, "vrt_reduce_counters: NULL argument");
    if (n_rays > 0 && (!aligned(rays->status, 4) || !aligned(rays->steps, 4) ||
                       !aligned(rays->n_tir, 4) || !aligned(rays->n_btir, 4) ||
                       !aligned(rays->flags, 4)))
        return fail(VRT_EINVAL, "vrt_reduce_counters: result array NULL or misaligned");
    if (n_rays > 0) {
        const void *uptrs[] = {rays->status, rays->steps, rays->n_tir, rays->n_btir, rays->flags};
        for (const void *q : uptrs)
            if (!gpu_accessible(q))
                return fail(VRT_EINVAL, "vrt_reduce_counters: a result array is pageable host "
                                        "memory (not GPU-accessible)");
    }
    int rc = set_device(ctx);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->counters_mu);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long h[kNumCounters] = {0};
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, ctx->counters, kNumCounters);
    if (n_rays > 0) {
        size_t blocks = (n_rays + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(reduce_counters_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           rays->status, rays->steps, rays->n_tir, rays->n_btir, rays->flags,
                           n_rays, ctx->counters);
    }
    HIP_TRY(hipGetLastError(), "vrt_reduce_counters: launch");
    HIP_TRY(hipMemcpyAsync(h, ctx->counters, sizeof h, hipMemcpyDeviceToHost, s),
            "vrt_reduce_counters: copy");
    HIP_TRY(hipStreamSynchronize(s), "vrt_reduce_counters: synchronize");
    out->rays = h[0];
    out->steps = h[1];
    out->exited = h[2];
    out->missed = h[3];
    out->truncated = h[4];
    out->no_plane = h[5];
    out->invalid = h[6];
    out->reflected_at_entry = h[7];
    out->tir_interior = h[8];
    out->tir_boundary = h[9];
    out->flagged_near_critical = h[10];
    out->tangent = h[11];
    out->straight = h[12];
    out->flagged_near_tie = h[13];
    out->flagged_near_grazing = h[14];
    return VRT_OK;
}

}  // extern "C"
