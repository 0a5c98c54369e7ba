// march_fp32c.hip -- persistent batch kernel of the single-precision
// compensated VRT march: lanes refilled from the batch's ray queue.  For the
// grid and Zernike-lens media an eager launch first enters every ray in a
// kernel of its own and the march starts rays from the stored states.
#include "lane32.h"

namespace vrt {

// Everything a launch reads, passed as one kernel argument and read through a
// pointer: the fields of the rare paths are then loaded when used instead of
// being held in scalar registers for the whole kernel.
struct Launch32 {
    MediumDev m;
    MedF mf;
    BoundaryDev b;
    TraceDev t;
    RaysDev<float> io;
};

// Media whose launches run the entry kernel first when the library can hold
// the entry states (80 bytes per ray): without the double-precision entry
// code the grid and Zernike-lens marches fit 3 waves per SIMD instead of 2.
template <int MK>
constexpr bool kPreEntry = MK == VRT_MEDIUM_GRID || MK == VRT_MEDIUM_ZERNIKE;

template <int MK, bool kPre>
constexpr int march_occupancy() {
    return (MK == VRT_MEDIUM_GRID || MK == VRT_MEDIUM_ZERNIKE) && !kPre ? 2 : 3;
}

// One thread per ray: launch, flight to the enclosing surface and entry
// refraction (lane_init); rays that end there are written, the others'
// states stored for the march.
template <int MK>
__global__ __launch_bounds__(256) void entry_kernel(Launch32 desc, const float4 *__restrict__ rec,
                                                    uint32_t n, EntryState *__restrict__ es) {
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r >= n) return;
    const Launch32 *__restrict__ D = &desc;
    Lane L;
    GridCache gc;
    grid_invalidate(gc);
    L.r = r;
    const bool active = lane_init<MK>(D->m, rec, D->b, D->t, D->io, L, gc);
    EntryState e;
    entry_store<MK>(L, active, e);
    es[r] = e;
}

template <int MK, bool kPre>
__global__ __launch_bounds__(256, (march_occupancy<MK, kPre>())) void march_fp32c_kernel(
    Launch32 desc, const float *__restrict__ bumps, const float4 *__restrict__ rec, uint32_t n,
    uint32_t *queue, const EntryState *__restrict__ es) {
    const Launch32 *__restrict__ D = &desc;
    const MediumDev &m = D->m;
    const MedF &mf = D->mf;
    const BoundaryDev &b = D->b;
    const TraceDev &t = D->t;
    const RaysDev<float> &io = D->io;
    Lane L;
    GridCache gc;
    grid_invalidate(gc);
    bool active = false, done = false;
    const float dL0 = (float)t.dL0;
    const float eps_tan = (float)t.eps_tan;
    const float crit_f = (float)t.crit_rad;
    // a step whose end is this far inside cannot be within tie_eps of a cut
    const float mrg = fmaxf(2e-6f, 4.0f * (float)t.tie_eps);
    const int lane = __lane_id();
    // wave masks (uniform): lanes with a ray, lanes that found the queue empty.
    // Waves are always full (256-lane blocks), so a lane needs a ray iff its
    // bit is in neither mask.
    uint64_t act = 0, done_m = 0;
    // Media evaluated in double end their traces with a few rays trapped
    // along a wall, each a long dependent chain of FP64 work per step: a wave
    // that holds a ray past a sixth of the step cap raises its issue priority,
    // so that such rays advance while the device is still full instead of
    // alone at the end.  (The other media gain nothing from it: their long
    // rays are short chains, and the per-step test costs them ~2 %.)
    const uint32_t long_steps =
        (uint32_t)(t.max_steps / 6 > 1024 ? (t.max_steps / 6 < 0x7FFFFFFF ? t.max_steps / 6 : 0x7FFFFFFF)
                                          : 1024);
    bool raised = false;
    for (;;) {
        const uint64_t nm = ~(act | done_m);
        if (nm) {  // refill idle lanes from the queue with one atomic per wave
            const bool need = !active && !done;
            const int leader = __ffsll((unsigned long long)nm) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(queue, (uint32_t)__popcll(nm));
            base = __shfl(base, leader);
            if (need) {
                const uint32_t r = base + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull));
                if (r >= n) {
                    done = true;
                } else {
                    L.r = r;
                    if constexpr (kPre) {
                        active = lane_load<MK>(es, L, gc);
                    } else {
                        active = lane_init<MK>(m, rec, b, t, io, L, gc);
                    }
                }
            }
            done_m = __ballot(done);
            act = __ballot(active);
        }
        if (!act && done_m == ~0ull) break;
        if (active) active = lane_step<MK>(m, mf, bumps, rec, b, t, io, L, gc, dL0, eps_tan, mrg,
                                           crit_f);
        act = __ballot(active);
        if constexpr (kIndexIn64<MK>) {
            const bool hold_long = __ballot(active && L.steps > long_steps) != 0;
            if (hold_long != raised) {
                if (hold_long) __builtin_amdgcn_s_setprio(3);
                else __builtin_amdgcn_s_setprio(0);
                raised = hold_long;
            }
        }
    }
}

__global__ void queue_reset_kernel(uint32_t *q) { *q = 0u; }

template <int MK, bool kPre>
static hipError_t launch32(const LaunchArgs &a) {
    static int occ = -1;
    if (occ < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, march_fp32c_kernel<MK, kPre>, 256,
                                                         0) != hipSuccess ||
            nb <= 0)
            nb = 4;
        occ = nb;
    }
    const int per_cu = a.blocks_per_cu > 0 ? a.blocks_per_cu : occ;
    uint32_t blocks = (uint32_t)(a.num_cu > 0 ? a.num_cu : 256) * (uint32_t)per_cu;
    const uint32_t need = (a.n + 255u) / 256u;
    if (blocks > need) blocks = need;
    if (a.max_blocks > 0 && blocks > a.max_blocks) blocks = a.max_blocks;
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, a.stream, a.queue);
    const Launch32 desc{a.m, a.mf, a.b, a.t, a.io32};
    if constexpr (kPre)
        hipLaunchKernelGGL(entry_kernel<MK>, dim3((a.n + 255u) / 256u), dim3(256), 0, a.stream,
                           desc, a.m.rec, a.n, a.entry);
    hipLaunchKernelGGL((march_fp32c_kernel<MK, kPre>), dim3(blocks), dim3(256), 0, a.stream, desc,
                       a.m.bumps_f, a.m.rec, a.n, a.queue, (const EntryState *)a.entry);
    return hipGetLastError();
}

template <int MK>
static hipError_t launch32(const LaunchArgs &a) {
    if constexpr (kPreEntry<MK>) {
        if (a.entry) return launch32<MK, true>(a);
    }
    return launch32<MK, false>(a);
}

bool fp32c_pre_entry(int kind) {
    switch (kind) {
    case VRT_MEDIUM_GRID: return kPreEntry<VRT_MEDIUM_GRID>;
    case VRT_MEDIUM_ZERNIKE: return kPreEntry<VRT_MEDIUM_ZERNIKE>;
    default: return false;
    }
}

hipError_t launch_march_fp32c(const LaunchArgs &a) {
    if (a.n == 0) return hipSuccess;
    switch (a.m.kind) {
    case VRT_MEDIUM_HOMOGENEOUS: return launch32<VRT_MEDIUM_HOMOGENEOUS>(a);
    case VRT_MEDIUM_LINEAR: return launch32<VRT_MEDIUM_LINEAR>(a);
    case VRT_MEDIUM_LUNEBURG: return launch32<VRT_MEDIUM_LUNEBURG>(a);
    case VRT_MEDIUM_FIBER: return launch32<VRT_MEDIUM_FIBER>(a);
    case VRT_MEDIUM_GAUSSIAN: return launch32<VRT_MEDIUM_GAUSSIAN>(a);
    case VRT_MEDIUM_GRID: return launch32<VRT_MEDIUM_GRID>(a);
    case VRT_MEDIUM_SPHERICAL: return launch32<VRT_MEDIUM_SPHERICAL>(a);
    case VRT_MEDIUM_N2P: return launch32<VRT_MEDIUM_N2P>(a);
    case VRT_MEDIUM_ZERNIKE: return launch32<VRT_MEDIUM_ZERNIKE>(a);
    }
    return hipErrorInvalidValue;
}

}  // namespace vrt
