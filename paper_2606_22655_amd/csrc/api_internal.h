// api_internal.h -- host-side handles and error helpers shared by the
// library's translation units (vrt_api.hip, serve.hip).  Not installed.
#pragma once

#include <math.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "dispatch.h"

namespace vrt {

// Record a message for vrt_last_error() (thread-local) and return code.
int fail(int code, const char *fmt, ...);
// device, managed or pinned host memory (a kernel may touch it); false for
// pageable host memory
bool gpu_accessible(const void *p);
int fail_hip(hipError_t e, const char *what);

}  // namespace vrt

#define HIP_TRY(call, what)                                        \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::vrt::fail_hip(e_, (what));  \
    } while (0)

// Ray-queue counters of the single-precision batch kernel.  The first
// kEagerSlots are recycled round-robin by eager launches, each guarded by an
// event: a launch that takes a slot first makes its stream wait for the slot's
// previous launch.  A launch captured in a graph takes one of the other slots
// for good (the graph replays on it), so no eager launch ever shares it.
static constexpr int kQueueSlots = 1024;
static constexpr int kEagerSlots = 64;
static constexpr int kQueueStride = 16;  // uint32 per slot: one 64-byte line each
static constexpr int kNumCounters = 15;

struct vrt_context_s {
    int device = 0;
    int num_cu = 256;
    uint32_t *queues = nullptr;  // kQueueSlots ray-queue counters
    unsigned long long *counters = nullptr;
    hipStream_t aux = nullptr;   // library stream: medium uploads and stream-ordered frees
    std::mutex slot_mu;          // guards the slot state below
    hipEvent_t slot_ev[kEagerSlots] = {};
    bool slot_recorded[kEagerSlots] = {};
    uint32_t next_eager = 0;
    uint32_t n_captured = 0;     // slots given to captured launches
    bool async_pools = false;    // the device has the stream-ordered allocator
    std::atomic<int> n_media{0};
    std::atomic<int> n_servers{0};
    std::mutex counters_mu;
};

// The last launch on a medium from one stream (its event), for the deferred free.
struct MediumUse {
    hipStream_t stream;
    hipEvent_t ev;
};

struct vrt_medium_s {
    vrt_context_t ctx = nullptr;
    vrt::MediumDev dev{};
    vrt::MedF mf{};
    double fp32_max_dL0 = INFINITY;  // longest step the single-precision path accepts
    vrt::BoundaryDev bnd{};
    size_t bytes = 0;
    std::vector<void *> allocs;
    bool async_allocs = true;  // allocs come from the stream-ordered allocator
    std::mutex use_mu;
    std::vector<MediumUse> uses;  // eager launches that may still read the medium
    std::atomic<int> jobs{0};  // server jobs submitted on it and not yet done
};

inline int set_device(vrt_context_t c) {
    HIP_TRY(hipSetDevice(c->device), "hipSetDevice");
    return VRT_OK;
}
