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

static constexpr int kQueueSlots = 1024;
static constexpr int kQueueStride = 16;  // uint32 per slot: one 64-byte line each
static constexpr int kNumCounters = 15;

struct vrt_context_s {
    int device = 0;
    int num_cu = 256;
    uint32_t *queues = nullptr;  // kQueueSlots ray-queue counters
    unsigned long long *counters = nullptr;
    std::atomic<uint32_t> next_slot{0};
    std::atomic<int> n_media{0};
    std::atomic<int> n_servers{0};
    std::mutex counters_mu;
};

struct vrt_medium_s {
    vrt_context_t ctx = nullptr;
    vrt::MediumDev dev{};
    vrt::MedF mf{};
    double fp32_max_dL0 = INFINITY;  // longest step the single-precision path accepts
    vrt::BoundaryDev bnd{};
    size_t bytes = 0;
    std::vector<void *> allocs;
    std::atomic<int> jobs{0};  // server jobs submitted on it and not yet done
};

inline int set_device(vrt_context_t c) {
    HIP_TRY(hipSetDevice(c->device), "hipSetDevice");
    return VRT_OK;
}
