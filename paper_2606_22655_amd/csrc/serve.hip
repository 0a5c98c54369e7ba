// serve.hip -- continuous batching of trace jobs: one persistent kernel
// marches the rays of every admitted job while a host thread admits new jobs
// into a device pool of fixed size, publishes them to the running kernel and
// copies finished jobs back.
//
// Device protocol (per server):
//   table[kSlots]  job descriptors (device), slot = sequence % kSlots, written
//                  by an input copy before the job is published;
//   ctl[kSlots]    per slot: 64-bit claim word (sequence << 32 | next ray to
//                  hand out), rays not yet retired, sum of retired steps;
//   sc             pinned host words: tail (jobs [0, tail) are published),
//                  stop;
//   done[kSlots]   pinned host records: sequence + 1 and the ray-step total of
//                  the job that last finished in the slot.
// A wave works on one job at a time (the medium is uniform across its lanes).
// Its idle lanes claim rays of that job with one compare-and-swap on the claim
// word, which also checks that the slot still holds the job; once the job has
// no rays left to hand out and the wave's lanes have retired theirs, the wave
// moves to the next published job with unclaimed rays.  Adopting a job is an
// acquire at system scope (it reads the tail the host wrote), which
// invalidates the wave's L2 so that the job's descriptor and inputs, copied in
// while the kernel ran, are read fresh.  Retiring rays is a release at agent
// scope before the count of unretired rays is decremented, so outputs reach
// memory; the wave that retires the last ray of a job writes its done record
// with a system-scope release.  A wave with no job polls the tail, sleeping
// between polls, and leaves after kIdlePolls empty polls or when stop is set;
// the host relaunches the kernel (a captured hipGraph) when jobs are published
// and it is not running.
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "api_internal.h"
#include "lane32.h"

namespace vrt {
namespace serve {

constexpr uint32_t kSlots = 4096;   // job table ring
constexpr size_t kDescBytes = 1024;  // one descriptor slot
constexpr uint32_t kIdlePolls = 600; // ~2 ms of empty polls before a wave leaves

struct alignas(16) JobDesc {
    MediumDev m;
    MedF mf;
    BoundaryDev b;
    TraceDev t;
    RaysDev<float> io;
    uint32_t n;
    int32_t kind;
    float dL0, eps_tan, mrg, crit;
};
static_assert(sizeof(JobDesc) <= kDescBytes, "job descriptor slot");
static_assert(sizeof(JobDesc) % 16 == 0, "descriptor copied in 16-byte pieces");

struct JobCtl {
    unsigned long long claim;  // (sequence << 32) | next ray index to hand out
    uint32_t left;             // rays not retired yet
    uint32_t pad;
    unsigned long long steps;  // steps of the retired rays
    unsigned long long pad2;
};

struct ServeCtl {
    uint32_t tail;
    uint32_t stop;
    uint32_t pad[14];
};

struct DoneRec {
    unsigned long long steps;
    uint32_t seq1;  // sequence + 1 of the finished job
    uint32_t pad;
};

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
template <class T>
__device__ __forceinline__ T *rfl_ptr(T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

template <int MK>
__device__ __forceinline__ bool init_k(const JobDesc &D, const float4 *rec, Lane &L, GridCache &gc) {
    return lane_init<MK>(D.m, rec, D.b, D.t, D.io, L, gc);
}
template <int MK>
__device__ __forceinline__ bool step_k(const JobDesc &D, const float *bumps, const float4 *rec,
                                       Lane &L, GridCache &gc) {
    return lane_step<MK>(D.m, D.mf, bumps, rec, D.b, D.t, D.io, L, gc, D.dL0, D.eps_tan, D.mrg,
                         D.crit);
}

__device__ __forceinline__ bool init_any(int kind, const JobDesc &D, const float4 *rec, Lane &L,
                                         GridCache &gc) {
    switch (kind) {
    case VRT_MEDIUM_HOMOGENEOUS: return init_k<VRT_MEDIUM_HOMOGENEOUS>(D, rec, L, gc);
    case VRT_MEDIUM_LINEAR: return init_k<VRT_MEDIUM_LINEAR>(D, rec, L, gc);
    case VRT_MEDIUM_LUNEBURG: return init_k<VRT_MEDIUM_LUNEBURG>(D, rec, L, gc);
    case VRT_MEDIUM_FIBER: return init_k<VRT_MEDIUM_FIBER>(D, rec, L, gc);
    case VRT_MEDIUM_GAUSSIAN: return init_k<VRT_MEDIUM_GAUSSIAN>(D, rec, L, gc);
    default: return init_k<VRT_MEDIUM_GRID>(D, rec, L, gc);
    }
}
__device__ __forceinline__ bool step_any(int kind, const JobDesc &D, const float *bumps,
                                         const float4 *rec, Lane &L, GridCache &gc) {
    switch (kind) {
    case VRT_MEDIUM_HOMOGENEOUS: return step_k<VRT_MEDIUM_HOMOGENEOUS>(D, bumps, rec, L, gc);
    case VRT_MEDIUM_LINEAR: return step_k<VRT_MEDIUM_LINEAR>(D, bumps, rec, L, gc);
    case VRT_MEDIUM_LUNEBURG: return step_k<VRT_MEDIUM_LUNEBURG>(D, bumps, rec, L, gc);
    case VRT_MEDIUM_FIBER: return step_k<VRT_MEDIUM_FIBER>(D, bumps, rec, L, gc);
    case VRT_MEDIUM_GAUSSIAN: return step_k<VRT_MEDIUM_GAUSSIAN>(D, bumps, rec, L, gc);
    default: return step_k<VRT_MEDIUM_GRID>(D, bumps, rec, L, gc);
    }
}

__global__ __launch_bounds__(256, 2) void serve_kernel(const JobDesc *__restrict__ table,
                                                       JobCtl *ctl, const ServeCtl *sc,
                                                       DoneRec *done, uint32_t *first_open) {
    __shared__ JobDesc wdesc[4];  // one descriptor per wave of the block
    JobDesc &D = wdesc[threadIdx.x >> 6];
    const int lane = __lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    Lane L;
    GridCache gc;
    gc.ci = -1;
    bool active = false;
    uint64_t act = 0;  // wave mask of lanes holding a ray
    uint32_t j = rfl(__hip_atomic_load(first_open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    bool have = false, exhausted = true;
    int kind = 0;
    uint32_t n = 0, slot = 0, idle = 0;
    const float *bumps = nullptr;
    const float4 *rec = nullptr;
    for (;;) {
        if (!act && (!have || exhausted)) {
            // the wave is empty: find the next published job with rays to hand out
            if (have) ++j;
            have = false;
            const uint32_t tail =
                rfl(__hip_atomic_load(&sc->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
            while (j < tail) {
                const uint32_t s = j % kSlots;
                const unsigned long long c =
                    __hip_atomic_load(&ctl[s].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t cs = rfl((uint32_t)(c >> 32)), cn = rfl((uint32_t)c);
                if (cs == j && cn < rfl(table[s].n)) break;
                ++j;
                if (lane == 0) atomicMax(first_open, j);
            }
            if (j >= tail) {
                if (__hip_atomic_load(&sc->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ||
                    ++idle > kIdlePolls)
                    break;
                __builtin_amdgcn_s_sleep(127);
                continue;
            }
            slot = j % kSlots;
            const uint4 *src = (const uint4 *)(table + slot);
            uint4 *dst = (uint4 *)&D;
            for (uint32_t q = lane; q < sizeof(JobDesc) / 16; q += 64) dst[q] = src[q];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            have = true;
            exhausted = false;
            idle = 0;
            kind = (int)rfl((uint32_t)D.kind);
            n = rfl(D.n);
            bumps = rfl_ptr(D.m.bumps_f);
            rec = rfl_ptr(D.m.rec);
            gc.ci = -1;
        }
        bool ended = false;
        if (!exhausted) {
            const uint64_t nm = ~act;  // lanes without a ray (waves are full)
            if (nm) {
                const uint32_t want = (uint32_t)__popcll(nm);
                const int leader = __ffsll((unsigned long long)nm) - 1;
                uint32_t base = 0, got = 0;
                if (lane == leader) {
                    unsigned long long c =
                        __hip_atomic_load(&ctl[slot].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    for (;;) {
                        const uint32_t cs = (uint32_t)(c >> 32), cn = (uint32_t)c;
                        if (cs != j || cn >= n) {  // job gone or no rays left
                            got = 0;
                            break;
                        }
                        const uint32_t take = min(want, n - cn);
                        if (__hip_atomic_compare_exchange_strong(
                                &ctl[slot].claim, &c, c + take, __ATOMIC_RELAXED,
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            base = cn;
                            got = take;
                            break;
                        }
                    }
                }
                base = rfl(__shfl(base, leader));
                got = rfl(__shfl(got, leader));
                if (got < want) exhausted = true;
                if (!active) {
                    const uint32_t k = (uint32_t)__popcll(nm & below);
                    if (k < got) {
                        L.r = base + k;
                        active = init_any(kind, D, rec, L, gc);
                        ended = !active;
                    }
                }
            }
        }
        if (active) {
            active = step_any(kind, D, bumps, rec, L, gc);
            ended = !active;
        }
        const uint64_t fin = __ballot(ended);
        if (fin) {
            if (ended)
                __hip_atomic_fetch_add(&ctl[slot].steps, (unsigned long long)L.steps,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();  // outputs and step sums before the retire count
            const int leader = __ffsll((unsigned long long)fin) - 1;
            if (lane == leader) {
                const uint32_t cnt = (uint32_t)__popcll(fin);
                const uint32_t old = __hip_atomic_fetch_sub(&ctl[slot].left, cnt, __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                if (old == cnt) {  // the job's last rays
                    const unsigned long long st = __hip_atomic_load(
                        &ctl[slot].steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __threadfence_system();
                    __hip_atomic_store(&done[slot].steps, st, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&done[slot].seq1, j + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
        act = __ballot(active);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct HostJob {
    uint32_t seq = 0;
    vrt_medium_t med = nullptr;
    vrt_trace_params p{};
    vrt_rays host{};
    size_t n = 0;
    size_t off = 0, bytes = 0;
    int state = VRT_JOB_QUEUED;
    int error = 0;
    uint64_t steps = 0;
    double t_submit = 0, t_admit = 0, t_start = 0, t_retired = 0, t_done = 0;
    hipEvent_t ev = nullptr;
};

// First-fit allocator over [0, size) in 256-byte units.
class Pool {
  public:
    void reset(size_t size) {
        free_.clear();
        free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = used_ > peak_ ? used_ : peak_;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

constexpr size_t kRayBytes = 6 * 4 + 6 * 4 + 5 * 4;  // inputs, outputs, per-ray words

}  // namespace serve
}  // namespace vrt

using namespace vrt;
using namespace vrt::serve;

struct vrt_server_s {
    vrt_context_t ctx = nullptr;
    size_t budget = 0;
    char *pool = nullptr;
    Pool alloc;
    JobDesc *table = nullptr;
    JobCtl *ctl = nullptr;
    uint32_t *first_open = nullptr;
    ServeCtl *sc = nullptr;         // pinned
    DoneRec *done = nullptr;        // pinned
    unsigned char *stage = nullptr; // pinned: descriptor + claim record per slot
    hipStream_t copy_s = nullptr, run_s = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_run = nullptr;
    bool running = false;
    uint32_t futile = 0;  // kernel runs since a job last retired
    uint32_t blocks = 0;
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::deque<HostJob *> queued, staged;
    std::vector<HostJob *> live, copying;
    std::unordered_map<uint64_t, HostJob *> jobs;
    uint32_t next_seq = 0;
    uint32_t in_flight = 0;  // admitted and not done
    bool quit = false;
    int fatal = 0;
    std::string fatal_msg;
    std::thread th;
    std::chrono::steady_clock::time_point t0;
    vrt_server_stats st{};

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static const int kStageBytes = (int)(kDescBytes + sizeof(JobCtl));

// Issue a job's input copies and its descriptor (scheduler thread, mu held).
static hipError_t stage_job(vrt_server_t s, HostJob *J) {
    const size_t n = J->n;
    char *base = s->pool + J->off;
    float *f = (float *)base;
    uint32_t *u = (uint32_t *)(base + 12 * n * sizeof(float));
    const void *in[6] = {J->host.px, J->host.py, J->host.pz, J->host.dx, J->host.dy, J->host.dz};
    hipError_t e = hipSuccess;
    for (int a = 0; a < 6 && e == hipSuccess; ++a)
        e = hipMemcpyAsync(f + a * n, in[a], n * sizeof(float), hipMemcpyHostToDevice, s->copy_s);
    if (e != hipSuccess) return e;
    const uint32_t slot = J->seq % kSlots;
    JobDesc d{};
    vrt_medium_t m = J->med;
    d.m = m->dev;
    d.mf = m->mf;
    d.b = m->bnd;
    d.t.dL0 = J->p.dL0;
    d.t.max_steps = J->p.max_steps;
    d.t.eps_tan = J->p.eps_tan;
    d.t.crit_rad = J->p.crit_rad;
    d.t.tie_eps = J->p.tie_eps;
    d.t.has_plane = isnan(J->p.exit_plane_z) ? 0 : 1;
    d.t.plane_z = d.t.has_plane ? J->p.exit_plane_z : 0.0;
    d.io = RaysDev<float>{f, f + n, f + 2 * n, f + 3 * n, f + 4 * n, f + 5 * n,
                          f + 6 * n, f + 7 * n, f + 8 * n, f + 9 * n, f + 10 * n, f + 11 * n,
                          u, u + n, u + 2 * n, u + 3 * n, u + 4 * n};
    d.n = (uint32_t)n;
    d.kind = m->dev.kind;
    d.dL0 = (float)J->p.dL0;
    d.eps_tan = (float)J->p.eps_tan;
    d.mrg = fmaxf(2e-6f, 4.0f * (float)J->p.tie_eps);
    d.crit = (float)J->p.crit_rad;
    JobCtl c{};
    c.claim = (unsigned long long)J->seq << 32;
    c.left = (uint32_t)n;
    unsigned char *st = s->stage + (size_t)slot * kStageBytes;
    memcpy(st, &d, sizeof d);
    memcpy(st + kDescBytes, &c, sizeof c);
    e = hipMemcpyAsync(s->table + slot, st, sizeof(JobDesc), hipMemcpyHostToDevice, s->copy_s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->ctl + slot, st + kDescBytes, sizeof(JobCtl), hipMemcpyHostToDevice,
                           s->copy_s);
    if (e == hipSuccess) e = hipEventRecord(J->ev, s->copy_s);
    return e;
}

static hipError_t fetch_job(vrt_server_t s, HostJob *J) {
    const size_t n = J->n;
    char *base = s->pool + J->off;
    float *f = (float *)base;
    uint32_t *u = (uint32_t *)(base + 12 * n * sizeof(float));
    void *outf[6] = {J->host.ox, J->host.oy, J->host.oz, J->host.odx, J->host.ody, J->host.odz};
    uint32_t *outu[5] = {J->host.status, J->host.steps, J->host.n_tir, J->host.n_btir,
                         J->host.flags};
    hipError_t e = hipSuccess;
    for (int a = 0; a < 6 && e == hipSuccess; ++a)
        e = hipMemcpyAsync(outf[a], f + (6 + a) * n, n * sizeof(float), hipMemcpyDeviceToHost,
                           s->copy_s);
    for (int a = 0; a < 5 && e == hipSuccess; ++a)
        e = hipMemcpyAsync(outu[a], u + a * n, n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           s->copy_s);
    if (e == hipSuccess) e = hipEventRecord(J->ev, s->copy_s);
    return e;
}

static void finish_job(vrt_server_t s, HostJob *J, int err) {
    J->state = VRT_JOB_DONE;
    J->error = err;
    J->t_done = s->now();
    s->alloc.release(J->off, J->bytes);
    s->in_flight--;
    J->med->jobs--;
    s->st.jobs_done++;
    s->st.rays_done += J->n;
    s->st.ray_steps_done += J->steps;
}

// One pass of the scheduler (mu held).  Returns true if anything moved.
static bool schedule_once(vrt_server_t s) {
    bool moved = false;
    hipError_t e = hipSuccess;
    // 1. admission in submission order: pool space and a job slot
    while (!s->queued.empty() && s->in_flight < kSlots - 1) {
        HostJob *J = s->queued.front();
        if (!s->alloc.alloc(J->bytes, &J->off)) break;
        s->queued.pop_front();
        s->in_flight++;
        s->st.pool_bytes = s->alloc.used();
        s->st.pool_peak_bytes = s->alloc.peak();
        J->state = VRT_JOB_STAGED;
        J->t_admit = s->now();
        if ((e = stage_job(s, J)) != hipSuccess) goto fail;
        s->staged.push_back(J);
        moved = true;
    }
    // 2. publish, in order, the jobs whose inputs have arrived
    while (!s->staged.empty()) {
        HostJob *J = s->staged.front();
        e = hipEventQuery(J->ev);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) goto fail;
        s->staged.pop_front();
        J->state = VRT_JOB_RUNNING;
        J->t_start = s->now();
        std::atomic_thread_fence(std::memory_order_seq_cst);
        __atomic_store_n(&s->sc->tail, J->seq + 1, __ATOMIC_RELEASE);
        s->live.push_back(J);
        moved = true;
    }
    // 3. the persistent kernel: relaunch when it idled out and work is live
    if (s->running) {
        e = hipEventQuery(s->ev_run);
        if (e == hipSuccess) s->running = false;
        else if (e != hipErrorNotReady) goto fail;
    }
    if (!s->running && !s->live.empty()) {
        // a run that retires nothing while jobs are live can only repeat: stop
        if (++s->futile > 2000) {
            s->fatal = VRT_EHIP;
            s->fatal_msg = "server: published jobs make no progress";
            return false;
        }
        if ((e = hipGraphLaunch(s->gexec, s->run_s)) != hipSuccess) goto fail;
        if ((e = hipEventRecord(s->ev_run, s->run_s)) != hipSuccess) goto fail;
        s->running = true;
        s->st.kernel_launches++;
        moved = true;
    }
    // 4. retired jobs: copy their outputs back
    for (size_t i = 0; i < s->live.size();) {
        HostJob *J = s->live[i];
        const DoneRec *d = &s->done[J->seq % kSlots];
        if (__atomic_load_n(&d->seq1, __ATOMIC_ACQUIRE) == J->seq + 1) {
            J->steps = __atomic_load_n(&d->steps, __ATOMIC_RELAXED);
            J->t_retired = s->now();
            J->state = VRT_JOB_COPYING;
            s->futile = 0;
            if ((e = fetch_job(s, J)) != hipSuccess) goto fail;
            s->copying.push_back(J);
            s->live[i] = s->live.back();
            s->live.pop_back();
            moved = true;
        } else {
            ++i;
        }
    }
    // 5. outputs in host memory: done
    for (size_t i = 0; i < s->copying.size();) {
        HostJob *J = s->copying[i];
        e = hipEventQuery(J->ev);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (e != hipSuccess) goto fail;
        finish_job(s, J, 0);
        s->copying[i] = s->copying.back();
        s->copying.pop_back();
        moved = true;
    }
    if (moved) s->cv_done.notify_all();
    return moved;
fail:
    s->fatal = e == hipErrorOutOfMemory ? VRT_ENOMEM : VRT_EHIP;
    s->fatal_msg = std::string("server: ") + hipGetErrorString(e);
    return false;
}

static void fail_all(vrt_server_t s) {
    for (auto *v : {&s->queued, &s->staged}) {
        for (HostJob *J : *v) {
            if (J->state != VRT_JOB_QUEUED) s->in_flight--;
            J->state = VRT_JOB_DONE;
            J->error = s->fatal;
            J->med->jobs--;
        }
        v->clear();
    }
    for (auto *v : {&s->live, &s->copying}) {
        for (HostJob *J : *v) {
            J->state = VRT_JOB_DONE;
            J->error = s->fatal;
            J->med->jobs--;
            s->in_flight--;
        }
        v->clear();
    }
    s->cv_done.notify_all();
}

static void scheduler(vrt_server_t s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->fatal) {
            fail_all(s);
            break;
        }
        const bool busy = !s->queued.empty() || !s->staged.empty() || !s->live.empty() ||
                          !s->copying.empty();
        if (s->quit && !busy) break;
        const bool moved = schedule_once(s);
        if (moved) continue;
        if (busy)  // work on the device: poll again soon
            s->cv_submit.wait_for(lk, std::chrono::microseconds(20));
        else
            s->cv_submit.wait_for(lk, std::chrono::milliseconds(5));
    }
}

static int server_free(vrt_server_t s) {
    int rc = VRT_OK;
    if (s->run_s && hipStreamSynchronize(s->run_s) != hipSuccess) rc = VRT_EHIP;
    if (s->copy_s && hipStreamSynchronize(s->copy_s) != hipSuccess) rc = VRT_EHIP;
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->ev_run) (void)hipEventDestroy(s->ev_run);
    for (auto &kv : s->jobs) {
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    if (s->run_s) (void)hipStreamDestroy(s->run_s);
    if (s->copy_s) (void)hipStreamDestroy(s->copy_s);
    if (s->pool) (void)hipFree(s->pool);
    if (s->table) (void)hipFree(s->table);
    if (s->ctl) (void)hipFree(s->ctl);
    if (s->first_open) (void)hipFree(s->first_open);
    if (s->sc) (void)hipHostFree(s->sc);
    if (s->done) (void)hipHostFree(s->done);
    if (s->stage) (void)hipHostFree(s->stage);
    if (s->ctx) s->ctx->n_servers--;
    delete s;
    return rc;
}

extern "C" int vrt_server_create(vrt_context_t ctx, size_t hbm_budget, int max_lanes,
                                 vrt_server_t *out) {
    if (!ctx || !out) return fail(VRT_EINVAL, "vrt_server_create: NULL argument");
    if (hbm_budget < (1u << 20)) return fail(VRT_EINVAL, "vrt_server_create: budget < 1 MiB");
    if (max_lanes < 0) return fail(VRT_EINVAL, "vrt_server_create: max_lanes < 0");
    int rc = set_device(ctx);
    if (rc) return rc;
    vrt_server_t s = new vrt_server_s();
    s->ctx = ctx;
    ctx->n_servers++;
    s->budget = hbm_budget & ~(size_t)255;
    s->alloc.reset(s->budget);
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e;
#define SV_TRY(call, what)                    \
    if ((e = (call)) != hipSuccess) {         \
        rc = fail_hip(e, "vrt_server_create: " what); \
        server_free(s);                       \
        return rc;                            \
    }
    SV_TRY(hipMalloc((void **)&s->pool, s->budget), "pool");
    SV_TRY(hipMalloc((void **)&s->table, sizeof(JobDesc) * kSlots), "job table");
    SV_TRY(hipMalloc((void **)&s->ctl, sizeof(JobCtl) * kSlots), "job counters");
    SV_TRY(hipMalloc((void **)&s->first_open, 256), "first-open word");
    SV_TRY(hipHostMalloc((void **)&s->sc, sizeof(ServeCtl), hipHostMallocCoherent), "control words");
    SV_TRY(hipHostMalloc((void **)&s->done, sizeof(DoneRec) * kSlots, hipHostMallocCoherent),
           "done records");
    SV_TRY(hipHostMalloc((void **)&s->stage, (size_t)kStageBytes * kSlots, hipHostMallocDefault),
           "staging");
    memset(s->sc, 0, sizeof(ServeCtl));
    memset(s->done, 0, sizeof(DoneRec) * kSlots);
    SV_TRY(hipStreamCreateWithFlags(&s->copy_s, hipStreamNonBlocking), "copy stream");
    SV_TRY(hipStreamCreateWithFlags(&s->run_s, hipStreamNonBlocking), "run stream");
    SV_TRY(hipEventCreateWithFlags(&s->ev_run, hipEventDisableTiming), "event");
    // claim words of empty slots name no job (sequence 0xffffffff)
    {
        std::vector<JobCtl> c0(kSlots);
        for (auto &c : c0) c.claim = 0xffffffffull << 32;
        SV_TRY(hipMemcpy(s->ctl, c0.data(), sizeof(JobCtl) * kSlots, hipMemcpyHostToDevice),
               "counter init");
        std::vector<JobDesc> d0(1);
        for (uint32_t k = 0; k < kSlots; ++k)
            SV_TRY(hipMemcpy(s->table + k, d0.data(), sizeof(JobDesc), hipMemcpyHostToDevice),
                   "table init");
        uint32_t z[64] = {0};
        SV_TRY(hipMemcpy(s->first_open, z, 256, hipMemcpyHostToDevice), "first-open init");
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, serve_kernel, 256, 0) != hipSuccess ||
        nb <= 0)
        nb = 1;
    s->blocks = (uint32_t)ctx->num_cu * (uint32_t)nb;
    if (max_lanes > 0) s->blocks = std::min(s->blocks, (uint32_t)((max_lanes + 255) / 256));
    s->st.job_slots = kSlots;
    s->st.lanes = s->blocks * 256;
    // capture the persistent kernel's launch once; relaunches replay it
    SV_TRY(hipStreamBeginCapture(s->run_s, hipStreamCaptureModeThreadLocal), "capture");
    hipLaunchKernelGGL(serve_kernel, dim3(s->blocks), dim3(256), 0, s->run_s, s->table, s->ctl,
                       s->sc, s->done, s->first_open);
    SV_TRY(hipStreamEndCapture(s->run_s, &s->graph), "capture end");
    SV_TRY(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0), "graph instantiate");
#undef SV_TRY
    s->th = std::thread(scheduler, s);
    *out = s;
    return VRT_OK;
}

extern "C" int vrt_server_submit(vrt_server_t s, vrt_medium_t m, const vrt_trace_params *p,
                                 const vrt_rays *host_rays, size_t n_rays, uint64_t *job) {
    if (!s || !m || !p || !host_rays || !job)
        return fail(VRT_EINVAL, "vrt_server_submit: NULL argument");
    if (m->ctx != s->ctx) return fail(VRT_EINVAL, "vrt_server_submit: medium of another context");
    if (p->precision != VRT_FP32_COMP || p->max_lanes != 0)
        return fail(VRT_EINVAL, "vrt_server_submit: precision must be VRT_FP32_COMP, max_lanes 0");
    if (!(p->dL0 > 0.0) || !isfinite(p->dL0) || p->max_steps <= 0 ||
        p->max_steps > 0xFFFFFFFFll || !(p->eps_tan >= 0.0) || !(p->crit_rad >= 0.0) ||
        !(p->tie_eps >= 0.0) || !(p->tie_eps <= 1e-6))
        return fail(VRT_EINVAL, "vrt_server_submit: trace parameters out of range");
    if (p->dL0 > m->fp32_max_dL0)
        return fail(VRT_EINVAL, "vrt_server_submit: dL0 = %g exceeds %g for this medium", p->dL0,
                    m->fp32_max_dL0);
    if (n_rays == 0 || n_rays >= (1ull << 31))
        return fail(VRT_EINVAL, "vrt_server_submit: n_rays must be in [1, 2^31)");
    const void *ptrs[] = {host_rays->px, host_rays->py, host_rays->pz, host_rays->dx,
                          host_rays->dy, host_rays->dz, host_rays->ox, host_rays->oy,
                          host_rays->oz, host_rays->odx, host_rays->ody, host_rays->odz,
                          host_rays->status, host_rays->steps, host_rays->n_tir,
                          host_rays->n_btir, host_rays->flags};
    for (const void *q : ptrs)
        if (!q || ((uintptr_t)q & 3)) return fail(VRT_EINVAL, "vrt_server_submit: NULL or misaligned array");
    const size_t bytes = ((n_rays * kRayBytes + 255) & ~(size_t)255) + 256;
    if (bytes > s->budget)
        return fail(VRT_EINVAL, "vrt_server_submit: %zu rays need %zu bytes, the pool has %zu",
                    n_rays, bytes, s->budget);
    HostJob *J = new HostJob();
    if (hipEventCreateWithFlags(&J->ev, hipEventDisableTiming) != hipSuccess) {
        delete J;
        return fail(VRT_EHIP, "vrt_server_submit: event");
    }
    J->med = m;
    J->p = *p;
    J->host = *host_rays;
    J->n = n_rays;
    J->bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->fatal) {
            (void)hipEventDestroy(J->ev);
            delete J;
            return fail(s->fatal, "%s", s->fatal_msg.c_str());
        }
        J->seq = s->next_seq++;
        J->t_submit = s->now();
        m->jobs++;
        s->jobs[J->seq] = J;
        s->queued.push_back(J);
        s->st.jobs_submitted++;
        *job = J->seq;
    }
    s->cv_submit.notify_one();
    return VRT_OK;
}

static void fill_info(const HostJob *J, vrt_job_info *out) {
    out->state = J->state;
    out->error = J->error;
    out->n_rays = J->n;
    out->ray_steps = J->steps;
    out->t_submit = J->t_submit;
    out->t_admit = J->t_admit;
    out->t_start = J->t_start;
    out->t_retired = J->t_retired;
    out->t_done = J->t_done;
}

extern "C" int vrt_server_query(vrt_server_t s, uint64_t job, vrt_job_info *out) {
    if (!s || !out) return fail(VRT_EINVAL, "vrt_server_query: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(VRT_EINVAL, "vrt_server_query: unknown job %llu",
                                         (unsigned long long)job);
    fill_info(it->second, out);
    return VRT_OK;
}

extern "C" int vrt_server_wait(vrt_server_t s, uint64_t job, double timeout_s, vrt_job_info *out) {
    if (!s || !out) return fail(VRT_EINVAL, "vrt_server_wait: NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return fail(VRT_EINVAL, "vrt_server_wait: unknown job %llu",
                                         (unsigned long long)job);
    HostJob *J = it->second;
    auto pred = [&] { return J->state == VRT_JOB_DONE; };
    if (timeout_s < 0)
        s->cv_done.wait(lk, pred);
    else
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
    fill_info(J, out);
    if (J->state != VRT_JOB_DONE) return fail(VRT_ETIMEOUT, "vrt_server_wait: job not done");
    if (J->error) return fail(J->error, "vrt_server_wait: job failed: %s", s->fatal_msg.c_str());
    return VRT_OK;
}

extern "C" int vrt_server_stats_get(vrt_server_t s, vrt_server_stats *out) {
    if (!s || !out) return fail(VRT_EINVAL, "vrt_server_stats_get: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return VRT_OK;
}

extern "C" int vrt_server_destroy(vrt_server_t s) {
    if (!s) return fail(VRT_EINVAL, "vrt_server_destroy: NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->quit = true;
    }
    s->cv_submit.notify_all();
    if (s->th.joinable()) s->th.join();
    // every job is done: tell the kernel to leave, and wait for it
    __atomic_store_n(&s->sc->stop, 1u, __ATOMIC_RELEASE);
    const int fatal = s->fatal;
    const std::string msg = s->fatal_msg;
    const int rc = server_free(s);
    if (fatal) return fail(fatal, "%s", msg.c_str());
    if (rc) return fail(rc, "vrt_server_destroy: stream synchronize failed");
    return VRT_OK;
}
