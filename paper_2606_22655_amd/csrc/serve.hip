// serve.hip -- continuous batching of trace jobs: a persistent kernel marches
// the rays of every admitted job of one medium kind at a time, while a host
// thread admits new jobs into a device pool of fixed size, hands them to the
// running kernel and copies finished jobs back.  Each medium kind has its own
// persistent kernel (the batch kernel's march of that kind, compiled for the
// occupancy its registers allow); when jobs of several kinds are admitted the
// kinds take turns, a run yielding after kSliceSec.
//
// The running kernel never waits for anything queued on a stream: a
// persistent kernel can hold the hardware queue (and the compute units) that
// such work would need.  Host and kernel talk through memory only:
//   hdesc[kSlots]  job descriptors in coherent pinned host memory, written by
//                  the host (slot = sequence % kSlots);
//   mb             host mailbox (coherent pinned): htail (jobs [0, htail) are
//                  staged: descriptor written, inputs in the pool), live
//                  (admitted jobs not yet retired), stop; and, written by the
//                  device, lost;
//   table, ctl     device copies of the descriptors and, per slot, a 64-bit
//                  claim word (sequence << 32 | next ray to hand out), the
//                  count of unretired rays and the sum of retired steps;
//   dc             device words: dtail (jobs [0, dtail) are active on the
//                  device), the activation lock, first_open, exiting;
//   done[kSlots]   done records in coherent pinned host memory: sequence + 1
//                  and the step total of the job last finished in the slot.
// Inputs and outputs move between the job's host arrays and the pool on the
// SDMA engines (HSA asynchronous copies), which need no compute unit and no
// kernel queue.  The host publishes a staged job by writing its descriptor
// and then htail.  A wave that finds htail ahead of dtail (polled at most
// every kPollTicks) takes the activation lock, copies the new descriptors
// into the device table, initialises their claim words and counts, and
// releases dtail.  Seeing a new dtail is an acquire at system scope, which
// invalidates the wave's L2 so that inputs the copy engine wrote are read
// fresh.
//
// A wave works on one group at a time -- the jobs with the same medium and
// trace parameters -- whose descriptor it copies to a slot of its own and then
// reads, with the medium's Gaussian bump table, as constants through the
// scalar cache (as the batch kernel reads its kernel arguments).
// Its idle lanes claim rays, in job order, from the group's jobs with one
// fetch-and-add per job on the claim word, whose sequence bits confirm that
// the slot still held the job; a lane's ray keeps its own job (inputs,
// outputs, accounting).  Retired rays are counted per lane and accounted in
// wave flushes (a release at system scope, so outputs reach memory, then one
// decrement of each job's count); the lane that brings a count to zero writes
// the done record with a system-scope release.  When its group has no rays
// left and its lanes are empty, the wave takes the group of the first job
// with rays left.
//
// Leaving is all or nothing: a wave that has polled kIdlePolls times without
// work while no job is live (or kLingerPolls times in any case) sets exiting;
// from then on waves claim no new rays, finish the ones they hold and leave,
// so the kernel ends promptly and the host's next launch (a captured hipGraph
// replay) has the whole device again.
#include <stdio.h>
#include <string.h>

#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "api_internal.h"
#include "lane32.h"
#include "pool.h"

namespace vrt {
namespace serve {

constexpr uint32_t kSlots = 4096;       // job table ring
constexpr size_t kDescBytes = 1024;     // one descriptor slot
constexpr uint32_t kIdlePolls = 40;     // empty polls (backing off to ~55 us apart) before leaving
constexpr uint32_t kLingerPolls = 20000;  // ~1 s of empty polls: leave even with jobs live
// iterations (~2 ms) between tail reads of a wave whose group ran dry: the
// words read are the same few lines for every wave, and polled every 64
// iterations they queue up enough to slow grid jobs, whose long rays keep
// dry waves busy, by a fifth
constexpr uint32_t kDryEvery = 1024;
constexpr uint64_t kPollTicks = 200;    // 2 us at the 100 MHz wall clock between host-tail polls
constexpr int kRanges = 4;              // job ranges one refill may draw from
constexpr uint32_t kScan = 64;          // jobs a refill looks ahead for its group
constexpr uint32_t kFlushEvery = 256;   // refill iterations between accounting flushes
constexpr int kMaxBlocksPerCu = 4;      // wave descriptor copies are sized for this
constexpr double kSliceSec = 0.025;     // a class's run yields after this when the other waits

// One persistent kernel per medium kind: each is the batch kernel's march of
// its kind wrapped in the job claiming and accounting, compiled for the
// occupancy its registers allow (analytic media at 3 blocks per CU, grids and
// the Zernike lens, whose marches with the entry inline need 190-215 VGPRs, at
// 2).  One kind's kernel is resident at a time; the kinds with admitted jobs
// take turns.
constexpr int kClasses = VRT_MEDIUM_ZERNIKE + 1;
__host__ __device__ constexpr int medium_class(int kind) { return kind; }
__host__ __device__ constexpr int class_occupancy(int kind) {
    return kind == VRT_MEDIUM_GRID || kind == VRT_MEDIUM_ZERNIKE ? 2 : 3;
}

struct alignas(16) JobDesc {
    MediumDev m;
    MedF mf;
    BoundaryDev b;
    TraceDev t;
    RaysDev<float> io;
    uint32_t n;
    int32_t kind;
    float dL0, eps_tan, mrg, crit;
    uint32_t group;  // jobs with the same medium and trace parameters share a group
    uint32_t pad[3];
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

// device words, one 64-byte line each
struct DevCtl {
    uint32_t dtail, pad0[15];
    uint32_t act, pad1[15];               // activation lock
    unsigned long long poll_t, pad2[7];   // wall clock of the last host-tail poll
    uint32_t first_open[kClasses][16];    // per class: jobs below it have no rays for it
    uint32_t exiting, pad4[15];           // the kernel is leaving: claim nothing more
};

// host mailbox (coherent pinned host memory), one 64-byte line each
struct Mailbox {
    uint32_t htail, pad0[15];  // host: jobs [0, htail) are staged
    uint32_t live[kClasses][16];  // host, per class: admitted jobs not yet retired
    uint32_t stop, pad2[15];   // host: leave
    uint32_t yield, pad4[15];  // host: the running class's kernel leaves (the other waits)
    uint32_t lost, pad3[15];   // device: a claim met a reused slot (fatal for the server)
};

struct DoneRec {
    unsigned long long steps;
    uint32_t seq1;  // sequence + 1 of the finished job
    uint32_t pad;
};

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The wave's group descriptor and bump table are read through the scalar
// data cache, as kernel arguments are: pointers in the constant address space
// whose value is wave-uniform.
using ConstF = const __attribute__((address_space(4))) float *;
using ConstDesc = const __attribute__((address_space(4))) JobDesc *;
template <class P>
__device__ __forceinline__ P rfl_cptr(P p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P)(((uint64_t)hi << 32) | lo);
}

// The server's arrays, passed as the kernel's one argument and read through
// a pointer to it: like the batch kernel's launch descriptor, its fields live
// in constant memory and are loaded where used, not held in scalar registers
// across the march.
struct SrvPtrs {
    const JobDesc *hdesc;
    JobDesc *table;
    JobCtl *ctl;
    DevCtl *dc;
    Mailbox *mb;
    DoneRec *done;
    JobDesc *wdg;  // each wave's copy of its group descriptor
};

// Pointers and wave-uniform progress of one wave.
struct WaveCtx {
    const SrvPtrs *__restrict__ P;
    unsigned long long *wacc;  // two LDS words of the wave
    int lane;
    uint32_t jcur;  // no job below it has rays for this wave
    uint32_t seen;  // jobs [0, seen) are known active (acquired)
    uint32_t it;
};

// Copy the descriptors of jobs staged by the host and not yet active into the
// device table, initialise their claim words and counts, and publish them.
// At most one wave at a time, at most once per kPollTicks.
__device__ __forceinline__ void maybe_activate(WaveCtx &c) {
    const unsigned long long now = wall_clock64();
    uint32_t go = 0;
    if (c.lane == 0) {
        const unsigned long long last =
            __hip_atomic_load(&c.P->dc->poll_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (now - last >= kPollTicks) {
            uint32_t z = 0;
            go = __hip_atomic_compare_exchange_strong(&c.P->dc->act, &z, 1u, __ATOMIC_ACQUIRE,
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     ? 1u
                     : 0u;
        }
    }
    if (!rfl(__shfl(go, 0))) return;
    if (c.lane == 0 &&
        __hip_atomic_load(&c.P->mb->yield, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
        __hip_atomic_store(&c.P->dc->exiting, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t ht =
        rfl(__hip_atomic_load(&c.P->mb->htail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
    const uint32_t dt =
        rfl(__hip_atomic_load(&c.P->dc->dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    for (uint32_t j = dt; j < ht; ++j) {
        const uint32_t sl = j % kSlots;
        const uint4 *src = (const uint4 *)(c.P->hdesc + sl);
        uint4 *dst = (uint4 *)(c.P->table + sl);
        for (uint32_t q = c.lane; q < sizeof(JobDesc) / 16; q += 64) dst[q] = src[q];
        if (c.lane == 0) {
            __hip_atomic_store(&c.P->ctl[sl].steps, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c.P->ctl[sl].left, c.P->hdesc[sl].n, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c.P->ctl[sl].claim, (unsigned long long)j << 32, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // descriptors and counts before dtail
    if (c.lane == 0) {
        if (ht > dt) __hip_atomic_store(&c.P->dc->dtail, ht, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&c.P->dc->poll_t, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&c.P->dc->act, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Take up jobs activated since the wave last looked.  Returns true if any.
__device__ __forceinline__ bool refresh_tail(WaveCtx &c) {
    const uint32_t dt =
        rfl(__hip_atomic_load(&c.P->dc->dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (dt <= c.seen) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // system scope: fresh descriptors and inputs
    c.seen = dt;
    return true;
}

__device__ __forceinline__ bool exiting(const WaveCtx &c) {
    return __hip_atomic_load(&c.P->dc->exiting, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Account the wave's retired rays: one release at system scope (the outputs
// of the retired rays reach memory, where the copy engine reads them), then
// per job one step-sum add and one decrement of its unretired count; the lane
// that brings a count to zero writes the job's done record.  Lanes' counts
// are summed per job in LDS.
__device__ __forceinline__ void flush_acc(WaveCtx &c, uint32_t aslot, uint32_t &acnt,
                                          unsigned long long &asteps) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    uint64_t pend = __ballot(acnt != 0);
    while (pend) {
        const int first = __ffsll((unsigned long long)pend) - 1;
        const uint32_t s0 = rfl(__shfl(aslot, first));
        const bool mine = acnt != 0 && aslot == s0;
        if (c.lane == first) {
            c.wacc[0] = 0;
            c.wacc[1] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (mine) {
            atomicAdd(&c.wacc[0], (unsigned long long)acnt);
            atomicAdd(&c.wacc[1], asteps);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (c.lane == first) {
            const uint32_t cnt = (uint32_t)c.wacc[0];
            JobCtl *jc = c.P->ctl + s0;
            __hip_atomic_fetch_add(&jc->steps, c.wacc[1], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t old =
                __hip_atomic_fetch_sub(&jc->left, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old == cnt) {  // the job's last rays
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const unsigned long long st =
                    __hip_atomic_load(&jc->steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t seq = (uint32_t)(
                    __hip_atomic_load(&jc->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32);
                __hip_atomic_store(&c.P->done[s0].steps, st, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&c.P->done[s0].seq1, seq + 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        if (mine) {
            acnt = 0;
            asteps = 0;
        }
        pend = __ballot(acnt != 0);
    }
}

// Job jj is of medium class cls and has rays to hand out (its slot still
// holds it).
__device__ __forceinline__ bool claimable(const WaveCtx &c, uint32_t jj, int cls) {
    const uint32_t sl = jj % kSlots;
    const unsigned long long w =
        __hip_atomic_load(&c.P->ctl[sl].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint32_t)(w >> 32) == jj && (uint32_t)w < c.P->table[sl].n &&
           medium_class(c.P->table[sl].kind) == cls;
}

// March rays of the wave's group (its descriptor copy and the medium's bump
// table read as constants) until
// the group has no rays left for it and its lanes are empty.  One function
// per medium kind, not inlined: each gets the registers of its own march
// (inlined side by side, the kinds' marches spill).
template <int MK>
__device__ __forceinline__ void march_group(WaveCtx &cw, ConstDesc Dp, uint32_t group_in) {
    WaveCtx c;  // wave-uniform copies in scalar registers
    c.P = cw.P;
    c.wacc = cw.wacc;
    c.lane = __lane_id();
    c.jcur = rfl(cw.jcur);
    c.seen = rfl(cw.seen);
    c.it = rfl(cw.it);
    const uint32_t group = rfl(group_in);
    const ConstDesc Du = rfl_cptr(Dp);
    const JobDesc &D = *(const JobDesc *)Du;
    const ConstF B = rfl_cptr((ConstF)D.m.bumps_f);
    const uint64_t below = (1ull << c.lane) - 1ull;
    Lane L;
    GridCache gc;
    grid_invalidate(gc);
    bool active = false;
    uint64_t act = 0;              // wave mask of lanes holding a ray
    uint32_t lslot = 0;            // job slot of the lane's ray
    uint32_t aslot = 0, acnt = 0;  // retired rays not yet accounted (all of job slot aslot)
    unsigned long long asteps = 0;
    bool dry = false;  // the group had fewer rays than idle lanes at the last claim
    uint32_t dry_it = 0;
    // The loop has the batch kernel's shape: an iteration in which every lane
    // holds a ray only steps; claims, accounting and activation polls happen
    // in iterations that find idle lanes (a ray ends every ~50 iterations of
    // a wave, so they stay frequent).
    for (;;) {
        const uint64_t nm = ~act;  // lanes without a ray
        if (nm) {
            bool fresh = false, claimed = false;
            ++c.it;
            // The tail and claim words are contended addresses: a wave whose
            // group ran dry looks for new jobs only every kDryEvery iterations.
            if (dry && ++dry_it % kDryEvery == 0) {
                maybe_activate(c);
                if (refresh_tail(c) && !exiting(c)) dry = false;
            }
            if (!dry) {
                const uint32_t want = (uint32_t)__popcll(nm);
                const int leader = __ffsll((unsigned long long)nm) - 1;
                // the wave marches a ray of job jcur: that job is not done, so its
                // slot still holds it, and it is of the wave's group
                const bool hold = __ballot(active && lslot == c.jcur % kSlots) != 0;
                uint32_t r0 = 0, b0 = 0, c0 = 0, r1 = 0, b1 = 0, c1 = 0, r2 = 0, b2 = 0, c2 = 0,
                         r3 = 0, b3 = 0, c3 = 0, nr = 0, jc = c.jcur, unmet = 0;
                if (c.lane == leader) {
                    // claim, in job order, from the jobs of the wave's group
                    uint32_t need = exiting(c) ? 0u : want;
                    unmet = need == 0;
                    const uint32_t lim = min(c.seen, c.jcur + kScan);
                    for (uint32_t jj = c.jcur; need && jj < lim && nr < (uint32_t)kRanges; ++jj) {
                        const uint32_t sl = jj % kSlots;
                        const uint32_t nj = c.P->table[sl].n;
                        const bool held = hold && jj == c.jcur;
                        bool gone = false;
                        if (!held) {
                            const unsigned long long w = __hip_atomic_load(
                                &c.P->ctl[sl].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            gone = (uint32_t)(w >> 32) != jj || (uint32_t)w >= nj;
                        }
                        if (!gone && (held || c.P->table[sl].group == group)) {
                            // one fetch-and-add (a compare-and-swap loop here stalls
                            // every wave on one contended word); an add past the end
                            // only takes what is left, and n < 2^31 keeps the
                            // overshoot out of the sequence bits.
                            const unsigned long long o = __hip_atomic_fetch_add(
                                &c.P->ctl[sl].claim, (unsigned long long)need, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
                            const uint32_t cn = (uint32_t)o;
                            if ((uint32_t)(o >> 32) != jj) {
                                // the slot was reused between the check and the add:
                                // the new job lost rays it can never get back --
                                // report it
                                __hip_atomic_store(&c.P->mb->lost, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM);
                                gone = true;
                            } else if (cn >= nj) {
                                gone = true;
                            } else {
                                const uint32_t take = min(need, nj - cn);
                                if (nr == 0) { r0 = sl; b0 = cn; c0 = take; }
                                else if (nr == 1) { r1 = sl; b1 = cn; c1 = take; }
                                else if (nr == 2) { r2 = sl; b2 = cn; c2 = take; }
                                else { r3 = sl; b3 = cn; c3 = take; }
                                ++nr;
                                need -= take;
                                gone = cn + take >= nj;
                            }
                        }
                        if (gone && jj == jc) {  // nothing for anyone below jc
                            jc = jj + 1;
                            atomicMax(&c.P->dc->first_open[medium_class(MK)][0], jc);
                        }
                    }
                    unmet |= need;
                }
                nr = rfl(__shfl(nr, leader));
                c.jcur = rfl(__shfl(jc, leader));
                claimed = nr != 0;
                if (nr < (uint32_t)kRanges && rfl(__shfl(unmet, leader)))
                    dry = true;  // fewer rays than idle lanes: the group has nothing more for now
                if (nr) {
                    // hand the ranges to the idle lanes in lane order
                    uint32_t k = (uint32_t)__popcll(nm & below);
                    const uint32_t rr[kRanges] = {rfl(__shfl(r0, leader)), rfl(__shfl(r1, leader)),
                                                  rfl(__shfl(r2, leader)), rfl(__shfl(r3, leader))};
                    const uint32_t bb[kRanges] = {rfl(__shfl(b0, leader)), rfl(__shfl(b1, leader)),
                                                  rfl(__shfl(b2, leader)), rfl(__shfl(b3, leader))};
                    const uint32_t cc[kRanges] = {rfl(__shfl(c0, leader)), rfl(__shfl(c1, leader)),
                                                  rfl(__shfl(c2, leader)), rfl(__shfl(c3, leader))};
                    if (!active) {
#pragma unroll
                        for (int q = 0; q < kRanges; ++q) {
                            if (!fresh && (uint32_t)q < nr) {
                                if (k < cc[q]) {
                                    L.r = bb[q] + k;
                                    lslot = rr[q];
                                    fresh = true;
                                } else {
                                    k -= cc[q];
                                }
                            }
                        }
                    }
                }
            }
            // a lane may only start a ray of another job once its count is
            // accounted
            const bool periodic = c.it % kFlushEvery == 0;
            if (__ballot(fresh && acnt && aslot != lslot) || (periodic && __ballot(acnt)))
                flush_acc(c, aslot, acnt, asteps);
            // busy waves also take their turn at activating staged jobs (and at
            // relaying the host's yield)
            if (periodic) maybe_activate(c);
            if (fresh) {
                aslot = lslot;
                grid_invalidate(gc);
                active = lane_init<MK>(D.m, D.m.rec, D.b, D.t, c.P->table[lslot].io, L, gc);
                if (!active) {
                    acnt++;
                    asteps += L.steps;
                }
            }
            act = __ballot(active);
            if (!act && (dry || !claimed)) {
                if (__ballot(acnt)) flush_acc(c, aslot, acnt, asteps);
                cw.jcur = c.jcur;
                cw.seen = c.seen;
                cw.it = c.it;
                return;
            }
        }
        if (active) {
            active = lane_step<MK>(D.m, D.mf, B, D.m.rec, D.b, D.t, c.P->table[lslot].io, L, gc,
                                   D.dL0, D.eps_tan, D.mrg, D.crit);
            if (!active) {
                acnt++;
                asteps += L.steps;
            }
        }
        act = __ballot(active);
    }
}

template <int kClass>
__global__ __launch_bounds__(256, class_occupancy(kClass)) void serve_kernel(SrvPtrs args) {
    __shared__ unsigned long long wacc_all[4][2];
    const SrvPtrs *__restrict__ P = &args;
    JobDesc *table = P->table;
    DevCtl *dc = P->dc;
    Mailbox *mb = P->mb;
    const int w = threadIdx.x >> 6;
    JobDesc *mine = P->wdg + (size_t)blockIdx.x * 4 + w;  // the wave's copy of its group descriptor
    WaveCtx c;
    c.P = P;
    c.wacc = wacc_all[w];
    c.lane = __lane_id();
    uint32_t *first_open = &dc->first_open[kClass][0];
    c.jcur = rfl(__hip_atomic_load(first_open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    c.seen = 0;
    c.it = 0;
    uint32_t idle = 0;
    for (;;) {
        // the wave is empty and accounted: find the first job with rays left
        maybe_activate(c);
        refresh_tail(c);
        if (exiting(c)) break;
        uint32_t fo =
            rfl(__hip_atomic_load(first_open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (fo > c.jcur) c.jcur = fo;
        while (c.jcur < c.seen && !claimable(c, c.jcur, kClass)) {
            if (c.jcur == fo) {
                fo = c.jcur + 1;
                if (c.lane == 0) atomicMax(first_open, fo);
            }
            ++c.jcur;
        }
        if (c.jcur < c.seen) {
            // adopt the job's group: copy its descriptor to the wave's own slot
            // (the job's table slot may be reused while the wave still marches
            // the group's other jobs), then drop stale scalar-cache lines of
            // that slot before march_group reads it as constants
            const uint32_t sl = c.jcur % kSlots;
            const uint4 *src = (const uint4 *)(table + sl);
            uint4 *dst = (uint4 *)mine;
            for (uint32_t q = c.lane; q < sizeof(JobDesc) / 16; q += 64) dst[q] = src[q];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_dcache_inv();
            const uint32_t group = rfl(table[sl].group);
            const ConstDesc Dc = (ConstDesc)mine;
            march_group<kClass>(c, Dc, group);
            idle = 0;
            continue;
        }
        // nothing to do: leave once idle long enough (all waves then leave)
        ++idle;
        if (idle > kIdlePolls && (idle % 8 == 0 || idle == kIdlePolls + 1)) {
            const bool stop =
                __hip_atomic_load(&mb->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
            const bool live = __hip_atomic_load(&mb->live[kClass][0], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_SYSTEM) != 0;
            if (stop || !live || idle > kLingerPolls) {
                if (c.lane == 0)
                    __hip_atomic_store(&dc->exiting, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        // back off: the tail is one address polled by every idle wave
        for (uint32_t q = 0; q < min(idle, 16u); ++q) __builtin_amdgcn_s_sleep(127);
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
    int cls = 0;  // medium class (which persistent kernel marches it)
    int error = 0;
    uint64_t steps = 0;
    double t_submit = 0, t_admit = 0, t_start = 0, t_retired = 0, t_done = 0;
    hsa_signal_t sig{0};  // completion of the job's input or output copies
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
    JobDesc *hdesc = nullptr;  // pinned, coherent
    Mailbox *mb = nullptr;     // pinned, coherent
    DoneRec *done = nullptr;   // pinned, coherent
    JobDesc *table = nullptr;  // device
    JobDesc *wdg = nullptr;    // device: each wave's copy of its group descriptor
    JobCtl *ctl = nullptr;     // device
    DevCtl *dc = nullptr;      // device
    std::vector<char> slot_busy;
    bool hsa_up = false;
    hsa_agent_t gpu{0}, cpu{0};
    std::vector<hsa_signal_t> free_sigs;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph[kClasses] = {};
    hipGraphExec_t exec[kClasses] = {};
    bool running = false;
    int run_cls = 0;         // class of the running (or last) kernel
    double run_t0 = 0;       // when it was launched
    bool yield_sent = false;
    uint32_t blocks[kClasses] = {};
    uint32_t futile = 0;  // kernel runs since a job last retired
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::deque<HostJob *> queued, staging;
    std::vector<HostJob *> live, copying;
    std::unordered_map<uint64_t, HostJob *> jobs;
    std::map<std::vector<uint64_t>, uint32_t> groups;  // (medium, trace parameters) -> group id
    uint32_t next_seq = 0;
    uint32_t admitted = 0;  // admitted and not retired
    uint32_t admitted_cls[kClasses] = {};  // the same per class (the mailbox's live)
    uint32_t published = 0; // jobs [0, published) staged and announced
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

static void set_fatal(vrt_server_t s, int code, const std::string &msg) {
    if (!s->fatal) {
        s->fatal = code;
        s->fatal_msg = msg;
    }
}

static bool get_signal(vrt_server_t s, hsa_signal_value_t v, hsa_signal_t *out) {
    if (!s->free_sigs.empty()) {
        *out = s->free_sigs.back();
        s->free_sigs.pop_back();
        hsa_signal_store_screlease(*out, v);
        return true;
    }
    return hsa_signal_create(v, 0, nullptr, out) == HSA_STATUS_SUCCESS;
}

static void put_signal(vrt_server_t s, hsa_signal_t &sg) {
    if (sg.handle) s->free_sigs.push_back(sg);
    sg.handle = 0;
}

// Copy engine transfer of `bytes` (the copy decrements `sig` when done).
static bool dma(vrt_server_t s, void *dst, bool dst_dev, const void *src, size_t bytes,
                hsa_signal_t sig) {
    return hsa_amd_memory_async_copy(dst, dst_dev ? s->gpu : s->cpu, src,
                                     dst_dev ? s->cpu : s->gpu, bytes, 0, nullptr,
                                     sig) == HSA_STATUS_SUCCESS;
}

// Device arrays of a job in the pool: 12 float arrays, then 5 uint32 arrays.
static void job_arrays(vrt_server_t s, const HostJob *J, float **f, uint32_t **u) {
    char *base = s->pool + J->off;
    *f = (float *)base;
    *u = (uint32_t *)(base + 12 * J->n * sizeof(float));
}

// Issue a job's input copies (scheduler thread, mu held).
static bool stage_job(vrt_server_t s, HostJob *J) {
    float *f;
    uint32_t *u;
    job_arrays(s, J, &f, &u);
    const void *in[6] = {J->host.px, J->host.py, J->host.pz, J->host.dx, J->host.dy, J->host.dz};
    if (!get_signal(s, 6, &J->sig)) return false;
    for (int a = 0; a < 6; ++a)
        if (!dma(s, f + a * J->n, true, in[a], J->n * sizeof(float), J->sig)) return false;
    return true;
}

// Write the descriptor of a staged job and announce it to the kernel.
static void publish_job(vrt_server_t s, HostJob *J) {
    const size_t n = J->n;
    float *f;
    uint32_t *u;
    job_arrays(s, J, &f, &u);
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
    {
        std::vector<uint64_t> key(8);
        key[0] = (uint64_t)(uintptr_t)m;
        const double pv[6] = {J->p.dL0, (double)J->p.max_steps, J->p.eps_tan, J->p.crit_rad,
                              J->p.tie_eps, J->p.exit_plane_z};
        for (int i = 0; i < 6; ++i) memcpy(&key[1 + i], &pv[i], 8);
        auto it = s->groups.find(key);
        if (it == s->groups.end()) it = s->groups.emplace(key, (uint32_t)s->groups.size()).first;
        d.group = it->second;
    }
    d.dL0 = (float)J->p.dL0;
    d.eps_tan = (float)J->p.eps_tan;
    d.mrg = fmaxf(2e-6f, 4.0f * (float)J->p.tie_eps);
    d.crit = (float)J->p.crit_rad;
    memcpy((void *)(s->hdesc + J->seq % kSlots), &d, sizeof d);
    s->published = J->seq + 1;
    __atomic_store_n(&s->mb->htail, s->published, __ATOMIC_RELEASE);
}

// Issue a retired job's output copies.
static bool fetch_job(vrt_server_t s, HostJob *J) {
    float *f;
    uint32_t *u;
    job_arrays(s, J, &f, &u);
    void *outf[6] = {J->host.ox, J->host.oy, J->host.oz, J->host.odx, J->host.ody, J->host.odz};
    void *outu[5] = {J->host.status, J->host.steps, J->host.n_tir, J->host.n_btir,
                     J->host.flags};
    if (!get_signal(s, 11, &J->sig)) return false;
    for (int a = 0; a < 6; ++a)
        if (!dma(s, outf[a], false, f + (6 + a) * J->n, J->n * sizeof(float), J->sig)) return false;
    for (int a = 0; a < 5; ++a)
        if (!dma(s, outu[a], false, u + a * J->n, J->n * sizeof(uint32_t), J->sig)) return false;
    return true;
}

static void finish_job(vrt_server_t s, HostJob *J, int err) {
    J->state = VRT_JOB_DONE;
    J->error = err;
    J->t_done = s->now();
    s->alloc.release(J->off, J->bytes);
    s->slot_busy[J->seq % kSlots] = 0;
    J->med->jobs--;
    s->st.jobs_done++;
    s->st.rays_done += J->n;
    s->st.ray_steps_done += J->steps;
    s->st.pool_bytes = s->alloc.used();
}

// Medium kind of the oldest published job that has not retired (-1: none).
static int oldest_kind(vrt_server_t s) {
    const HostJob *o = nullptr;
    for (const HostJob *J : s->live)
        if (!o || J->seq < o->seq) o = J;
    return o ? o->cls : -1;
}

static void set_live(vrt_server_t s) {
    for (int k = 0; k < kClasses; ++k)
        __atomic_store_n(&s->mb->live[k][0], s->admitted_cls[k], __ATOMIC_RELEASE);
}

// One pass of the scheduler (mu held).  Returns true if anything moved.
static bool schedule_once(vrt_server_t s) {
    bool moved = false;
    hipError_t e = hipSuccess;
    // 1. admission in submission order: pool space and the job's slot free;
    //    the input copies start at once
    while (!s->queued.empty()) {
        HostJob *J = s->queued.front();
        if (s->slot_busy[J->seq % kSlots]) break;
        if (!s->alloc.alloc(J->bytes, &J->off)) break;
        s->queued.pop_front();
        s->slot_busy[J->seq % kSlots] = 1;
        s->st.pool_bytes = s->alloc.used();
        s->st.pool_peak_bytes = s->alloc.peak();
        J->t_admit = s->now();
        J->state = VRT_JOB_RUNNING;
        s->admitted++;
        s->admitted_cls[J->cls]++;
        set_live(s);
        if (!stage_job(s, J)) {
            set_fatal(s, VRT_EHIP, "server: input copy could not be issued");
            return false;
        }
        s->staging.push_back(J);
        moved = true;
    }
    // 2. staged jobs are announced in order, once their inputs are in the pool
    while (!s->staging.empty()) {
        HostJob *J = s->staging.front();
        const hsa_signal_value_t v = hsa_signal_load_scacquire(J->sig);
        if (v < 0) {
            set_fatal(s, VRT_EHIP, "server: input copy failed");
            return false;
        }
        if (v > 0) break;
        put_signal(s, J->sig);
        publish_job(s, J);
        J->t_start = s->now();
        s->staging.pop_front();
        s->live.push_back(J);
        moved = true;
    }
    // 3. one persistent kernel at a time, of one medium kind, runs while jobs
    //    of its kind are admitted.  Jobs are served oldest first, as the waves
    //    of one kernel take them: the kernel run is of the oldest admitted
    //    job's kind, and a run yields (its waves claim no more rays, finish the
    //    ones they hold and leave) once it has run kSliceSec while the oldest
    //    admitted job is of another kind.
    if (s->running) {
        e = hipEventQuery(s->ev);
        if (e == hipSuccess) {
            s->running = false;
        } else if (e != hipErrorNotReady) {
            goto fail;
        } else if (!s->yield_sent && s->now() - s->run_t0 > kSliceSec &&
                   oldest_kind(s) != s->run_cls) {
            __atomic_store_n(&s->mb->yield, 1u, __ATOMIC_RELEASE);
            s->yield_sent = true;
        }
    }
    if (!s->running && !s->live.empty()) {
        // a run that retires nothing while jobs are live can only repeat: stop
        if (++s->futile > 64) {
            set_fatal(s, VRT_EHIP, "server: published jobs make no progress");
            return false;
        }
        const int cls = oldest_kind(s);
        // the previous run has ended: clear its exit flag (no wave reads it now)
        __atomic_store_n(&s->mb->yield, 0u, __ATOMIC_RELEASE);
        if ((e = hipMemsetAsync(&s->dc->exiting, 0, sizeof(uint32_t), s->stream)) != hipSuccess)
            goto fail;
        if ((e = hipGraphLaunch(s->exec[cls], s->stream)) != hipSuccess) goto fail;
        if ((e = hipEventRecord(s->ev, s->stream)) != hipSuccess) goto fail;
        s->running = true;
        s->run_cls = cls;
        s->run_t0 = s->now();
        s->yield_sent = false;
        s->st.kernel_launches++;
        s->st.lanes = s->blocks[cls] * 256;
        moved = true;
    }
    if (__atomic_load_n(&s->mb->lost, __ATOMIC_ACQUIRE)) {
        set_fatal(s, VRT_EHIP, "server: a ray claim met a reused job slot; rays were lost");
        return false;
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
            s->admitted--;
            s->admitted_cls[J->cls]--;
            set_live(s);
            if (!fetch_job(s, J)) {
                set_fatal(s, VRT_EHIP, "server: output copy could not be issued");
                return false;
            }
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
        const hsa_signal_value_t v = hsa_signal_load_scacquire(J->sig);
        if (v < 0) {
            set_fatal(s, VRT_EHIP, "server: output copy failed");
            return false;
        }
        if (v > 0) {
            ++i;
            continue;
        }
        put_signal(s, J->sig);
        finish_job(s, J, 0);
        s->copying[i] = s->copying.back();
        s->copying.pop_back();
        moved = true;
    }
    if (moved) s->cv_done.notify_all();
    return moved;
fail:
    set_fatal(s, e == hipErrorOutOfMemory ? VRT_ENOMEM : VRT_EHIP,
              std::string("server: ") + hipGetErrorString(e));
    return false;
}

static void fail_job(vrt_server_t s, HostJob *J) {
    J->state = VRT_JOB_DONE;
    J->error = s->fatal;
    J->med->jobs--;
}

// After a fatal error: every job not done fails.  Jobs whose copies may still
// be in flight keep their pool space (the pool is not reused after this).
static void fail_all(vrt_server_t s) {
    for (auto *v : {&s->queued, &s->staging}) {
        for (HostJob *J : *v) fail_job(s, J);
        v->clear();
    }
    for (auto *v : {&s->live, &s->copying}) {
        for (HostJob *J : *v) fail_job(s, J);
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
        const bool busy = !s->queued.empty() || !s->staging.empty() || !s->live.empty() ||
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

// Wait (bounded) for copies a failed server may still have in flight.
static void drain_signals(vrt_server_t s) {
    for (auto &kv : s->jobs) {
        HostJob *J = kv.second;
        if (J->sig.handle) {
            (void)hsa_signal_wait_scacquire(J->sig, HSA_SIGNAL_CONDITION_LT, 1, 10000000000ull,
                                            HSA_WAIT_STATE_BLOCKED);
            (void)hsa_signal_destroy(J->sig);
            J->sig.handle = 0;
        }
    }
}

static int server_free(vrt_server_t s) {
    int rc = VRT_OK;
    if (s->mb) __atomic_store_n(&s->mb->stop, 1u, __ATOMIC_RELEASE);
    if (s->stream && hipStreamSynchronize(s->stream) != hipSuccess) rc = VRT_EHIP;
    if (s->hsa_up) drain_signals(s);
    for (auto &sg : s->free_sigs) (void)hsa_signal_destroy(sg);
    s->free_sigs.clear();
    for (int k = 0; k < kClasses; ++k) {
        if (s->exec[k]) (void)hipGraphExecDestroy(s->exec[k]);
        if (s->graph[k]) (void)hipGraphDestroy(s->graph[k]);
    }
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    for (auto &kv : s->jobs) delete kv.second;
    if (s->pool) (void)hipFree(s->pool);
    if (s->table) (void)hipFree(s->table);
    if (s->wdg) (void)hipFree(s->wdg);
    if (s->ctl) (void)hipFree(s->ctl);
    if (s->dc) (void)hipFree(s->dc);
    if (s->hdesc) (void)hipHostFree(s->hdesc);
    if (s->mb) (void)hipHostFree(s->mb);
    if (s->done) (void)hipHostFree(s->done);
    if (s->hsa_up) (void)hsa_shut_down();
    if (s->ctx) s->ctx->n_servers--;
    delete s;
    return rc;
}

// The HSA agent owning an allocation (GPU for device memory, CPU for pinned
// host memory), and whether [p, p + bytes) lies inside that allocation.
static bool owner_of(const void *p, size_t bytes, hsa_agent_t *agent) {
    hsa_amd_pointer_info_t info;
    memset(&info, 0, sizeof info);
    info.size = sizeof info;
    if (hsa_amd_pointer_info(p, &info, nullptr, nullptr, nullptr) != HSA_STATUS_SUCCESS)
        return false;
    if (info.type == HSA_EXT_POINTER_TYPE_UNKNOWN) return false;
    const char *base = (const char *)info.hostBaseAddress;
    if (!base) base = (const char *)info.agentBaseAddress;
    if (!base || (const char *)p < base || (const char *)p + bytes > base + info.sizeInBytes)
        return false;
    *agent = info.agentOwner;
    return true;
}

static bool is_cpu(hsa_agent_t a) {
    hsa_device_type_t t;
    return hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) == HSA_STATUS_SUCCESS &&
           t == HSA_DEVICE_TYPE_CPU;
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
    s->slot_busy.assign(kSlots, 0);
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e;
#define SV_TRY(call, what)                            \
    if ((e = (call)) != hipSuccess) {                 \
        rc = fail_hip(e, "vrt_server_create: " what); \
        server_free(s);                               \
        return rc;                                    \
    }
#define SV_FAIL(what)                                            \
    do {                                                         \
        rc = fail(VRT_EHIP, "vrt_server_create: %s", what);      \
        server_free(s);                                          \
        return rc;                                               \
    } while (0)
    SV_TRY(hipMalloc((void **)&s->pool, s->budget), "pool");
    SV_TRY(hipMalloc((void **)&s->table, sizeof(JobDesc) * kSlots), "job table");
    SV_TRY(hipMalloc((void **)&s->wdg, sizeof(JobDesc) * 4 * (size_t)ctx->num_cu * kMaxBlocksPerCu),
           "wave descriptors");
    SV_TRY(hipMalloc((void **)&s->ctl, sizeof(JobCtl) * kSlots), "job counters");
    SV_TRY(hipMalloc((void **)&s->dc, sizeof(DevCtl)), "control words");
    SV_TRY(hipHostMalloc((void **)&s->hdesc, sizeof(JobDesc) * kSlots, hipHostMallocCoherent),
           "descriptors");
    SV_TRY(hipHostMalloc((void **)&s->mb, sizeof(Mailbox), hipHostMallocCoherent), "mailbox");
    SV_TRY(hipHostMalloc((void **)&s->done, sizeof(DoneRec) * kSlots, hipHostMallocCoherent),
           "done records");
    memset((void *)s->hdesc, 0, sizeof(JobDesc) * kSlots);
    memset((void *)s->mb, 0, sizeof(Mailbox));
    memset((void *)s->done, 0, sizeof(DoneRec) * kSlots);
    if (hsa_init() != HSA_STATUS_SUCCESS) SV_FAIL("hsa_init");
    s->hsa_up = true;
    if (!owner_of(s->pool, s->budget, &s->gpu) || is_cpu(s->gpu)) SV_FAIL("pool agent");
    if (!owner_of(s->mb, sizeof(Mailbox), &s->cpu) || !is_cpu(s->cpu)) SV_FAIL("host agent");
    SV_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "stream");
    SV_TRY(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming), "event");
    // claim words of empty slots name no job (sequence 0xffffffff)
    {
        std::vector<JobCtl> c0(kSlots);
        for (auto &c : c0) c.claim = 0xffffffffull << 32;
        SV_TRY(hipMemcpy(s->ctl, c0.data(), sizeof(JobCtl) * kSlots, hipMemcpyHostToDevice),
               "counter init");
        SV_TRY(hipMemset(s->table, 0, sizeof(JobDesc) * kSlots), "table init");
        SV_TRY(hipMemset(s->dc, 0, sizeof(DevCtl)), "control init");
    }
    const void *fns[kClasses] = {
        (const void *)serve_kernel<0>, (const void *)serve_kernel<1>, (const void *)serve_kernel<2>,
        (const void *)serve_kernel<3>, (const void *)serve_kernel<4>, (const void *)serve_kernel<5>,
        (const void *)serve_kernel<6>, (const void *)serve_kernel<7>, (const void *)serve_kernel<8>};
    for (int k = 0; k < kClasses; ++k) {
        const void *fn = fns[k];
        int occ = 0;
        SV_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 256, 0), "occupancy");
        occ = std::min(std::max(occ, 1), kMaxBlocksPerCu);
        s->blocks[k] = (uint32_t)ctx->num_cu * (uint32_t)occ;
        if (max_lanes > 0)
            s->blocks[k] = std::min(s->blocks[k], std::max(1u, (uint32_t)max_lanes / 256u));
        SV_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal), "capture");
        SrvPtrs ptrs{s->hdesc, s->table, s->ctl, s->dc, s->mb, s->done, s->wdg};
        void *args[] = {&ptrs};
        SV_TRY(hipLaunchKernel(fn, dim3(s->blocks[k]), dim3(256), args, 0, s->stream), "launch");
        SV_TRY(hipStreamEndCapture(s->stream, &s->graph[k]), "capture");
        SV_TRY(hipGraphInstantiate(&s->exec[k], s->graph[k], nullptr, nullptr, 0), "graph");
    }
    s->st.job_slots = kSlots;
#undef SV_TRY
#undef SV_FAIL
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
    for (const void *q : ptrs) {
        if (!q || ((uintptr_t)q & 3))
            return fail(VRT_EINVAL, "vrt_server_submit: NULL or misaligned array");
        hsa_agent_t a;
        if (!owner_of(q, n_rays * 4, &a) || !is_cpu(a))
            return fail(VRT_EINVAL,
                        "vrt_server_submit: every array must lie in pinned host memory "
                        "(hipHostMalloc)");
    }
    const size_t bytes = ((n_rays * kRayBytes + 255) & ~(size_t)255) + 256;
    if (bytes > s->budget)
        return fail(VRT_EINVAL, "vrt_server_submit: %zu rays need %zu bytes, the pool has %zu",
                    n_rays, bytes, s->budget);
    HostJob *J = new HostJob();
    J->med = m;
    J->cls = medium_class(m->dev.kind);
    J->p = *p;
    J->host = *host_rays;
    J->n = n_rays;
    J->bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->fatal) {
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
    // every job is done (or failed): server_free tells the kernel to leave and waits
    const int fatal = s->fatal;
    const std::string msg = s->fatal_msg;
    const int rc = server_free(s);
    if (fatal) return fail(fatal, "%s", msg.c_str());
    if (rc) return fail(rc, "vrt_server_destroy: stream synchronize failed");
    return VRT_OK;
}
