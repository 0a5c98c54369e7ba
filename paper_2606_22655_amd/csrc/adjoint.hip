// adjoint.hip -- exit-plane loss of a grid medium and its gradient with
// respect to the node values (the paper's direct-design use of the march,
// Sec. VI, made differentiable): one lane per ray, FP64.
//
// Forward: each lane marches its ray as a sequence of operations
// (adjoint64.h) and saves its state every K operations (checkpoints, SoA in
// HBM).  Backward: for each checkpoint interval, last first, the lane replays
// the interval's operations from the checkpoint -- bit for bit the forward
// ones -- saving the state before each into a per-lane tape, then walks the
// tape backwards applying each operation's vector-Jacobian product.  Grid
// evaluations sum their contributions to the node values and node central
// differences of the current cell in per-lane LDS accumulators, which are
// added to the node arrays in HBM (atomically) when the ray changes cell; a
// last kernel folds the central differences back onto the node values.
#pragma clang fp contract(off)
#include <string.h>

#include <vector>

#include "adjoint64.h"
#include "api_internal.h"

namespace vrt {
namespace adj {

constexpr int kF = 12;  // doubles per saved state
constexpr size_t kScratchBudget = 8ull << 30;  // checkpoints + tapes of one launch pair

struct AdjIn {
    const double *px, *py, *pz, *dx, *dy, *dz, *tx, *ty;
};

// state j of lane `lane` in a buffer of `lanes` lanes: field f at ((j kF + f) lanes + lane)
__device__ __forceinline__ void put_state(double *buf, uint32_t j, uint32_t lane, uint32_t lanes,
                                          const St &s) {
    double *q = buf + (size_t)j * kF * lanes + lane;
    const double v[kF] = {s.P.x, s.P.y, s.P.z, s.I.x, s.I.y, s.I.z, s.R.x, s.R.y, s.R.z,
                          s.n_last, s.Delta,
                          __longlong_as_double((long long)(((uint64_t)(uint32_t)s.phase << 32) |
                                                           s.steps))};
#pragma unroll
    for (int f = 0; f < kF; ++f) q[(size_t)f * lanes] = v[f];
}

__device__ __forceinline__ St get_state(const double *buf, uint32_t j, uint32_t lane,
                                        uint32_t lanes) {
    const double *q = buf + (size_t)j * kF * lanes + lane;
    St s;
    s.P = mk(q[0], q[(size_t)lanes], q[2 * (size_t)lanes]);
    s.I = mk(q[3 * (size_t)lanes], q[4 * (size_t)lanes], q[5 * (size_t)lanes]);
    s.R = mk(q[6 * (size_t)lanes], q[7 * (size_t)lanes], q[8 * (size_t)lanes]);
    s.n_last = q[9 * (size_t)lanes];
    s.Delta = q[10 * (size_t)lanes];
    const uint64_t w = (uint64_t)__double_as_longlong(q[11 * (size_t)lanes]);
    s.steps = (uint32_t)w;
    s.phase = (int32_t)(w >> 32);
    return s;
}

// Forward march of rays [r0, r0 + n): exit-plane point and loss per ray;
// checkpoints every kops operations when ck is not null.
__global__ __launch_bounds__(256) void adj_forward_kernel(MediumDev m, BoundaryDev b, TraceDev t,
                                                          AdjIn in, uint32_t r0, uint32_t n,
                                                          uint32_t kops, uint32_t n_ck, double *ck,
                                                          uint32_t *nops, double *xy, int32_t *endv,
                                                          double *loss_ray, int32_t *end_out) {
    const uint32_t lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= n) return;
    const uint32_t r = r0 + lane;
    St s;
    int end;
    fwd_entry(m, b, t, mk(in.px[r], in.py[r], in.pz[r]), mk(in.dx[r], in.dy[r], in.dz[r]), s, end);
    uint32_t o = 0;
    double x = 0.0, y = 0.0;
    // Ops alternate decide, move (a boundary TIR adds a move).  One iteration
    // runs one op and then the move that follows a decide, so lanes of a wave
    // that fell out of step after a boundary TIR are back in step at the next
    // iteration instead of running decides and moves on alternate passes.
    while (s.phase != PH_DONE) {
        if (ck && o % kops == 0) {
            if (o / kops >= n_ck) {  // cannot happen within max_steps; never write past the buffer
                end = END_OTHER;
                break;
            }
            put_state(ck, o / kops, lane, n, s);
        }
        const bool decided = s.phase == PH_DECIDE;
        fwd_op(m, b, t, s, x, y, end);
        ++o;
        if (decided && s.phase == PH_MOVE) {
            if (ck && o % kops == 0) {
                if (o / kops >= n_ck) {
                    end = END_OTHER;
                    break;
                }
                put_state(ck, o / kops, lane, n, s);
            }
            fwd_op(m, b, t, s, x, y, end);
            ++o;
        }
    }
    if (end != END_PLANE) end = END_OTHER;
    double l = 0.0;
    if (end == END_PLANE) {
        const double ex = x - in.tx[r], ey = y - in.ty[r];
        l = ex * ex + ey * ey;
    }
    if (loss_ray) loss_ray[r] = l;
    if (end_out) end_out[r] = end;
    if (nops) {
        nops[lane] = o;
        endv[lane] = end;
        xy[2 * lane] = x;
        xy[2 * lane + 1] = y;
    }
}

// Reverse sweep of rays [r0, r0 + n) that reached the exit plane.
__global__ __launch_bounds__(256, 2) void adj_backward_kernel(MediumDev m, BoundaryDev b, TraceDev t,
                                                           AdjIn in, uint32_t r0, uint32_t n,
                                                           uint32_t kops, const double *ck,
                                                           const uint32_t *nops, const double *xy,
                                                           const int32_t *endv, double *tape,
                                                           double scale, GradOut go) {
    const uint32_t lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= n || endv[lane] != END_PLANE) return;
    const uint32_t r = r0 + lane;
    const double xbar = 2.0 * scale * (xy[2 * lane] - in.tx[r]);
    const double ybar = 2.0 * scale * (xy[2 * lane + 1] - in.ty[r]);
    const uint32_t total = nops[lane];
    // per-lane cell accumulators in LDS: slot q of thread x at [q][x]
    __shared__ double acc_lds[32 * 256];
    GradAcc acc = make_acc(acc_lds + threadIdx.x, blockDim.x, m, go);
    Adj a = zero_adj();
    for (int seg = (int)((total - 1) / kops); seg >= 0; --seg) {
        St s = get_state(ck, (uint32_t)seg, lane, n);
        const uint32_t o0 = (uint32_t)seg * kops;
        const uint32_t o1 = min(total, o0 + kops);
        double x, y;
        int end;
        for (uint32_t o = o0; o < o1;) {  // the forward kernel's op pairing
            const bool decided = s.phase == PH_DECIDE;
            put_state(tape, o - o0, lane, n, s);
            fwd_op(m, b, t, s, x, y, end);
            ++o;
            if (decided && o < o1 && s.phase == PH_MOVE) {
                put_state(tape, o - o0, lane, n, s);
                fwd_op(m, b, t, s, x, y, end);
                ++o;
            }
        }
        for (uint32_t o = o1; o > o0;) {  // reversed, the same (decide, move) pairs
            --o;
            const St si = get_state(tape, o - o0, lane, n);
            const bool moved = si.phase == PH_MOVE;
            vjp_op(m, b, t, si, a, xbar, ybar, acc);
            if (moved && o > o0) {
                const St sp = get_state(tape, o - 1 - o0, lane, n);
                if (sp.phase == PH_DECIDE) {
                    --o;
                    vjp_op(m, b, t, sp, a, xbar, ybar, acc);
                }
            }
        }
    }
    vjp_entry(m, b, t, mk(in.px[r], in.py[r], in.pz[r]), mk(in.dx[r], in.dy[r], in.dz[r]), a, acc);
    acc.flush();
}

__global__ void fill_kernel(double *p, size_t n, double v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fold_cdiff_kernel(MediumDev m, const double *gH, double *grad, size_t nodes) {
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < nodes;
         p += (size_t)gridDim.x * blockDim.x)
        cdiff_transpose(m, p, gH, grad, nodes);
}

}  // namespace adj
}  // namespace vrt

using namespace vrt;
using namespace vrt::adj;

extern "C" int vrt_grid_loss_grad(vrt_medium_t grid, const vrt_trace_params *p,
                                  const vrt_adjoint_rays *rays, size_t n_rays, double scale,
                                  int checkpoint_every, double *loss, double *grad, void *stream) {
    if (!grid || !p || !rays || !loss) return fail(VRT_EINVAL, "vrt_grid_loss_grad: NULL argument");
    if (grid->dev.kind != VRT_MEDIUM_GRID || grid->bnd.kind != VRT_BOUNDARY_BOX)
        return fail(VRT_EINVAL, "vrt_grid_loss_grad: needs a grid medium in a box");
    if (p->precision != VRT_FP64 || p->max_lanes != 0 || isnan(p->exit_plane_z))
        return fail(VRT_EINVAL, "vrt_grid_loss_grad: VRT_FP64, max_lanes 0 and an exit plane");
    if (!(p->dL0 > 0.0) || !isfinite(p->dL0) || p->max_steps <= 0 || p->max_steps > 1000000 ||
        p->eps_tan != 0.0 || !(p->crit_rad >= 0.0) || !(p->tie_eps >= 0.0) || !(p->tie_eps <= 1e-6))
        return fail(VRT_EINVAL,
                    "vrt_grid_loss_grad: dL0 > 0, max_steps in [1, 1e6], eps_tan = 0, tie_eps <= 1e-6");
    if (checkpoint_every < 1 || checkpoint_every > 4096)
        return fail(VRT_EINVAL, "vrt_grid_loss_grad: checkpoint_every must be in [1, 4096]");
    if (n_rays >= (1ull << 31) || !isfinite(scale))
        return fail(VRT_EINVAL, "vrt_grid_loss_grad: n_rays < 2^31 and a finite scale");
    const void *ptrs[] = {rays->px, rays->py, rays->pz, rays->dx, rays->dy, rays->dz, rays->tx,
                          rays->ty};
    for (const void *q : ptrs)
        if (!q || ((uintptr_t)q & 7))
            return fail(VRT_EINVAL, "vrt_grid_loss_grad: ray array NULL or misaligned");
    for (const void *q : ptrs)
        if (!gpu_accessible(q))
            return fail(VRT_EINVAL, "vrt_grid_loss_grad: a ray array is pageable host memory");
    if ((grad && !gpu_accessible(grad)) || (rays->end && !gpu_accessible(rays->end)) ||
        (rays->loss_ray && !gpu_accessible(rays->loss_ray)))
        return fail(VRT_EINVAL,
                    "vrt_grid_loss_grad: grad, end or loss_ray is pageable host memory");
    int rc = set_device(grid->ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const MediumDev &m = grid->dev;
    TraceDev t{};
    t.dL0 = p->dL0;
    t.max_steps = p->max_steps;
    t.eps_tan = 0.0;
    t.crit_rad = p->crit_rad;
    t.tie_eps = p->tie_eps;
    t.has_plane = 1;
    t.plane_z = p->exit_plane_z;
    const AdjIn in{rays->px, rays->py, rays->pz, rays->dx, rays->dy, rays->dz, rays->tx, rays->ty};
    const size_t nodes = (size_t)m.nx * m.ny * m.nz;
    const uint32_t kops = 2u * (uint32_t)checkpoint_every;  // a step is a decision and a move
    const uint32_t n_ck = (uint32_t)((2 * p->max_steps + 1) / kops + 2);
    // rays per forward/backward launch pair: all of them for the loss alone;
    // with the gradient, as many as the scratch budget holds (at least 4,096)
    const size_t per_lane = sizeof(double) * kF * ((size_t)n_ck + kops) + 32;
    size_t cap = grad ? kScratchBudget / per_lane : n_rays;
    cap = cap < 4096 ? 4096 : cap;
    const uint32_t lanes = (uint32_t)(n_rays < cap ? n_rays : cap);
    double *loss_ray = rays->loss_ray, *own_loss = nullptr, *ck = nullptr, *tape = nullptr,
           *xy = nullptr, *gH = nullptr;
    uint32_t *nops = nullptr;
    int32_t *endv = nullptr;
    hipError_t e = hipSuccess;
    if (!loss_ray && n_rays) e = hipMalloc((void **)&own_loss, sizeof(double) * n_rays);
    if (!loss_ray) loss_ray = own_loss;
    if (grad && n_rays && e == hipSuccess) {
        e = hipMalloc((void **)&ck, sizeof(double) * kF * (size_t)n_ck * lanes);
        if (e == hipSuccess) e = hipMalloc((void **)&tape, sizeof(double) * kF * (size_t)kops * lanes);
        if (e == hipSuccess) e = hipMalloc((void **)&xy, sizeof(double) * 2 * (size_t)lanes);
        if (e == hipSuccess) e = hipMalloc((void **)&nops, sizeof(uint32_t) * lanes);
        if (e == hipSuccess) e = hipMalloc((void **)&endv, sizeof(int32_t) * lanes);
    }
    if (grad && e == hipSuccess) e = hipMalloc((void **)&gH, sizeof(double) * 3 * nodes);
    if (grad && e == hipSuccess) {
        hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, st, grad, nodes, 0.0);
        hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, st, gH, 3 * nodes, 0.0);
        e = hipGetLastError();
    }
    const GradOut go{grad, gH, nodes};
    for (size_t r0 = 0; r0 < n_rays && e == hipSuccess; r0 += lanes) {
        const uint32_t n = (uint32_t)((n_rays - r0) < lanes ? (n_rays - r0) : lanes);
        const uint32_t blocks = (n + 255) / 256;
        hipLaunchKernelGGL(adj_forward_kernel, dim3(blocks), dim3(256), 0, st, m, grid->bnd, t, in,
                           (uint32_t)r0, n, kops, n_ck, ck, nops, xy, endv, loss_ray, rays->end);
        if (grad)
            hipLaunchKernelGGL(adj_backward_kernel, dim3(blocks), dim3(256), 0, st, m, grid->bnd, t,
                               in, (uint32_t)r0, n, kops, ck, nops, xy, endv, tape, scale, go);
        e = hipGetLastError();
    }
    if (grad && e == hipSuccess) {
        hipLaunchKernelGGL(fold_cdiff_kernel, dim3(1024), dim3(256), 0, st, m, gH, grad, nodes);
        e = hipGetLastError();
    }
    std::vector<double> lr(n_rays);
    if (e == hipSuccess && n_rays)
        e = hipMemcpyAsync(lr.data(), loss_ray, sizeof(double) * n_rays, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(own_loss);
    (void)hipFree(ck);
    (void)hipFree(tape);
    (void)hipFree(xy);
    (void)hipFree(nops);
    (void)hipFree(endv);
    (void)hipFree(gH);
    if (e != hipSuccess) return fail_hip(e, "vrt_grid_loss_grad");
    double sum = 0.0;
    for (size_t i = 0; i < n_rays; ++i) sum += lr[i];  // fixed order
    *loss = scale * sum;
    return VRT_OK;
}
