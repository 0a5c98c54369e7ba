/*
 * vrt.h -- C ABI of libvrt, the MI355X (gfx950) library for the constant
 * optical-path-length vectorial ray march (VRT) through gradient-index media.
 *
 * The method (Sec. II of "Generalized vectorial ray tracing for optical
 * analysis and design in freeform gradient-index media"): a ray advances in
 * steps of constant optical path length dL0, i.e. geometric length
 * Delta_i = dL0 / n_i (Eqs. (3)-(4)).  At every point P_i the library
 * evaluates n and grad n, takes the local isoindicial normal N = grad n/|grad n|
 * (Eq. (5)) and applies the vectorial law of refraction R = mu I + gamma N
 * (Eqs. (9)-(10), mu = n(P_{i-1}) / n(P_i)), total internal reflection when
 * mu^2 (1 - (N.I)^2) >= 1 (Eqs. (19)-(20), the reflected step uses
 * Delta_{i-1}), the tangential arc rule when N.I = 0 (Eqs. (16)-(18)) and a
 * straight step where the gradient vanishes or is undefined (Eqs. (11)-(12)).
 * Where the step would cross the enclosing surface it is cut there and the
 * same law is applied with the surface normal (case (i)): the ray leaves into
 * the homogeneous surroundings or is reflected back inside.
 *
 * Conventions
 *   - Every function returns VRT_OK (0) or a negative vrt_error; nothing
 *     throws across the ABI.  vrt_last_error() gives a thread-local message
 *     for the most recent failure on the calling thread.
 *   - "device pointer" means memory on the context's HIP device (e.g. the
 *     data_ptr() of a torch tensor on that device).  The caller owns every ray
 *     and result buffer; the library never frees them.
 *   - The library owns the device copies of media until vrt_medium_destroy.
 *   - vrt_trace is asynchronous on the given HIP stream (a hipStream_t passed
 *     as void*; NULL = the null stream).  Results are valid once the stream
 *     has been synchronised.  Calls on one medium from several streams may
 *     overlap; the library keeps no per-trace mutable state on the medium
 *     except its ray-queue counter, which is per call (see vrt_trace).
 */
#ifndef VRT_H
#define VRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VRT_ABI_VERSION 1

typedef struct vrt_context_s *vrt_context_t;
typedef struct vrt_medium_s *vrt_medium_t;

/* return codes */
enum vrt_error {
    VRT_OK = 0,
    VRT_EINVAL = -1,       /* bad argument: null/misaligned pointer, dL0 <= 0, n <= 0, NaN parameter */
    VRT_ENOMEM = -2,       /* device allocation failed */
    VRT_EHIP = -3,         /* HIP runtime error; the message carries hipGetErrorString */
    VRT_EUNSUPPORTED = -4, /* valid request this library version does not implement */
    VRT_ETIMEOUT = -5      /* vrt_server_wait: the job is not done yet */
};

/* medium kinds (index distributions n(P)) */
enum vrt_medium_kind {
    VRT_MEDIUM_HOMOGENEOUS = 0, /* params [n_h]                        Sec. II case (iii)          */
    VRT_MEDIUM_LINEAR = 1,      /* params [n0, gx, gy, gz]             n = n0 + g.P (stratified)   */
    VRT_MEDIUM_LUNEBURG = 2,    /* params [R, cx, cy, cz]              n = sqrt(2 - |P-C|^2/R^2)  */
    VRT_MEDIUM_FIBER = 3,       /* params [n_c, Delta, R, cx, cy]      Sec. IV, Eq. (21), axis z   */
    VRT_MEDIUM_GAUSSIAN = 4,    /* params [n0, K, (A, sigma, cx, cy, cz) x K], K <= VRT_MAX_BUMPS
                                   n = n0 + sum A exp(-|P-c|^2 / (2 sigma^2))                     */
    VRT_MEDIUM_GRID = 5,        /* discretized medium, see vrt_medium_create_grid                  */
    VRT_MEDIUM_SPHERICAL = 6,   /* params [a0, a1, a2, a3, cx, cy, cz]  Sec. V, Eq. (26): spherical
                                 * freeform n = a0 + a1 G1 + a2 G2 + a3 G3 about c,
                                 * G1 = 0.3 (r^2 - 1), G2 = r cos(5 theta), G3 = r^2 sin^2(theta)
                                 * cos(2 phi); the gradient is undefined at r = 0 (case (ii)) */
    VRT_MEDIUM_N2P = 7,         /* params [R, F, beta, gamma]  Sec. VI, Eq. (27): cylindrical N2P
                                 * lens n = [1 + ((R^2 - (rho/2)^2) / F^2)^beta]^gamma, rho the
                                 * distance from the z axis; the lens volume is the boundary
                                 * (cylinder 0 <= rho <= R), n_ambient the surroundings (1) */
    VRT_MEDIUM_ZERNIKE = 8      /* params [n_lo, n_hi, rho_max, z_max, K, (j, l, c) x K]  Sec. V:
                                 * freeform cylindrical lens n = n0 + dn sum c Z_j(x', y') V_l(z'),
                                 * n0 = (n_hi + n_lo)/2, dn = (n_hi - n_lo)/2, x' = x/rho_max,
                                 * y' = y/rho_max, z' = 2z/z_max - 1; Z_j the Fringe Zernike
                                 * polynomial j (1..16, unnormalised: Z4 = 2 rho^2 - 1,
                                 * Z5 = rho^2 cos 2theta, ...), V_l the Legendre polynomial
                                 * l (0..3); repeated (j, l) pairs add; K <= 64.  The lens
                                 * volume is the boundary (normally the cylinder rho <= rho_max,
                                 * 0 <= z <= z_max) */
};
#define VRT_MAX_BUMPS 64

/* enclosing convex surface (Sec. II case (i)) */
enum vrt_boundary_kind {
    VRT_BOUNDARY_BOX = 0,      /* params [lox, loy, loz, hix, hiy, hiz]   */
    VRT_BOUNDARY_SPHERE = 1,   /* params [cx, cy, cz, r]                  */
    VRT_BOUNDARY_CYLINDER = 2  /* params [cx, cy, r, z0, z1], axis along z */
};

typedef struct {
    int32_t kind;     /* vrt_boundary_kind */
    int32_t reserved; /* must be 0 */
    double params[6];
} vrt_boundary;

/* arithmetic of the march */
enum vrt_precision {
    VRT_FP64 = 0,      /* plain double-precision march, one lane per ray, one launch per batch */
    VRT_FP32_COMP = 1  /* single precision with compensated position / direction accumulation,
                          double precision for the refraction/TIR discriminant, surface events
                          and the exit plane; persistent lanes refilled from a ray queue */
};

typedef struct {
    double dL0;           /* optical path length per step (> 0), Eqs. (3)-(4) */
    int64_t max_steps;    /* per-ray step budget (> 0); rays that use it up end TRUNCATED */
    double eps_tan;       /* |N.I| <= eps_tan selects the tangential rule (iv); 0 = exact zero only */
    double crit_rad;      /* near-critical flag window (radians, >= 0) */
    double tie_eps;       /* near-tie flag window (length, >= 0, <= 1e-6), see VRT_FLAG_NEAR_TIE */
    double exit_plane_z;  /* NaN: no exit plane; otherwise exiting rays are continued
                             straight to z = exit_plane_z (status NO_PLANE if they cannot) */
    int32_t precision;    /* vrt_precision */
    int32_t max_lanes;    /* VRT_FP32_COMP: at most this many persistent lanes (rounded up to a
                             multiple of 256) pull rays from the batch's queue; 0 = as many as
                             the device keeps resident.  A ray's result does not depend on it.
                             Must be 0 for VRT_FP64 (one lane per ray). */
} vrt_trace_params;

/* Ray batch, structure of arrays, all device pointers.  Element type is
 * double for VRT_FP64 and float for VRT_FP32_COMP.  Inputs: launch point
 * (px,py,pz) and launch direction (dx,dy,dz, any non-zero length; it is
 * normalised).  Outputs: exit point (ox,oy,oz) -- on the surface, or on the
 * exit plane when one is set -- and exit direction (odx,ody,odz); per-ray
 * status (vrt_ray_status), steps (moves made, including moves cut at the
 * surface), n_tir (interior TIRs), n_btir (TIRs at the surface) and flags
 * (vrt_ray_flag bits).  Input and output arrays must not overlap. */
typedef struct {
    const void *px, *py, *pz, *dx, *dy, *dz;
    void *ox, *oy, *oz, *odx, *ody, *odz;
    uint32_t *status, *steps, *n_tir, *n_btir, *flags;
} vrt_rays;

enum vrt_ray_status {
    VRT_RAY_EXITED = 0,
    VRT_RAY_MISSED = 1,             /* launched outside, the line misses the medium */
    VRT_RAY_TRUNCATED = 2,          /* max_steps used up; exit state = last point / direction */
    VRT_RAY_NO_PLANE = 3,           /* exited, but cannot reach the exit plane; exit state on the surface */
    VRT_RAY_INVALID_INPUT = 4,      /* non-finite launch state or zero direction */
    VRT_RAY_REFLECTED_AT_ENTRY = 5  /* TIR at the entry point (denser surroundings) */
};

enum vrt_ray_flag {
    VRT_FLAG_NEAR_CRITICAL = 1, /* some decision with mu > 1 had |acos|N.I| - asin(1/mu)| < crit_rad */
    VRT_FLAG_TANGENT = 2,       /* the tangential rule (iv) was used */
    VRT_FLAG_STRAIGHT = 4,      /* a straight step at zero / undefined gradient (ii)/(iii) */
    VRT_FLAG_BOUNDARY_TIR = 8,  /* reflected at the enclosing surface at least once */
    VRT_FLAG_NEAR_TIE = 16,     /* some move ended within tie_eps of the enclosing surface,
                                   measured perpendicular to it ("full step or cut" is then
                                   decided by rounding) */
    VRT_FLAG_NEAR_GRAZING = 32  /* some refraction with mu < 1 had |N.I| < crit_rad (Eq. (10)
                                   sends the ray to the side of the isoindicial surface given
                                   by sgn(N.I)) */
};

typedef struct {
    uint64_t rays, steps, exited, missed, truncated, no_plane, invalid, reflected_at_entry;
    uint64_t tir_interior, tir_boundary, flagged_near_critical, tangent, straight, flagged_near_tie;
    uint64_t flagged_near_grazing;
} vrt_counters;

/* Version of this ABI (VRT_ABI_VERSION). */
int vrt_abi_version(void);

/* Create a context on HIP device `hip_device` (makes it current for the
 * calling thread).  *out receives the handle.  Errors: EINVAL (bad device or
 * null out), EHIP. */
int vrt_context_create(int hip_device, vrt_context_t *out);

/* Destroy a context.  All media created on it must have been destroyed.
 * Errors: EINVAL (null, or media still alive). */
int vrt_context_destroy(vrt_context_t ctx);

/* Create an analytic medium (kind != GRID) inside boundary `bnd`, surrounded
 * by a homogeneous medium of index n_ambient.  params: host array of
 * n_params doubles (layout in vrt_medium_kind); copied, the caller keeps
 * ownership.  Errors: EINVAL (unknown kind, wrong n_params, n <= 0 or
 * non-finite parameters, K > VRT_MAX_BUMPS), ENOMEM, EHIP. */
int vrt_medium_create_analytic(vrt_context_t ctx, int kind, const double *params, int n_params,
                               const vrt_boundary *bnd, double n_ambient, vrt_medium_t *out);

/* Create a discretized medium from nx*ny*nz float index values (x fastest,
 * then y, then z) at nodes x_i = lo + i (hi - lo)/(nx - 1) (same for y, z),
 * bounded by the box [lo, hi] in surroundings of index n_ambient.  Between
 * nodes n is the trilinear interpolant and grad n the trilinear interpolant
 * of the node central differences (one-sided at the first and last node).
 * `values` is a host pointer if values_on_device == 0, else a device pointer
 * whose contents must be complete when the call is made (the copy runs on the
 * library's own stream, not the caller's); it is copied either way and the
 * call returns once the medium is ready.  Each dimension must be >= 2 and
 * <= 4096.
 * Errors: EINVAL (sizes, non-positive or non-finite values, lo >= hi),
 * ENOMEM, EHIP. */
int vrt_medium_create_grid(vrt_context_t ctx, const float *values, int nx, int ny, int nz,
                           const double lo[3], const double hi[3], double n_ambient,
                           int values_on_device, vrt_medium_t *out);

/* Destroy a medium.  Returns without waiting: its device memory is freed in
 * stream order on the library's own stream once every eager vrt_trace /
 * vrt_trace_paths launched on it has completed (the library records an event
 * per stream after each launch).  Launches captured in a graph are not
 * tracked: the owner of the graph must not replay it after destroying a
 * medium it reads.  Errors: EINVAL (NULL, or serving jobs on the medium not
 * yet done). */
int vrt_medium_destroy(vrt_medium_t m);

/* Device memory held by the medium, in bytes. */
int vrt_medium_device_bytes(vrt_medium_t m, size_t *out);

/* Trace n_rays rays (asynchronous on `stream`).  n_rays may be 0 (no-op).
 * Errors (nothing is launched): EINVAL for null or misaligned pointers, pointers
 * to pageable host memory (the arrays must be device, managed or pinned), dL0 <= 0,
 * max_steps <= 0, max_lanes < 0 (or != 0 with VRT_FP64), unknown precision,
 * n_rays >= 2^31, and for VRT_FP32_COMP in a Gaussian-sum medium a dL0 above
 * 0.05 n_min sigma_min (the single-precision index difference is kept to its
 * stated accuracy only below that); EUNSUPPORTED for combinations this library version
 * does not implement; EHIP for launch failures; ENOMEM when a trace is captured in a
 * graph and the context has no queue slot left for it.
 * Concurrency: traces may run on any streams at once.  A VRT_FP32_COMP launch
 * takes a ray-queue counter from the context: eager launches share 64 recycled
 * counters, each guarded by an event (a launch waits on its stream for the
 * counter's previous launch); a launch captured in a graph keeps a counter of
 * its own for the context's life (960 of them), so replays never share one
 * with any other launch.  A trace ends with its longest rays on a nearly
 * idle device; a caller with a stream of batches keeps two traces in flight
 * on two streams so that the next one fills it (a ray's result does not
 * depend on what runs beside it).
 * Device memory: an eager VRT_FP32_COMP launch on a grid or Zernike-lens
 * medium first enters every ray (launch, flight to the enclosing surface,
 * entry refraction) in a kernel of its own and keeps the 80-byte states in
 * memory taken from the device's stream-ordered pool on `stream` and returned
 * to it behind the march on the same stream.  A launch captured in a graph,
 * or one the pool cannot serve, enters the rays inside the march instead;
 * the results are the same bit for bit. */
int vrt_trace(vrt_medium_t m, const vrt_trace_params *p, const vrt_rays *rays, size_t n_rays,
              void *stream);

/* Trace n_rays rays with the plain double-precision march (p->precision must
 * be VRT_FP64) and record each ray's polyline P_0, P_1, ... of Sec. II
 * (Eqs. (3)-(4)): the launch point, the entry point on the enclosing surface,
 * the end of every constant-OPL step, and every point where a step meets the
 * surface (boundary TIR, exit).  The exit-plane continuation is not part of
 * the polyline.  Asynchronous on `stream`; the exit states go to `rays` as in
 * vrt_trace.
 *   path      device array of n_rays * cap * 3 doubles, point-major: point k
 *             of ray r at path[(k * n_rays + r) * 3 + {0,1,2}] for
 *             k < min(cap, n_points[r]); other entries are left untouched.
 *   cap       points kept per ray, >= 1.
 *   n_points  device array of n_rays uint64: the number of points of each
 *             ray's polyline (it may exceed cap; then only the first cap are
 *             stored).
 * The caller owns path and n_points.  Errors: as vrt_trace, and EINVAL for
 * another precision, cap == 0 or n_rays * cap * 24 bytes beyond the address
 * space, and a null or misaligned path or n_points. */
int vrt_trace_paths(vrt_medium_t m, const vrt_trace_params *p, const vrt_rays *rays,
                    size_t n_rays, double *path, uint64_t cap, uint64_t *n_points, void *stream);

/* Sum the per-ray outputs of a finished trace (status, steps, n_tir, n_btir,
 * flags of `rays`) into *out.  Runs a reduction kernel on `stream` and
 * synchronises that stream.  Errors: EINVAL, EHIP. */
int vrt_reduce_counters(vrt_context_t ctx, const vrt_rays *rays, size_t n_rays,
                        vrt_counters *out, void *stream);

/* ---------------------------------------------------------------------------
 * Design sweep of the cylindrical N2P-GRIN lens (Sec. VI, Eqs. (27)-(29)).
 *
 * `lens` is a VRT_MEDIUM_N2P medium (its R and F, its cylinder boundary on the
 * z axis from z0 = -L to z1 = 0, its surroundings) whose beta and gamma are
 * replaced, candidate by candidate, by beta_gamma[2c], beta_gamma[2c + 1]
 * (host array, n_cand pairs).  For each candidate, n_rays rays are launched
 * parallel to the axis from (0, y[i], z_launch) (host array of heights;
 * z_launch < z0) and traced with the plain FP64 march (p->precision VRT_FP64,
 * no exit plane).  z_int,i is the axial coordinate where the exit line of ray
 * i crosses the optical axis (the line is followed forwards only), and
 * rmse[c] = sqrt(mean_i (F - z_int,i)^2) (host array, n_cand values), or +inf
 * when a ray does not exit or does not head towards the axis.  z_int (host,
 * n_cand * n_rays, candidate-major) and steps (host, n_cand: the ray-steps
 * of each candidate's rays) are optional (NULL).  One launch on `stream`,
 * synchronised before returning; the few device buffers are allocated per
 * call.  Errors: EINVAL (arguments), EHIP.
 * --------------------------------------------------------------------------- */
int vrt_n2p_sweep(vrt_medium_t lens, const double *beta_gamma, size_t n_cand, const double *y,
                  size_t n_rays, double z_launch, const vrt_trace_params *p, double *rmse,
                  double *z_int, uint64_t *steps, void *stream);

/* vrt_n2p_sweep for callers that cannot allocate device memory (code that
 * must not call hipMalloc / hipFree, tight design loops that call the sweep
 * once per refinement level).  Same arguments, results and errors as
 * vrt_n2p_sweep; the sweep's device buffers (candidate descriptors, ray
 * heights, RMSE, and z_int / steps when asked for) are carved from one fixed
 * 4 MiB device array that the library holds on each device it runs on until
 * the process ends, instead of being allocated per call.  It calls no
 * hipMalloc, hipFree or allocating library routine.
 *   Limit: the buffers, each rounded up to 256 bytes -- 264 * n_cand
 *   (descriptors) + 8 * n_rays + 8 * n_cand (RMSE), plus 8 * n_cand * n_rays
 *   with z_int and 8 * n_cand with steps -- must fit in 4 MiB (about 14,900
 *   candidates of 10 rays, 11,600 with z_int and steps); beyond that the
 *   call returns EINVAL without touching the device.
 *   Every call on a device shares that device's array: calls that overlap in
 *   time on one device (from several threads or streams) race and must not
 *   be issued.  Each call synchronises `stream` before returning. */
int vrt_n2p_sweep_noalloc(vrt_medium_t lens, const double *beta_gamma, size_t n_cand,
                          const double *y, size_t n_rays, double z_launch,
                          const vrt_trace_params *p, double *rmse, double *z_int,
                          uint64_t *steps, void *stream);

/* ---------------------------------------------------------------------------
 * Gradient of an exit-plane loss with respect to a grid medium's node values
 * (the direct-design use of the march, Sec. VI, made differentiable).
 *
 * For rays j with launch state (P0_j, d0_j) and target point t_j on the exit
 * plane z = p->exit_plane_z, the plain FP64 march (Sec. II) gives the point
 * x_j where ray j meets the plane; the loss is L = scale * sum_j |x_j - t_j|^2
 * (x, y components), rays that do not reach the plane contributing 0.  The
 * gradient is that of the discrete march with its branch pattern held fixed
 * (Snell / TIR / straight decisions, step counts, surface events): the march
 * is piecewise smooth in the node values and this is its derivative wherever
 * no decision flips.  Computed by a hand-written reverse sweep: each ray's
 * state is checkpointed every checkpoint_every steps, each interval is
 * replayed from its checkpoint (bit for bit the forward march) and walked
 * backwards through the vector-Jacobian product of each operation.
 * --------------------------------------------------------------------------- */
typedef struct {
    const double *px, *py, *pz, *dx, *dy, *dz; /* launch states (device, n_rays each) */
    const double *tx, *ty;                     /* target point on the exit plane (device) */
    double *loss_ray;                          /* out (device, n_rays): |x_j - t_j|^2, 0 when
                                                  the ray misses the plane; may be NULL */
    int32_t *end;                              /* out (device, n_rays): 1 reached the plane,
                                                  2 did not; may be NULL */
} vrt_adjoint_rays;

/* grid: a VRT_MEDIUM_GRID medium in a box (its node values are the
 * parameters).  p: VRT_FP64, an exit plane, eps_tan = 0, max_steps <= 1e6.
 * *loss (host) receives L.  grad: device array of nz*ny*nx doubles (x
 * fastest), overwritten with dL/dv; NULL computes the loss only.  Runs on
 * `stream` and synchronises it; device scratch for the gradient
 * (checkpoints and tapes, about (max_steps / checkpoint_every + 2 +
 * 2 checkpoint_every) x 96 B per ray, for as many rays at a time as 8 GiB
 * holds) is allocated per call.  Errors: EINVAL (arguments), ENOMEM, EHIP. */
int vrt_grid_loss_grad(vrt_medium_t grid, const vrt_trace_params *p, const vrt_adjoint_rays *rays,
                       size_t n_rays, double scale, int checkpoint_every, double *loss,
                       double *grad, void *stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of trace jobs.
 *
 * A server owns a pool of device memory of `hbm_budget` bytes and one
 * persistent kernel that marches the rays of every admitted job, whatever
 * its medium kind (FP32_COMP only).  A job is a batch of rays against one
 * medium already resident on the device, given in PINNED HOST memory
 * (vrt_rays with host pointers into hipHostMalloc allocations, float
 * elements).  Jobs are admitted in submission order as soon as their rays fit
 * in the pool (68 bytes per ray) and their job slot is free; an admitted
 * job's inputs are copied in by the SDMA copy engines, and the running kernel
 * picks it up while it still marches earlier jobs: its waves move to the next
 * job with unclaimed rays as their lanes run dry, so the work of jobs
 * overlaps on the device.  When the last ray of a job retires, its outputs
 * are copied back into the job's host arrays and the job is done.  The
 * kernel never waits for work queued on a stream: host and kernel talk
 * through pinned host memory, so copies and new jobs reach it while it runs.
 * Each ray's result is the same as vrt_trace with VRT_FP32_COMP gives it
 * (same per-ray arithmetic), whatever else runs.  The kernel leaves about
 * 2 ms after the last job retired; relaunches replay a captured hipGraph.
 * While it runs it occupies every compute unit it was sized for, so other
 * kernels on the device wait for it.  Host scheduling runs on a thread owned
 * by the server; submit, query, wait and stats may be called from several
 * host threads at once (they serialise on the server's lock), destroy from
 * one thread once the others are done with the server.
 *
 * Not from the paper: the paper traces rays one at a time; this is the batch
 * scheduling of its per-ray march (Sec. II).
 * --------------------------------------------------------------------------- */
typedef struct vrt_server_s *vrt_server_t;

enum vrt_job_state {
    VRT_JOB_QUEUED = 0,   /* waiting for pool space / a job slot */
    VRT_JOB_RUNNING = 1,  /* admitted: inputs copied in, then visible to the kernel */
    VRT_JOB_COPYING = 2,  /* all rays retired, outputs being copied back */
    VRT_JOB_DONE = 3
};

typedef struct {
    int32_t state;        /* vrt_job_state */
    int32_t error;        /* 0, or the VRT_E* code the job failed with */
    uint64_t n_rays;
    uint64_t ray_steps;   /* sum of per-ray steps (valid when DONE) */
    double t_submit;      /* seconds on the server's steady clock */
    double t_admit;       /* pool space granted */
    double t_start;       /* inputs in the pool, job handed to the kernel */
    double t_retired;     /* last ray retired (observed by the host) */
    double t_done;        /* outputs in host memory */
} vrt_job_info;

typedef struct {
    uint64_t jobs_submitted, jobs_done, rays_done, ray_steps_done;
    uint64_t kernel_launches;   /* persistent-kernel runs (graph replays) */
    uint64_t pool_bytes, pool_peak_bytes;
    uint32_t job_slots, lanes;  /* job-table capacity, most persistent lanes running at once */
} vrt_server_stats;

/* Create a server on ctx with a device pool of hbm_budget bytes (>= 1 MiB,
 * allocated once here; nothing is allocated per job).  The persistent kernel
 * fills the device (all compute units at its occupancy); max_lanes caps its
 * lanes (multiples of 256; 0 = no cap).  Errors: EINVAL, ENOMEM, EHIP. */
int vrt_server_create(vrt_context_t ctx, size_t hbm_budget, int max_lanes, vrt_server_t *out);

/* Submit a job: n_rays rays of `host_rays` (host pointers, float elements,
 * layout as vrt_rays, every array inside one pinned host allocation; inputs
 * read and outputs written by the server until the job is DONE) against
 * medium m, which must stay alive until then (its destruction is refused
 * meanwhile).  p->precision must be VRT_FP32_COMP and p->max_lanes 0.  *job
 * receives the job id.  Errors: EINVAL (arguments, arrays not in pinned host
 * memory, a job larger than the whole pool, medium of another context), the
 * same parameter checks as vrt_trace. */
int vrt_server_submit(vrt_server_t s, vrt_medium_t m, const vrt_trace_params *p,
                      const vrt_rays *host_rays, size_t n_rays, uint64_t *job);

/* State of a job (non-blocking).  Errors: EINVAL (unknown job). */
int vrt_server_query(vrt_server_t s, uint64_t job, vrt_job_info *out);

/* Block until the job is DONE or timeout_s seconds passed (< 0: no limit).
 * Returns VRT_OK when done, VRT_ETIMEOUT otherwise (*out filled either way). */
int vrt_server_wait(vrt_server_t s, uint64_t job, double timeout_s, vrt_job_info *out);

/* Totals since creation. */
int vrt_server_stats_get(vrt_server_t s, vrt_server_stats *out);

/* Wait for every submitted job, stop the kernel and free the pool.
 * Errors: EHIP. */
int vrt_server_destroy(vrt_server_t s);

/* Thread-local description of the last error on this thread ("" if none). */
const char *vrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VRT_H */
