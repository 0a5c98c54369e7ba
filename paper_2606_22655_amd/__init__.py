"""Python binding of libvrt (include/vrt.h): the constant-OPL vectorial ray
march through gradient-index media on MI355X (gfx950).

The functions named ``vrt_*`` mirror the C entry points one to one and only
marshal arguments; every step of the march runs in the HIP kernels of
``libvrt.so``.  PyTorch provides device memory and the HIP stream.  There is
no CPU fallback: if the library has not been built, or no GPU is present,
the calls raise.

Convenience layer: ``Context``, ``Medium`` (built from the medium dicts of
``workloads.py``), ``trace`` (torch tensors in, dict of tensors out) and
``trace_batches`` (a list of batches, two traces in flight on two streams).
"""
from __future__ import annotations

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrt.so")

VRT_OK, VRT_EINVAL, VRT_ENOMEM, VRT_EHIP, VRT_EUNSUPPORTED, VRT_ETIMEOUT = 0, -1, -2, -3, -4, -5
MEDIUM_KINDS = {"homogeneous": 0, "linear": 1, "luneburg": 2, "fiber": 3, "gaussian": 4, "grid": 5,
                "spherical": 6, "n2p": 7, "zernike": 8}
BOUNDARY_KINDS = {"box": 0, "sphere": 1, "cylinder": 2}
VRT_FP64, VRT_FP32_COMP = 0, 1
PRECISIONS = {"fp64": VRT_FP64, "fp32c": VRT_FP32_COMP}
STATUS = {"EXITED": 0, "MISSED": 1, "TRUNCATED": 2, "NO_PLANE": 3, "INVALID_INPUT": 4,
          "REFLECTED_AT_ENTRY": 5}
FLAG_NEAR_CRITICAL, FLAG_TANGENT, FLAG_STRAIGHT, FLAG_BOUNDARY_TIR, FLAG_NEAR_TIE = 1, 2, 4, 8, 16
FLAG_NEAR_GRAZING = 32

EXPORTED = ["vrt_abi_version", "vrt_context_create", "vrt_context_destroy",
            "vrt_medium_create_analytic", "vrt_medium_create_grid", "vrt_medium_destroy",
            "vrt_medium_device_bytes", "vrt_trace", "vrt_reduce_counters", "vrt_last_error",
            "vrt_server_create", "vrt_server_submit", "vrt_server_query", "vrt_server_wait",
            "vrt_server_stats_get", "vrt_server_destroy", "vrt_n2p_sweep", "vrt_grid_loss_grad",
            "vrt_trace_paths", "vrt_n2p_sweep_noalloc"]
JOB_STATES = {0: "QUEUED", 1: "RUNNING", 2: "COPYING", 3: "DONE"}


class VrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvrt error {code}: {msg}")
        self.code = code


class vrt_boundary(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("params", C.c_double * 6)]


class vrt_trace_params(C.Structure):
    _fields_ = [("dL0", C.c_double), ("max_steps", C.c_int64), ("eps_tan", C.c_double),
                ("crit_rad", C.c_double), ("tie_eps", C.c_double), ("exit_plane_z", C.c_double),
                ("precision", C.c_int32), ("max_lanes", C.c_int32)]


class vrt_rays(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("px", "py", "pz", "dx", "dy", "dz", "ox", "oy", "oz",
                                          "odx", "ody", "odz", "status", "steps", "n_tir",
                                          "n_btir", "flags")]


COUNTER_FIELDS = ["rays", "steps", "exited", "missed", "truncated", "no_plane", "invalid",
                  "reflected_at_entry", "tir_interior", "tir_boundary", "flagged_near_critical",
                  "tangent", "straight", "flagged_near_tie", "flagged_near_grazing"]


class vrt_adjoint_rays(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("px", "py", "pz", "dx", "dy", "dz", "tx", "ty",
                                          "loss_ray", "end")]


class vrt_counters(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in COUNTER_FIELDS]


class vrt_job_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("error", C.c_int32), ("n_rays", C.c_uint64),
                ("ray_steps", C.c_uint64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_start", C.c_double), ("t_retired", C.c_double), ("t_done", C.c_double)]


class vrt_server_stats(C.Structure):
    _fields_ = [("jobs_submitted", C.c_uint64), ("jobs_done", C.c_uint64),
                ("rays_done", C.c_uint64), ("ray_steps_done", C.c_uint64),
                ("kernel_launches", C.c_uint64), ("pool_bytes", C.c_uint64),
                ("pool_peak_bytes", C.c_uint64), ("job_slots", C.c_uint32), ("lanes", C.c_uint32)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libvrt.so and declare its entry points (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libvrt.so is not built ({path}); run "
                          "`python -m paper_2606_22655_amd.build` first")
    # torch ships its own HIP runtime under the same soname as the system one
    # libvrt.so links against; whichever is loaded first serves the process.
    # Load torch's first so that both share one runtime (streams and device
    # pointers pass between them), and torch still finds its devices.
    import torch  # noqa: F401

    lib = C.CDLL(path)
    vp, i32 = C.c_void_p, C.c_int
    lib.vrt_abi_version.restype = i32
    lib.vrt_abi_version.argtypes = []
    lib.vrt_context_create.argtypes = [i32, C.POINTER(vp)]
    lib.vrt_context_destroy.argtypes = [vp]
    lib.vrt_medium_create_analytic.argtypes = [vp, i32, C.POINTER(C.c_double), i32,
                                               C.POINTER(vrt_boundary), C.c_double, C.POINTER(vp)]
    lib.vrt_medium_create_grid.argtypes = [vp, vp, i32, i32, i32, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.c_double, i32, C.POINTER(vp)]
    lib.vrt_medium_destroy.argtypes = [vp]
    lib.vrt_medium_device_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.vrt_trace.argtypes = [vp, C.POINTER(vrt_trace_params), C.POINTER(vrt_rays), C.c_size_t, vp]
    lib.vrt_trace_paths.argtypes = [vp, C.POINTER(vrt_trace_params), C.POINTER(vrt_rays),
                                    C.c_size_t, vp, C.c_uint64, vp, vp]
    lib.vrt_reduce_counters.argtypes = [vp, C.POINTER(vrt_rays), C.c_size_t,
                                        C.POINTER(vrt_counters), vp]
    lib.vrt_server_create.argtypes = [vp, C.c_size_t, i32, C.POINTER(vp)]
    lib.vrt_server_submit.argtypes = [vp, vp, C.POINTER(vrt_trace_params), C.POINTER(vrt_rays),
                                      C.c_size_t, C.POINTER(C.c_uint64)]
    lib.vrt_server_query.argtypes = [vp, C.c_uint64, C.POINTER(vrt_job_info)]
    lib.vrt_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(vrt_job_info)]
    lib.vrt_server_stats_get.argtypes = [vp, C.POINTER(vrt_server_stats)]
    lib.vrt_server_destroy.argtypes = [vp]
    lib.vrt_grid_loss_grad.argtypes = [vp, C.POINTER(vrt_trace_params), C.POINTER(vrt_adjoint_rays),
                                       C.c_size_t, C.c_double, i32, C.POINTER(C.c_double), vp, vp]
    dp = C.POINTER(C.c_double)
    lib.vrt_n2p_sweep.argtypes = [vp, dp, C.c_size_t, dp, C.c_size_t, C.c_double,
                                  C.POINTER(vrt_trace_params), dp, dp,
                                  C.POINTER(C.c_uint64), vp]
    lib.vrt_n2p_sweep_noalloc.argtypes = lib.vrt_n2p_sweep.argtypes
    lib.vrt_last_error.restype = C.c_char_p
    lib.vrt_last_error.argtypes = []
    for name in EXPORTED:
        if name not in ("vrt_last_error", "vrt_abi_version"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(rc):
    if rc != VRT_OK:
        raise VrtError(rc, vrt_last_error())
    return rc


# ---------------------------------------------------------------------------
# one-to-one entry points
# ---------------------------------------------------------------------------
def vrt_abi_version():
    return load_library().vrt_abi_version()


def vrt_last_error():
    return (load_library().vrt_last_error() or b"").decode()


def vrt_context_create(device=0):
    h = C.c_void_p()
    _check(load_library().vrt_context_create(int(device), C.byref(h)))
    return h


def vrt_context_destroy(ctx):
    _check(load_library().vrt_context_destroy(ctx))


def vrt_medium_create_analytic(ctx, kind, params, boundary, n_ambient):
    arr = (C.c_double * len(params))(*[float(x) for x in params])
    h = C.c_void_p()
    _check(load_library().vrt_medium_create_analytic(ctx, int(kind), arr, len(params),
                                                     C.byref(boundary), float(n_ambient),
                                                     C.byref(h)))
    return h


def vrt_medium_create_grid(ctx, values_ptr, nx, ny, nz, lo, hi, n_ambient, values_on_device):
    lo3 = (C.c_double * 3)(*[float(x) for x in lo])
    hi3 = (C.c_double * 3)(*[float(x) for x in hi])
    h = C.c_void_p()
    _check(load_library().vrt_medium_create_grid(ctx, C.c_void_p(values_ptr), int(nx), int(ny),
                                                 int(nz), lo3, hi3, float(n_ambient),
                                                 int(values_on_device), C.byref(h)))
    return h


def vrt_medium_destroy(m):
    _check(load_library().vrt_medium_destroy(m))


def vrt_medium_device_bytes(m):
    v = C.c_size_t()
    _check(load_library().vrt_medium_device_bytes(m, C.byref(v)))
    return v.value


def vrt_trace(medium, params, rays, n_rays, stream):
    return _check(load_library().vrt_trace(medium, C.byref(params), C.byref(rays), int(n_rays),
                                           C.c_void_p(stream)))


def vrt_trace_paths(medium, params, rays, n_rays, path, cap, n_points, stream):
    return _check(load_library().vrt_trace_paths(medium, C.byref(params), C.byref(rays),
                                                 int(n_rays), C.c_void_p(path), int(cap),
                                                 C.c_void_p(n_points), C.c_void_p(stream)))


def vrt_n2p_sweep(lens, beta_gamma, y, z_launch, params, stream=0, want_z=False,
                  want_steps=False):
    """RMSE_LSA per (beta, gamma) candidate, then (if asked) the axis
    crossings (n_cand, n_rays) and the ray-steps per candidate."""
    return _sweep(load_library().vrt_n2p_sweep, lens, beta_gamma, y, z_launch, params, stream,
                  want_z, want_steps)


def vrt_n2p_sweep_noalloc(lens, beta_gamma, y, z_launch, params, stream=0, want_z=False,
                          want_steps=False):
    """vrt_n2p_sweep with the device buffers in the library's fixed scratch
    array (no device allocation per call)."""
    return _sweep(load_library().vrt_n2p_sweep_noalloc, lens, beta_gamma, y, z_launch, params,
                  stream, want_z, want_steps)


def _sweep(fn, lens, beta_gamma, y, z_launch, params, stream, want_z, want_steps):
    import numpy as np

    bg = np.ascontiguousarray(beta_gamma, dtype=np.float64).reshape(-1, 2)
    yy = np.ascontiguousarray(y, dtype=np.float64).ravel()
    rmse = np.zeros(bg.shape[0])
    z = np.zeros((bg.shape[0], yy.size)) if want_z else None
    st = np.zeros(bg.shape[0], dtype=np.uint64) if want_steps else None
    dp = C.POINTER(C.c_double)
    _check(fn(
        lens, bg.ctypes.data_as(dp), bg.shape[0], yy.ctypes.data_as(dp), yy.size,
        float(z_launch), C.byref(params), rmse.ctypes.data_as(dp),
        z.ctypes.data_as(dp) if want_z else None,
        st.ctypes.data_as(C.POINTER(C.c_uint64)) if want_steps else None, C.c_void_p(stream)))
    out = (rmse,) + ((z,) if want_z else ()) + ((st,) if want_steps else ())
    return out if len(out) > 1 else rmse


def vrt_grid_loss_grad(grid, params, rays, n_rays, scale, checkpoint_every, grad_ptr, stream):
    """Exit-plane loss (returned) and, when grad_ptr is not 0, dL/d(node values)
    written to the device array at grad_ptr."""
    loss = C.c_double()
    _check(load_library().vrt_grid_loss_grad(grid, C.byref(params), C.byref(rays), int(n_rays),
                                             float(scale), int(checkpoint_every), C.byref(loss),
                                             C.c_void_p(grad_ptr or None), C.c_void_p(stream)))
    return loss.value


def vrt_server_create(ctx, hbm_budget, max_lanes=0):
    h = C.c_void_p()
    _check(load_library().vrt_server_create(ctx, int(hbm_budget), int(max_lanes), C.byref(h)))
    return h


def vrt_server_submit(server, medium, params, host_rays, n_rays):
    job = C.c_uint64()
    _check(load_library().vrt_server_submit(server, medium, C.byref(params), C.byref(host_rays),
                                            int(n_rays), C.byref(job)))
    return job.value


def _info(i):
    return {"state": JOB_STATES.get(i.state, i.state), "error": i.error, "n_rays": i.n_rays,
            "ray_steps": i.ray_steps, "t_submit": i.t_submit, "t_admit": i.t_admit,
            "t_start": i.t_start, "t_retired": i.t_retired, "t_done": i.t_done}


def vrt_server_query(server, job):
    i = vrt_job_info()
    _check(load_library().vrt_server_query(server, int(job), C.byref(i)))
    return _info(i)


def vrt_server_wait(server, job, timeout_s=-1.0):
    """Returns the job's info; raises VrtError(VRT_ETIMEOUT) if not done in time."""
    i = vrt_job_info()
    _check(load_library().vrt_server_wait(server, int(job), float(timeout_s), C.byref(i)))
    return _info(i)


def vrt_server_stats_get(server):
    st = vrt_server_stats()
    _check(load_library().vrt_server_stats_get(server, C.byref(st)))
    return {k: int(getattr(st, k)) for k, _ in vrt_server_stats._fields_}


def vrt_server_destroy(server):
    _check(load_library().vrt_server_destroy(server))


def vrt_reduce_counters(ctx, rays, n_rays, stream):
    out = vrt_counters()
    _check(load_library().vrt_reduce_counters(ctx, C.byref(rays), int(n_rays), C.byref(out),
                                              C.c_void_p(stream)))
    return {k: int(getattr(out, k)) for k in COUNTER_FIELDS}


# ---------------------------------------------------------------------------
# convenience layer over torch tensors
# ---------------------------------------------------------------------------
def _torch():
    import torch

    return torch


class Context:
    def __init__(self, device=0):
        self.device = int(device)
        self.handle = vrt_context_create(self.device)

    def close(self):
        if self.handle is not None:
            vrt_context_destroy(self.handle)
            self.handle = None


class Medium:
    """Device-resident medium built from a ``workloads`` medium dict."""

    def __init__(self, ctx, spec):
        self.ctx = ctx
        self.spec = spec
        kind = spec["kind"]
        if kind == "grid":
            torch = _torch()
            g = spec["grid"]
            t = torch.as_tensor(g, dtype=torch.float32).contiguous()
            nz, ny, nx = t.shape
            self.handle = vrt_medium_create_grid(ctx.handle, t.data_ptr(), nx, ny, nz,
                                                 spec["grid_lo"], spec["grid_hi"], spec["n_amb"], 0)
        else:
            b = vrt_boundary()
            b.kind = BOUNDARY_KINDS[spec["boundary"]["kind"]]
            for i, v in enumerate(spec["boundary"]["params"]):
                b.params[i] = float(v)
            self.handle = vrt_medium_create_analytic(ctx.handle, MEDIUM_KINDS[kind],
                                                     list(spec["params"]), b, spec["n_amb"])

    @property
    def device_bytes(self):
        return vrt_medium_device_bytes(self.handle)

    def close(self):
        if self.handle is not None:
            vrt_medium_destroy(self.handle)
            self.handle = None


def _grid_from_device(ctx, values, lo, hi, n_amb):
    """A grid medium built on the device from a (nz, ny, nx) float32 CUDA tensor
    (the library copies it on its own stream: the tensor's writes on the current
    stream must be complete first)."""
    _torch().cuda.current_stream().synchronize()
    nz, ny, nx = values.shape
    return vrt_medium_create_grid(ctx.handle, values.data_ptr(), nx, ny, nz, lo, hi, n_amb, 1)


class ExitPlaneLoss:
    """L(v) = scale * sum_j |x_j(v) - t_j|^2: rays (P0, d0) marched in FP64
    through the grid medium whose node values are v (a (nz, ny, nx) float32
    CUDA tensor, nodes spanning lo..hi, surroundings n_amb) to the exit plane
    z = params["exit_plane_z"], where ray j lands at x_j; t_j its target.
    Calling it returns L as a torch scalar that backpropagates to v through
    the library's adjoint (vrt_grid_loss_grad)."""

    def __init__(self, ctx, P0, d0, targets, params, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 n_amb=1.0, scale=None, checkpoint_every=64):
        torch = _torch()
        self.ctx = ctx
        P0 = torch.as_tensor(P0, dtype=torch.float64)
        d0 = torch.as_tensor(d0, dtype=torch.float64)
        tg = torch.as_tensor(targets, dtype=torch.float64)
        self.n = P0.shape[0]
        self.buf = torch.empty((8, self.n), dtype=torch.float64, device="cuda")
        self.buf[0:3].copy_(P0.T)
        self.buf[3:6].copy_(d0.T)
        self.buf[6:8].copy_(tg.T)
        self.loss_ray = torch.zeros(self.n, dtype=torch.float64, device="cuda")
        self.end = torch.zeros(self.n, dtype=torch.int32, device="cuda")
        self.rays = vrt_adjoint_rays()
        for i, k in enumerate(("px", "py", "pz", "dx", "dy", "dz", "tx", "ty")):
            setattr(self.rays, k, self.buf[i].data_ptr())
        self.rays.loss_ray = self.loss_ray.data_ptr()
        self.rays.end = self.end.data_ptr()
        self.params = make_params(params, "fp64")
        self.lo, self.hi, self.n_amb = lo, hi, n_amb
        self.scale = 1.0 / max(self.n, 1) if scale is None else float(scale)
        self.checkpoint_every = int(checkpoint_every)

    def evaluate(self, values, grad=None):
        """Loss at values (float); the gradient into `grad` (float64 tensor of
        the same shape) when given."""
        torch = _torch()
        v = values.detach().to(torch.float32).contiguous()
        med = _grid_from_device(self.ctx, v, self.lo, self.hi, self.n_amb)
        try:
            return vrt_grid_loss_grad(med, self.params, self.rays, self.n, self.scale,
                                      self.checkpoint_every,
                                      grad.data_ptr() if grad is not None else 0,
                                      torch.cuda.current_stream().cuda_stream)
        finally:
            vrt_medium_destroy(med)

    def __call__(self, values):
        return _ExitPlaneLossFn.apply(values, self)


def _make_loss_fn():
    torch = _torch()

    class Fn(torch.autograd.Function):
        @staticmethod
        def forward(fctx, values, spec):
            fctx.save_for_backward(values)
            fctx.spec = spec
            return torch.tensor(spec.evaluate(values), dtype=torch.float64, device=values.device)

        @staticmethod
        def backward(fctx, gout):
            (values,) = fctx.saved_tensors
            g = torch.empty(values.shape, dtype=torch.float64, device=values.device)
            fctx.spec.evaluate(values, g)
            return (gout * g).to(values.dtype), None

    return Fn


class _LazyFn:
    fn = None

    def apply(self, *a):
        if _LazyFn.fn is None:
            _LazyFn.fn = _make_loss_fn()
        return _LazyFn.fn.apply(*a)


_ExitPlaneLossFn = _LazyFn()


def make_params(p, precision):
    q = vrt_trace_params()
    q.dL0 = float(p["dL0"])
    q.max_steps = int(p["max_steps"])
    q.eps_tan = float(p.get("eps_tan", 0.0))
    q.crit_rad = float(p.get("crit_rad", 1e-6))
    q.tie_eps = float(p.get("tie_eps", 1e-7))
    z = p.get("exit_plane_z")
    q.exit_plane_z = math.nan if z is None else float(z)
    q.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    q.max_lanes = int(p.get("max_lanes", 0))
    return q


class RayBatch:
    """Structure-of-arrays device buffers for one trace."""

    def __init__(self, P0, d0, precision, device="cuda"):
        torch = _torch()
        dt = torch.float64 if precision in ("fp64", VRT_FP64) else torch.float32
        P0 = torch.as_tensor(P0, dtype=dt)
        d0 = torch.as_tensor(d0, dtype=dt)
        n = P0.shape[0]
        self.n = n
        self.inp = torch.empty((6, n), dtype=dt, device=device)
        self.inp[0:3].copy_(P0.T)
        self.inp[3:6].copy_(d0.T)
        self.out = torch.empty((6, n), dtype=dt, device=device)
        self.u32 = torch.empty((5, n), dtype=torch.int32, device=device)
        self.rays = vrt_rays()
        names_in = ("px", "py", "pz", "dx", "dy", "dz")
        names_out = ("ox", "oy", "oz", "odx", "ody", "odz")
        for i, k in enumerate(names_in):
            setattr(self.rays, k, self.inp[i].data_ptr() if n else None)
        for i, k in enumerate(names_out):
            setattr(self.rays, k, self.out[i].data_ptr() if n else None)
        for i, k in enumerate(("status", "steps", "n_tir", "n_btir", "flags")):
            setattr(self.rays, k, self.u32[i].data_ptr() if n else None)

    def results(self):
        """Exit state as CPU numpy arrays (synchronises)."""
        o = self.out.double().cpu().numpy()
        u = self.u32.cpu().numpy().view("uint32")
        return {"P": o[0:3].T.copy(), "D": o[3:6].T.copy(), "status": u[0].copy(),
                "steps": u[1].copy(), "ntir": u[2].copy(), "nbtir": u[3].copy(),
                "flags": u[4].copy()}


def trace(medium, batch, params, precision, stream=None):
    """Enqueue the march of ``batch`` through ``medium`` on ``stream``
    (default: torch's current stream)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    vrt_trace(medium.handle, make_params(params, precision), batch.rays, batch.n, stream)


def trace_batches(medium, batches, params, precision, streams=None):
    """Enqueue the marches of several batches through ``medium``, two at a
    time: batch k goes to ``streams[k % 2]`` (default: two new streams), so
    that each trace's last long rays share the device with the next trace's
    start.  Both streams first wait for torch's current stream (inputs written
    there are visible), and the current stream then waits for both (results
    are ready in its order).  Each batch's result is the one ``trace`` gives."""
    if streams is not None and len(streams) != 2:
        raise ValueError("trace_batches: two streams")
    torch = _torch()
    cur = torch.cuda.current_stream()
    if streams is None:
        streams = (torch.cuda.Stream(), torch.cuda.Stream())
    for s in streams:
        s.wait_stream(cur)
    for k, b in enumerate(batches):
        trace(medium, b, params, precision, stream=streams[k % 2].cuda_stream)
    for s in streams:
        cur.wait_stream(s)


def trace_paths(medium, batch, params, cap, stream=None):
    """Enqueue the FP64 march of ``batch`` (an fp64 RayBatch) with its
    polylines recorded; returns device tensors ``path`` (cap, n, 3), point k
    of ray r at path[k, r], and ``n_points`` (n,) int64 (points of each
    polyline, possibly above cap)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    path = torch.empty((int(cap), batch.n, 3), dtype=torch.float64, device=batch.inp.device)
    n_points = torch.empty((batch.n,), dtype=torch.int64, device=batch.inp.device)
    vrt_trace_paths(medium.handle, make_params(params, "fp64"), batch.rays, batch.n,
                    path.data_ptr() if batch.n else None, cap,
                    n_points.data_ptr() if batch.n else None, stream)
    return path, n_points


def counters(ctx, batch, stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    return vrt_reduce_counters(ctx.handle, batch.rays, batch.n, stream)


def trace_numpy(spec, rays, params, precision="fp32c", device=0):
    """One-shot helper: build the medium, trace (P0, d0), return numpy results."""
    torch = _torch()
    ctx = Context(device)
    med = Medium(ctx, spec)
    try:
        b = RayBatch(rays[0], rays[1], precision)
        trace(med, b, params, precision)
        torch.cuda.synchronize()
        return b.results()
    finally:
        med.close()
        ctx.close()


class HostRays:
    """Structure-of-arrays HOST buffers of one served job (pinned float32 for
    the inputs and outputs, uint32 for the per-ray words)."""

    def __init__(self, P0, d0, pin=True):
        torch = _torch()
        P0 = torch.as_tensor(P0, dtype=torch.float32)
        d0 = torch.as_tensor(d0, dtype=torch.float32)
        n = P0.shape[0]
        self.n = n
        self.inp = torch.empty((6, n), dtype=torch.float32, pin_memory=pin)
        self.inp[0:3].copy_(P0.T)
        self.inp[3:6].copy_(d0.T)
        self.out = torch.empty((6, n), dtype=torch.float32, pin_memory=pin)
        self.u32 = torch.empty((5, n), dtype=torch.int32, pin_memory=pin)
        self.rays = vrt_rays()
        for i, k in enumerate(("px", "py", "pz", "dx", "dy", "dz")):
            setattr(self.rays, k, self.inp[i].data_ptr())
        for i, k in enumerate(("ox", "oy", "oz", "odx", "ody", "odz")):
            setattr(self.rays, k, self.out[i].data_ptr())
        for i, k in enumerate(("status", "steps", "n_tir", "n_btir", "flags")):
            setattr(self.rays, k, self.u32[i].data_ptr())

    def results(self):
        """Exit state as numpy arrays (valid once the job is DONE)."""
        o = self.out.double().numpy()
        u = self.u32.numpy().view("uint32")
        return {"P": o[0:3].T.copy(), "D": o[3:6].T.copy(), "status": u[0].copy(),
                "steps": u[1].copy(), "ntir": u[2].copy(), "nbtir": u[3].copy(),
                "flags": u[4].copy()}


class Server:
    """Continuous batching of trace jobs on one device (FP32 + compensation):
    a pool of hbm_budget bytes, a persistent kernel, a host scheduler thread."""

    def __init__(self, ctx, hbm_budget, max_lanes=0):
        self.handle = vrt_server_create(ctx.handle, hbm_budget, max_lanes)
        self._keep = {}

    def submit(self, medium, host_rays, params):
        job = vrt_server_submit(self.handle, medium.handle, make_params(params, "fp32c"),
                                host_rays.rays, host_rays.n)
        self._keep[job] = host_rays  # host buffers must outlive the job
        return job

    def wait(self, job, timeout_s=-1.0):
        info = vrt_server_wait(self.handle, job, timeout_s)
        self._keep.pop(job, None)
        return info

    def query(self, job):
        return vrt_server_query(self.handle, job)

    def stats(self):
        return vrt_server_stats_get(self.handle)

    def close(self):
        if self.handle is not None:
            vrt_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()
