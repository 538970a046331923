"""Python binding of libodp.so: the gfx950 time-dependent HJ level-set solver.

Argument marshalling only.  Every step of the solve runs in the library's HIP
kernels; torch provides device memory and streams.  The entry points keep
the C names of include/odp.h (odp_grid_create, odp_hj_solve, odp_hj_batch,
odp_server_create, odp_serve_submit, odp_serve_poll, ...); `solve`,
`batch` and `Server` are thin conveniences on top of them.

If libodp.so has not been built the first call raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libodp.so")

ODP_TILE_AUTOTUNE = -1  # odp_solve_opts.tile_chunk: timed candidates, cached per shape
ODP_OK = 0
ODP_PENDING = 1
ODP_EINVAL = -1
ODP_ENOMEM = -2
ODP_EHIP = -3
ODP_EUNSUPPORTED = -4
ODP_EAGAIN = -5
ODP_ENONFINITE = -6
ODP_ECANCELED = -7

ODP_BRS = 0
ODP_BRT = 1
ODP_MIN_V0, ODP_MAX_V0, ODP_MIN_VINIT, ODP_MAX_VINIT, ODP_MIN_TARGET, ODP_MAX_TARGET = 1, 2, 3, 4, 5, 6
ODP_MIN_OBSTACLE, ODP_MAX_OBSTACLE = 1, 2
# the computation methods of the paper's table, by name
METHODS = {"None": ODP_BRS, "minVWithV0": ODP_MIN_V0, "maxVWithV0": ODP_MAX_V0,
           "minVWithVInit": ODP_MIN_VINIT, "maxVWithVInit": ODP_MAX_VINIT,
           "minVWithVTarget": ODP_MIN_TARGET, "maxVWithVTarget": ODP_MAX_TARGET}
OBSTACLE_METHODS = {"None": 0, "minVWithObstacle": ODP_MIN_OBSTACLE,
                    "maxVWithObstacle": ODP_MAX_OBSTACLE}

SYMBOLS = [
    "odp_strerror", "odp_last_error", "odp_grid_create", "odp_grid_destroy", "odp_grid_points",
    "odp_hj_workspace_bytes", "odp_hj_solve", "odp_hj_batch_workspace_bytes", "odp_hj_batch",
    "odp_server_create", "odp_serve_submit", "odp_serve_poll", "odp_serve_cancel",
    "odp_server_counts", "odp_server_destroy", "odp_ttr_workspace_bytes", "odp_ttr_solve",
    "odp_hj_solve_noalloc",
]


class OdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"odp error {code}: {msg}")
        self.code = code


class odp_dynamics(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int32), ("u_mode", ctypes.c_int32), ("d_mode", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("p", ctypes.c_double * 16)]


class odp_solve_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rk_order", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("mode", ctypes.c_int32), ("dissipation", ctypes.c_int32), ("max_dt", ctypes.c_double),
                ("save_all", ctypes.c_int32), ("tile_chunk", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("xcd_group", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("obstacle_mode", ctypes.c_int32), ("set_slices", ctypes.c_int32),
                ("target_dev", ctypes.c_void_p), ("obstacle_dev", ctypes.c_void_p),
                ("space_order", ctypes.c_int32), ("pad2_", ctypes.c_int32)]


class odp_solve_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double),
                ("t_final", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("alg_gbps", ctypes.c_double),
                ("roofline_frac", ctypes.c_double), ("alpha_max", ctypes.c_double * 6),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double), ("admit_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("retire_ms", ctypes.c_double),
                ("nonfinite", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k == "alpha_max" else getattr(self, k))
                for k, _ in self._fields_ if k != "pad_"}


class odp_ttr_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("check_every", ctypes.c_int32), ("eps", ctypes.c_double),
                ("max_iters", ctypes.c_int64), ("big", ctypes.c_double), ("stream", ctypes.c_void_p)]


class odp_ttr_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("last_change", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("alg_gbps", ctypes.c_double),
                ("roofline_frac", ctypes.c_double), ("converged", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class odp_solve_desc(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("dyn", odp_dynamics), ("V0_dev", ctypes.c_void_p),
                ("tau", ctypes.POINTER(ctypes.c_double)), ("ntau", ctypes.c_int32),
                ("rk_order", ctypes.c_int32), ("V_out_dev", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libodp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c "
                               "'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        L.odp_strerror.restype = ctypes.c_char_p
        L.odp_strerror.argtypes = [i32]
        L.odp_last_error.restype = ctypes.c_char_p
        L.odp_last_error.argtypes = []
        L.odp_grid_create.restype = i32
        L.odp_grid_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int64), dp, dp,
                                      ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(vp)]
        L.odp_grid_destroy.restype = None
        L.odp_grid_destroy.argtypes = [vp]
        L.odp_grid_points.restype = i64
        L.odp_grid_points.argtypes = [vp]
        L.odp_hj_workspace_bytes.restype = ctypes.c_size_t
        L.odp_hj_workspace_bytes.argtypes = [vp, ctypes.POINTER(odp_dynamics), dp, i32,
                                             ctypes.POINTER(odp_solve_opts)]
        L.odp_hj_solve.restype = i32
        L.odp_hj_solve.argtypes = [vp, ctypes.POINTER(odp_dynamics), vp, vp, dp, i32,
                                   ctypes.POINTER(odp_solve_opts), vp, vp, vp,
                                   ctypes.POINTER(odp_solve_stats)]
        L.odp_hj_solve_noalloc.restype = i32
        L.odp_hj_solve_noalloc.argtypes = [vp, ctypes.POINTER(odp_dynamics), vp, vp, dp, i32,
                                           ctypes.POINTER(odp_solve_opts), vp, vp,
                                           ctypes.POINTER(odp_solve_stats)]
        if hasattr(L, "odp_hj_batch"):
            L.odp_hj_batch_workspace_bytes.restype = ctypes.c_size_t
            L.odp_hj_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(odp_solve_desc),
                                                       ctypes.POINTER(odp_solve_opts)]
            L.odp_hj_batch.restype = i32
            L.odp_hj_batch.argtypes = [i32, ctypes.POINTER(odp_solve_desc),
                                       ctypes.POINTER(odp_solve_opts), vp, ctypes.c_size_t,
                                       ctypes.POINTER(odp_solve_stats)]
        L.odp_ttr_workspace_bytes.restype = ctypes.c_size_t
        L.odp_ttr_workspace_bytes.argtypes = [vp, ctypes.POINTER(odp_ttr_opts)]
        L.odp_ttr_solve.restype = i32
        L.odp_ttr_solve.argtypes = [vp, ctypes.POINTER(odp_dynamics), vp, ctypes.POINTER(odp_ttr_opts), vp,
                                    ctypes.c_size_t, vp, ctypes.POINTER(odp_ttr_stats)]
        if hasattr(L, "odp_server_create"):
            L.odp_server_create.restype = i32
            L.odp_server_create.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(odp_solve_opts),
                                            ctypes.POINTER(vp)]
            L.odp_serve_submit.restype = i32
            L.odp_serve_submit.argtypes = [vp, ctypes.POINTER(odp_solve_desc),
                                           ctypes.POINTER(ctypes.c_uint64)]
            L.odp_serve_poll.restype = i32
            L.odp_serve_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_size_t,
                                         ctypes.POINTER(odp_solve_stats)]
            L.odp_serve_cancel.restype = i32
            L.odp_serve_cancel.argtypes = [vp, ctypes.c_uint64]
            L.odp_server_counts.restype = i32
            L.odp_server_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int)]
            L.odp_server_destroy.restype = None
            L.odp_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise OdpError(rc, f"{lib().odp_strerror(rc).decode()}: {lib().odp_last_error().decode()}")
    return rc


def odp_strerror(code: int) -> str:
    return lib().odp_strerror(code).decode()


def odp_last_error() -> str:
    return lib().odp_last_error().decode()


# ----------------------------------------------------------------- grid

class Grid:
    """Owning wrapper of an odp_grid handle."""

    def __init__(self, n: Sequence[int], lo: Sequence[float], hi: Sequence[float],
                 periodic: Sequence[int]):
        self.n = [int(x) for x in n]
        self.handle = odp_grid_create(len(n), n, lo, hi, periodic)

    @classmethod
    def from_spec(cls, g):
        return cls(g.n, g.lo, g.hi, g.periodic)

    @property
    def npts(self) -> int:
        return int(lib().odp_grid_points(self.handle))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.odp_grid_destroy(h)
            self.handle = None


def odp_grid_create(ndim, n, lo, hi, periodic):
    n_a = (ctypes.c_int64 * ndim)(*[int(x) for x in n])
    lo_a = (ctypes.c_double * ndim)(*[float(x) for x in lo])
    hi_a = (ctypes.c_double * ndim)(*[float(x) for x in hi])
    pe_a = (ctypes.c_uint8 * ndim)(*[1 if x else 0 for x in periodic])
    out = ctypes.c_void_p()
    _check(lib().odp_grid_create(ndim, n_a, lo_a, hi_a, pe_a, ctypes.byref(out)))
    return out.value


def odp_grid_destroy(handle):
    lib().odp_grid_destroy(handle)


def make_dynamics(dyn) -> odp_dynamics:
    d = odp_dynamics()
    d.id = int(dyn.id)
    d.u_mode = int(dyn.u_mode)
    d.d_mode = int(dyn.d_mode)
    for k, v in enumerate(dyn.params):
        d.p[k] = float(v)
    return d


def method_code(mode) -> int:
    """odp_mode from a computation-method name of the paper's table
    ("minVWithV0", ...), "None", or an int."""
    return METHODS[mode] if isinstance(mode, str) else int(mode)


def obstacle_code(mode) -> int:
    return OBSTACLE_METHODS[mode] if isinstance(mode, str) else int(mode)


def make_opts(precision=32, rk_order=1, cfl=0.8, mode=ODP_BRT, dissipation=0, max_dt=0.0,
              save_all=0, tile_chunk=0, stream=None, xcd_group=0, graph=0, obstacle_mode=0,
              target=None, obstacle=None, set_slices=0, space_order=1) -> odp_solve_opts:
    """target / obstacle: device tensors (or raw device addresses) for the
    target and obstacle methods: one grid, or set_slices grids (time-varying
    sets, one per tau point)."""
    o = odp_solve_opts()
    o.precision = precision
    o.rk_order = rk_order
    o.cfl = cfl
    o.mode = method_code(mode)
    o.obstacle_mode = obstacle_code(obstacle_mode)
    addr = lambda x: None if x is None else (x if isinstance(x, int) else int(x.data_ptr()))
    o.target_dev = addr(target)
    o.obstacle_dev = addr(obstacle)
    o.set_slices = set_slices
    o.space_order = space_order
    o.dissipation = dissipation
    o.max_dt = max_dt
    o.save_all = save_all
    o.tile_chunk = tile_chunk
    o.stream = stream
    o.xcd_group = xcd_group
    o.graph = graph
    return o


def _tau_array(tau):
    arr = (ctypes.c_double * len(tau))(*[float(x) for x in tau])
    return arr


def _stream_handle(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(int(stream.cuda_stream)) if hasattr(stream, "cuda_stream") else stream


def odp_hj_workspace_bytes(grid: Grid, dyn, tau, opts: odp_solve_opts) -> int:
    d = make_dynamics(dyn)
    t = _tau_array(tau)
    return int(lib().odp_hj_workspace_bytes(grid.handle, ctypes.byref(d), t, len(tau), ctypes.byref(opts)))


def odp_hj_solve(grid: Grid, dyn, V0, V_init, tau, opts: odp_solve_opts, workspace, V_out,
                 V_all=None, want_stats=True):
    """Raw entry point: tensors (or None) are passed by data_ptr."""
    d = make_dynamics(dyn)
    t = _tau_array(tau)
    st = odp_solve_stats()
    ptr = lambda x: None if x is None else ctypes.c_void_p(x.data_ptr())
    rc = lib().odp_hj_solve(grid.handle, ctypes.byref(d), ptr(V0), ptr(V_init), t, len(tau),
                            ctypes.byref(opts), ptr(workspace), ptr(V_out), ptr(V_all),
                            ctypes.byref(st) if want_stats else None)
    _check(rc)
    return st


def odp_hj_solve_noalloc(grid: Grid, dyn, V0, V_init, tau, opts: odp_solve_opts, V_out, V_all=None,
                         want_stats=True):
    """Raw allocation-free entry point (the library's fixed scratch array as
    the workspace): tensors (or None) are passed by data_ptr."""
    d = make_dynamics(dyn)
    t = _tau_array(tau)
    st = odp_solve_stats()
    ptr = lambda x: None if x is None else ctypes.c_void_p(x.data_ptr())
    rc = lib().odp_hj_solve_noalloc(grid.handle, ctypes.byref(d), ptr(V0), ptr(V_init), t, len(tau),
                                    ctypes.byref(opts), ptr(V_out), ptr(V_all),
                                    ctypes.byref(st) if want_stats else None)
    _check(rc)
    return st


# ----------------------------------------------------------- conveniences

@dataclass
class SolveResult:
    V: "object"            # torch tensor on the device
    stats: dict
    V_all: Optional[object] = None


def _torch_dtype(precision):
    import torch
    return torch.float32 if precision == 32 else torch.float64


def check_device_tensor(x, precision, npts, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if x.dtype != _torch_dtype(precision) or not x.is_contiguous() or x.numel() != npts:
        raise ValueError(f"{name} must be contiguous {_torch_dtype(precision)} with {npts} elements")


def make_ttr_opts(precision=32, eps=1e-6, max_iters=100000, big=1e4, check_every=32,
                  stream=None) -> odp_ttr_opts:
    o = odp_ttr_opts()
    o.precision = precision
    o.check_every = check_every
    o.eps = eps
    o.max_iters = max_iters
    o.big = big
    o.stream = stream
    return o


def ttr_solve(grid_spec, dyn, target, precision=32, eps=1e-6, max_iters=100000, big=1e4,
              check_every=32, stream=None, workspace=None):
    """Time to reach {l <= 0} (odp_ttr_solve); target: device tensor l(z).
    Returns (phi tensor, stats dict)."""
    import torch
    grid = Grid.from_spec(grid_spec)
    check_device_tensor(target, precision, grid.npts, "target")
    o = make_ttr_opts(precision, eps, max_iters, big, check_every, _stream_handle(stream))
    d = make_dynamics(dyn)
    out = torch.empty_like(target)
    st = odp_ttr_stats()
    ws = None if workspace is None else ctypes.c_void_p(workspace.data_ptr())
    wsb = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().odp_ttr_solve(grid.handle, ctypes.byref(d), ctypes.c_void_p(target.data_ptr()),
                               ctypes.byref(o), ws, wsb, ctypes.c_void_p(out.data_ptr()), ctypes.byref(st)))
    return out, st.as_dict()


def solve(spec, V0, precision=32, V_init=None, tau=None, stream=None, save_all=False,
          dissipation=0, max_dt=0.0, tile_chunk=0, workspace=None, rk_order=None, cfl=None,
          mode=None, xcd_group=0, graph=0, obstacle_mode=0, target=None,
          obstacle=None, space_order=1) -> SolveResult:
    """One solve of a workloads.SolveSpec with a device V0 tensor.  mode and
    obstacle_mode take the paper's method names or the odp codes; target /
    obstacle are device tensors on the grid for the methods that use them, or
    of shape (len(tau), *grid) for time-varying sets (slice k at tau[k])."""
    import torch
    grid = Grid.from_spec(spec.grid)
    npts = grid.npts
    check_device_tensor(V0, precision, npts, "V0")
    tau = list(spec.tau if tau is None else tau)
    if V_init is not None:
        check_device_tensor(V_init, precision, npts, "V_init")
    sets = [x for x in (target, obstacle) if x is not None]
    slices = 0
    if sets:
        slices = len(tau) if sets[0].numel() == len(tau) * npts and len(tau) * npts != npts else 0
        for x, name in ((target, "target"), (obstacle, "obstacle")):
            if x is not None:
                check_device_tensor(x, precision, npts * max(slices, 1), name)
    opts = make_opts(precision, spec.rk_order if rk_order is None else rk_order,
                     spec.cfl if cfl is None else cfl, spec.mode if mode is None else mode,
                     dissipation, max_dt, 1 if save_all else 0, tile_chunk, _stream_handle(stream),
                     xcd_group, graph, obstacle_mode, target, obstacle, slices, space_order)
    out = torch.empty_like(V0)
    vall = torch.empty((len(tau),) + tuple(V0.shape), dtype=V0.dtype, device=V0.device) if save_all else None
    st = odp_hj_solve(grid, spec.dyn, V0, V_init, tau, opts, workspace, out, vall)
    return SolveResult(out, st.as_dict(), vall)


# ------------------------------------------- the paper's solver interface

def HJSolver(dyn, grid, targets, tau, comp_methods=None, save_all=False, precision=32,
             rk_order=1, cfl=0.8, space_order=1, device="cuda:0"):
    """The paper's HJSolver call (Solving HJ PDEs section): dyn and grid are
    workloads.DynSpec / GridSpec; targets is the initial value l(z) (host
    array on the grid), or [l, g] with g the obstacle for a reach-avoid
    problem (l then also serves as the target of the target-set methods); tau
    the output times; comp_methods {"TargetSetMode": ..., "ObstacleSetMode":
    ...} with the method names of the paper's table (default: none, the
    backward reachable set).  Returns V at tau[-1] as a host float64 array,
    or V at every tau (first axis) when save_all.  Runs odp_hj_solve on the
    device."""
    import numpy as np
    import torch
    from . import workloads as _W
    cm = dict(comp_methods or {})
    tmode = cm.get("TargetSetMode", "None")
    omode = cm.get("ObstacleSetMode", "None")
    if isinstance(targets, (list, tuple)):
        l, g = targets[0], (targets[1] if len(targets) > 1 else None)
    else:
        l, g = targets, None
    l = np.asarray(l, dtype=np.float64)
    dt = torch.float32 if precision == 32 else torch.float64
    dev = torch.device(device)
    V0 = torch.tensor(l, dtype=dt, device=dev)
    uses_target = tmode in ("minVWithVTarget", "maxVWithVTarget")
    uses_obst = omode != "None"
    if uses_obst and g is None:
        raise ValueError("the obstacle method needs targets = [l, g]")
    spec = _W.SolveSpec(grid, dyn, list(tau), rk_order=rk_order, cfl=cfl, mode=method_code(tmode))
    res = solve(spec, V0, precision=precision, save_all=save_all, mode=tmode, obstacle_mode=omode,
                target=V0 if uses_target else None,
                obstacle=torch.tensor(np.asarray(g, dtype=np.float64), dtype=dt, device=dev) if uses_obst else None,
                space_order=space_order)
    torch.cuda.synchronize()
    out = res.V_all if save_all else res.V
    return out.double().cpu().numpy()


def TTRSolver(dyn, grid, target, epsilon=1e-5, precision=32, max_iters=100000, device="cuda:0"):
    """The paper's TTRSolver call: the time to reach {l <= 0} (l: host array
    on the grid) by Lax-Friedrichs sweeping, to convergence epsilon.  dyn's
    control must minimise the time (u_mode 0).  Returns (phi as a host
    float64 array, stats).  Runs odp_ttr_solve on the device."""
    import numpy as np
    import torch
    dt = torch.float32 if precision == 32 else torch.float64
    tg = torch.tensor(np.asarray(target, dtype=np.float64), dtype=dt, device=torch.device(device))
    phi, st = ttr_solve(grid, dyn, tg, precision=precision, eps=epsilon, max_iters=max_iters)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy(), st


class BatchPlan:
    """Prebuilt odp_hj_batch arguments (grid handles, descriptors, tau arrays)
    for repeated calls on the same solves."""

    def __init__(self, specs, V0s, outs, precision=32, tile_chunk=0, dissipation=0, max_dt=0.0,
                 xcd_group=0, space_order=1):
        n = len(specs)
        self.n = n
        self.grids = [Grid.from_spec(s.grid) for s in specs]
        self.outs = outs
        self.descs = (odp_solve_desc * n)()
        self.taus = []
        for i, s in enumerate(specs):
            check_device_tensor(V0s[i], precision, self.grids[i].npts, f"V0[{i}]")
            check_device_tensor(outs[i], precision, self.grids[i].npts, f"V_out[{i}]")
            t = _tau_array(s.tau)
            self.taus.append(t)
            d = self.descs[i]
            d.grid = self.grids[i].handle
            d.dyn = make_dynamics(s.dyn)
            d.V0_dev = V0s[i].data_ptr()
            d.tau = ctypes.cast(t, ctypes.POINTER(ctypes.c_double))
            d.ntau = len(s.tau)
            d.rk_order = int(s.rk_order)
            d.V_out_dev = outs[i].data_ptr()
        s0 = specs[0]
        self.opts = make_opts(precision, s0.rk_order, s0.cfl, s0.mode, dissipation, max_dt, 0,
                              tile_chunk, None, xcd_group, space_order=space_order)
        self.stats = (odp_solve_stats * n)()

    def workspace_bytes(self) -> int:
        return int(lib().odp_hj_batch_workspace_bytes(self.n, self.descs, ctypes.byref(self.opts)))

    def run(self, stream=None, workspace=None, want_stats=True):
        self.opts.stream = _stream_handle(stream)
        ws = None if workspace is None else ctypes.c_void_p(workspace.data_ptr())
        wsb = 0 if workspace is None else workspace.numel() * workspace.element_size()
        _check(lib().odp_hj_batch(self.n, self.descs, ctypes.byref(self.opts), ws, wsb,
                                  self.stats if want_stats else None))
        return [self.stats[i].as_dict() for i in range(self.n)] if want_stats else None


def batch(specs, V0s, precision=32, stream=None, tile_chunk=0, dissipation=0, max_dt=0.0,
          workspace=None, want_stats=True, space_order=1):
    """odp_hj_batch over a list of SolveSpecs (common CFL / mode; each spec's
    own RK order)."""
    import torch
    outs = [torch.empty_like(v) for v in V0s]
    plan = BatchPlan(specs, V0s, outs, precision, tile_chunk, dissipation, max_dt,
                     space_order=space_order)
    return outs, plan.run(stream, workspace, want_stats)


# ----------------------------------------------------------------- serve

class Server:
    """Continuous-batching server (odp_server_create / odp_serve_*).

    Requests carry host V0 arrays (copied at submit); results come back as
    host arrays.  rk_order of a request defaults to the server's."""

    def __init__(self, budget_bytes: int, max_slots: int, precision=32, rk_order=1, cfl=0.8,
                 mode=ODP_BRT, dissipation=0, tile_chunk=0, space_order=1):
        self.precision = precision
        opts = make_opts(precision, rk_order, cfl, mode, dissipation, 0.0, 0, tile_chunk, None,
                         space_order=space_order)
        h = ctypes.c_void_p()
        _check(lib().odp_server_create(int(budget_bytes), int(max_slots), ctypes.byref(opts),
                                       ctypes.byref(h)))
        self.handle = h.value
        self._dtype = np.float32 if precision == 32 else np.float64

    def submit(self, spec, V0_host: np.ndarray, rk_order: int = 0) -> int:
        arr = np.ascontiguousarray(V0_host, dtype=self._dtype)
        grid = Grid.from_spec(spec.grid)
        if arr.size != grid.npts:
            raise ValueError("V0 does not match the grid")
        t = _tau_array(spec.tau)
        d = odp_solve_desc()
        d.grid = grid.handle
        d.dyn = make_dynamics(spec.dyn)
        d.V0_dev = arr.ctypes.data
        d.tau = ctypes.cast(t, ctypes.POINTER(ctypes.c_double))
        d.ntau = len(spec.tau)
        d.rk_order = int(rk_order)
        d.V_out_dev = None
        ticket = ctypes.c_uint64()
        _check(lib().odp_serve_submit(self.handle, ctypes.byref(d), ctypes.byref(ticket)))
        return int(ticket.value)

    def poll(self, ticket: int, out: np.ndarray):
        """Returns (status, stats dict or None); fills `out` when done."""
        st = odp_solve_stats()
        rc = lib().odp_serve_poll(self.handle, ctypes.c_uint64(ticket), out.ctypes.data,
                                  out.nbytes, ctypes.byref(st))
        if rc == ODP_PENDING:
            return rc, None
        _check(rc)
        return rc, st.as_dict()

    def cancel(self, ticket: int):
        _check(lib().odp_serve_cancel(self.handle, ctypes.c_uint64(ticket)))

    def counts(self):
        q, r, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().odp_server_counts(self.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(d)))
        return q.value, r.value, d.value

    def close(self):
        if self.handle:
            lib().odp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
