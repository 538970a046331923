"""CPU oracle for the time-dependent HJ level-set solve (float64).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg.  The HIP library and its Python binding
never import, link or call anything in this folder.

The arithmetic lives in odp_oracle.c (plain C, one grid point at a time, in
the order of the paper's Algorithm 1); this module only builds it with gcc
and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "odp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable -O2, OpenMP over grid points,
    no floating-point contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_hj_solve.restype = ctypes.c_int
        lib.oracle_hj_solve.argtypes = [
            ctypes.c_int, _lp, _dp, _dp, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
            _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
            _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _lp, _dp,
            _dp, _dp]
        lib.oracle_cfl_dt.restype = ctypes.c_int
        lib.oracle_cfl_dt.argtypes = [
            ctypes.c_int, _lp, _dp, _dp, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
            ctypes.c_double, _dp, _dp]
        lib.oracle_step_at.restype = ctypes.c_int
        lib.oracle_step_at.argtypes = [
            ctypes.c_int, _lp, _dp, _dp, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
            _dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
            ctypes.c_int, ctypes.c_int, ctypes.c_long, _lp, _dp]
        lib.oracle_alpha_box.restype = ctypes.c_int
        lib.oracle_alpha_box.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                         ctypes.c_long, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_hamiltonian.restype = ctypes.c_int
        lib.oracle_hamiltonian.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           _dp, ctypes.c_long, _dp, _dp, _dp]
        lib.oracle_ttr_solve.restype = ctypes.c_int
        lib.oracle_ttr_solve.argtypes = [
            ctypes.c_int, _lp, _dp, _dp, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp,
            ctypes.c_double, ctypes.c_double, ctypes.c_long, ctypes.c_int, _dp, _lp, _dp]
        lib.oracle_box_alpha_max.restype = ctypes.c_int
        lib.oracle_box_alpha_max.argtypes = [
            ctypes.c_int, _lp, _dp, _dp, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp,
            ctypes.c_int, _dp, _dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


class use_library:
    """Context manager that points this module at another build of the
    oracle (the mutation tests use it to check that the pins have teeth)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, _LIB
        self._saved = (_lib, _LIB)
        _lib, _LIB = None, self.path
        return _load()

    def __exit__(self, *exc):
        global _lib, _LIB
        _lib, _LIB = self._saved
        return False


def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _grid_args(grid):
    n = _arr(grid.n, np.int64)
    lo = _arr(grid.lo, np.float64)
    hi = _arr(grid.hi, np.float64)
    per = _arr(grid.periodic, np.int32)
    return n, lo, hi, per


def _params(dyn):
    p = np.zeros(16, dtype=np.float64)
    p[: len(dyn.params)] = dyn.params
    return p


@dataclass
class OracleResult:
    V: np.ndarray
    steps: int
    dt_first: float
    dt_min: float
    dt_max: float
    V_all: Optional[np.ndarray] = None


# computation methods (the paper's table): target-set operations
TMODES = {"none": 0, "minVWithV0": 1, "maxVWithV0": 2, "minVWithVInit": 3, "maxVWithVInit": 4,
          "minVWithVTarget": 5, "maxVWithVTarget": 6}
OMODES = {"none": 0, "minVWithObstacle": 1, "maxVWithObstacle": 2}


def _modes(brt, tmode, omode, target, obstacle, P, ntau=1):
    """Returns (tmode, omode, target, obstacle, slices): arrays of P points,
    or of ntau slices of P points (time-varying sets, slice k at tau[k])."""
    tm = (1 if brt else 0) if tmode is None else (TMODES[tmode] if isinstance(tmode, str) else int(tmode))
    om = OMODES[omode] if isinstance(omode, str) else int(omode)
    tg = None if target is None else _arr(target, np.float64).reshape(-1)
    ob = None if obstacle is None else _arr(obstacle, np.float64).reshape(-1)
    sizes = {a.size for a in (tg, ob) if a is not None}
    if len(sizes) > 1 or (sizes and sizes.pop() not in (P, ntau * P)):
        raise ValueError("target / obstacle must hold one grid, or one grid per tau point")
    slices = ntau if any(a is not None and a.size == ntau * P != P for a in (tg, ob)) else 1
    return tm, om, tg, ob, slices


def solve(grid, dyn, V0: np.ndarray, tau: Sequence[float], rk_order=1, cfl=0.8, brt=True,
          global_alpha=False, max_dt=0.0, V_init: Optional[np.ndarray] = None,
          save_all=False, tmode=None, omode=0, target=None, obstacle=None,
          space_order=1) -> OracleResult:
    """space_order: 1 first-order upwind, 2 second-order ENO differences.
    tmode (overrides brt): a computation-method name or code (TMODES);
    omode: obstacle method (OMODES); target / obstacle: arrays on the grid,
    or (time-varying sets) len(tau) grids, the set at each tau[k]."""
    lib = _load()
    n, lo, hi, per = _grid_args(grid)
    V0 = _arr(V0, np.float64).reshape(-1)
    Vi = None if V_init is None else _arr(V_init, np.float64).reshape(-1)
    tau = _arr(tau, np.float64)
    P = int(np.prod(n))
    if V0.size != P:
        raise ValueError("V0 size does not match the grid")
    tm, om, tg, ob, slices = _modes(brt, tmode, omode, target, obstacle, P, len(tau))
    out = np.empty(P, dtype=np.float64)
    vall = np.empty((len(tau), P), dtype=np.float64) if save_all else None
    steps = ctypes.c_long(0)
    d1, d2, d3 = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    p = _params(dyn)
    rc = lib.oracle_hj_solve(
        grid.ndim, _ptr(n, _lp), _ptr(lo, _dp), _ptr(hi, _dp), _ptr(per, _ip), dyn.id,
        dyn.u_mode, dyn.d_mode, _ptr(p, _dp), _ptr(V0, _dp),
        _ptr(Vi, _dp) if Vi is not None else None, _ptr(tau, _dp), len(tau), rk_order, cfl,
        tm, om, _ptr(tg, _dp) if tg is not None else None, _ptr(ob, _dp) if ob is not None else None,
        slices, int(space_order), 1 if global_alpha else 0, max_dt, _ptr(out, _dp),
        _ptr(vall, _dp) if vall is not None else None, ctypes.byref(steps), ctypes.byref(d1),
        ctypes.byref(d2), ctypes.byref(d3))
    if rc != 0:
        raise ValueError("oracle_hj_solve rejected its arguments")
    shape = tuple(int(x) for x in n)
    return OracleResult(out.reshape(shape), int(steps.value), d1.value, d2.value, d3.value,
                        None if vall is None else vall.reshape((len(tau),) + shape))


def solve_spec(spec, V0=None, **kw) -> OracleResult:
    from paper_2204_05520_amd import workloads
    if V0 is None:
        V0 = workloads.make_v0(spec)
    return solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order, cfl=spec.cfl,
                 brt=spec.mode == 1, **kw)


def cfl_dt(grid, dyn, cfl=0.8):
    lib = _load()
    n, lo, hi, per = _grid_args(grid)
    amax = np.zeros(6, dtype=np.float64)
    dt = ctypes.c_double(0)
    p = _params(dyn)
    rc = lib.oracle_cfl_dt(grid.ndim, _ptr(n, _lp), _ptr(lo, _dp), _ptr(hi, _dp),
                           _ptr(per, _ip), dyn.id, dyn.u_mode, dyn.d_mode, _ptr(p, _dp), cfl,
                           _ptr(amax, _dp), ctypes.byref(dt))
    if rc != 0:
        raise ValueError("oracle_cfl_dt rejected its arguments")
    return amax[: grid.ndim].copy(), dt.value


def box_alpha_max(grid, dyn, V: np.ndarray, space_order=1):
    """Algorithm 1's alpha^max for field V: (box, alpha_max), box = (D_min,
    D_max) of the costate over the grid, alpha_max the largest alpha over that
    box at any node."""
    lib = _load()
    n, lo, hi, per = _grid_args(grid)
    V = _arr(V, np.float64).reshape(-1)
    box = np.zeros(12, dtype=np.float64)
    amax = np.zeros(6, dtype=np.float64)
    p = _params(dyn)
    rc = lib.oracle_box_alpha_max(grid.ndim, _ptr(n, _lp), _ptr(lo, _dp), _ptr(hi, _dp),
                                  _ptr(per, _ip), dyn.id, dyn.u_mode, dyn.d_mode, _ptr(p, _dp),
                                  _ptr(V, _dp), int(space_order), _ptr(box, _dp), _ptr(amax, _dp))
    if rc != 0:
        raise ValueError("oracle_box_alpha_max rejected its arguments")
    N = grid.ndim
    return (box[:N].copy(), box[N:2 * N].copy()), amax[:N].copy()


def step_at(grid, dyn, V: np.ndarray, V0: np.ndarray, dt: float, idx, rk_order=1, brt=True,
            alpha_glob=None, tmode=None, omode=0, target=None, obstacle=None, space_order=1,
            eno_f32=False) -> np.ndarray:
    """One full time step of size dt from V, evaluated only at flat indices
    idx.  eno_f32: take the ENO stencil choices in float32 (from the
    float32-rounded stencil), as a float32 solve does."""
    lib = _load()
    n, lo, hi, per = _grid_args(grid)
    V = _arr(V, np.float64).reshape(-1)
    V0 = _arr(V0, np.float64).reshape(-1)
    tm, om, tg, ob, _ = _modes(brt, tmode, omode, target, obstacle, V.size)
    idx = _arr(idx, np.int64)
    out = np.empty(idx.size, dtype=np.float64)
    ag = None if alpha_glob is None else _arr(alpha_glob, np.float64)
    p = _params(dyn)
    rc = lib.oracle_step_at(grid.ndim, _ptr(n, _lp), _ptr(lo, _dp), _ptr(hi, _dp),
                            _ptr(per, _ip), dyn.id, dyn.u_mode, dyn.d_mode, _ptr(p, _dp),
                            _ptr(V, _dp), _ptr(V0, _dp), dt, rk_order, tm, om,
                            _ptr(tg, _dp) if tg is not None else None,
                            _ptr(ob, _dp) if ob is not None else None,
                            _ptr(ag, _dp) if ag is not None else None, int(space_order),
                            1 if eno_f32 else 0, idx.size,
                            _ptr(idx, _lp), _ptr(out, _dp))
    if rc != 0:
        raise ValueError("oracle_step_at rejected its arguments")
    return out


def alpha_box(dyn, ndim, z, dmin, dmax):
    """Dissipation coefficients at states z (m x ndim) over the costate box
    [dmin, dmax], and over all admissible inputs: (alpha_box, alpha_all)."""
    lib = _load()
    z = _arr(z, np.float64).reshape(-1, ndim)
    dmin, dmax = _arr(dmin, np.float64), _arr(dmax, np.float64)
    ab = np.empty_like(z)
    aa = np.empty_like(z)
    p = _params(dyn)
    rc = lib.oracle_alpha_box(ndim, dyn.id, dyn.u_mode, dyn.d_mode, _ptr(p, _dp), z.shape[0],
                              _ptr(z, _dp), _ptr(dmin, _dp), _ptr(dmax, _dp), _ptr(ab, _dp),
                              _ptr(aa, _dp))
    if rc != 0:
        raise ValueError("oracle_alpha_box rejected its arguments")
    return ab, aa


def hamiltonian(dyn, ndim, z, p):
    """p . f(z, u*(p), d*(p)) at states z for costates p (both m x ndim)."""
    lib = _load()
    z = _arr(z, np.float64).reshape(-1, ndim)
    p_ = _arr(p, np.float64).reshape(-1, ndim)
    H = np.empty(z.shape[0])
    prm = _params(dyn)
    rc = lib.oracle_hamiltonian(ndim, dyn.id, dyn.u_mode, dyn.d_mode, _ptr(prm, _dp), z.shape[0],
                                _ptr(z, _dp), _ptr(p_, _dp), _ptr(H, _dp))
    if rc != 0:
        raise ValueError("oracle_hamiltonian rejected its arguments")
    return H


@dataclass
class TTRResult:
    phi: np.ndarray
    iters: int
    change: float


def ttr_solve(grid, dyn, target, eps=1e-9, max_iters=100000, big=1e4, jacobi=False) -> TTRResult:
    """Time-to-reach by Lax-Friedrichs sweeping; target: l(z) on the grid
    (the target set is l <= 0).  dyn's u_mode / d_mode say which player
    minimises the time (u_mode 0) and which maximises it (d_mode 1).
    jacobi: every node of an iteration from the previous iterate (the
    parallel form) instead of the Gauss-Seidel sweep."""
    lib = _load()
    n, lo, hi, per = _grid_args(grid)
    tg = _arr(target, np.float64).reshape(-1)
    P = int(np.prod(n))
    if tg.size != P:
        raise ValueError("target size does not match the grid")
    phi = np.empty(P, dtype=np.float64)
    it = ctypes.c_long(0)
    ch = ctypes.c_double(0)
    p = _params(dyn)
    rc = lib.oracle_ttr_solve(grid.ndim, _ptr(n, _lp), _ptr(lo, _dp), _ptr(hi, _dp), _ptr(per, _ip),
                              dyn.id, dyn.u_mode, dyn.d_mode, _ptr(p, _dp), _ptr(tg, _dp), big, eps,
                              max_iters, 1 if jacobi else 0, _ptr(phi, _dp), ctypes.byref(it),
                              ctypes.byref(ch))
    if rc != 0:
        raise ValueError("oracle_ttr_solve rejected its arguments")
    return TTRResult(phi.reshape(tuple(int(x) for x in n)), int(it.value), ch.value)
