"""Seeded synthetic inputs for the time-dependent HJ level-set solve.

This module only *describes and generates inputs*: grids, dynamics parameter
sets, the implicit target function l(z) (the initial value V0) and request
streams.  It holds none of the solver's arithmetic (no derivatives, no
Hamiltonians, no time stepping), so both the HIP library and the CPU oracle
can consume what it produces without sharing any method code.

Grid convention (the paper's Grid section: bounds, node count and periodic
dimensions per axis; the periodic upper bound is excluded):
    non-periodic axis: dx = (hi - lo) / (n - 1),  x_k = lo + k dx, k = 0..n-1
    periodic axis:     dx = (hi - lo) / n,        x_k = lo + k dx, k = 0..n-1

Target shapes follow the paper's Shapes module: a cylinder is the signed
distance sqrt(sum over kept axes of (z_a - c_a)^2) - r with some axes ignored
(the initial-condition example around the CylinderShape call).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# Dynamics ids; the numbering is the C ABI's odp_dyn_id.
DYN_SINGLE_INTEGRATOR = 0   # z' = c + u, |u|_2 <= u_max (test-only, N-D)
DYN_DUBINS3D = 1            # (x, y, th): v cos th, v sin th, w, |w| <= w_max
DYN_DYNCAR4D = 2            # (x, y, v, th): v cos th, v sin th, a, w
DYN_TWODUBINS6D = 3         # evader (x,y,th) + pursuer (x,y,th), two Dubins cars
DYN_PE3D = 4                # relative pursuit-evasion (x, y, th): evader a, pursuer b

MAXIMISE = 1
MINIMISE = 0

BRS = 0
BRT = 1

SEED_BATCH = 220405520
SEED_SERVE = 220405521


@dataclass
class GridSpec:
    n: List[int]
    lo: List[float]
    hi: List[float]
    periodic: List[int]

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def npts(self) -> int:
        return int(np.prod(np.asarray(self.n, dtype=np.int64)))

    def axis(self, d: int) -> np.ndarray:
        """Coordinates of axis d in float64 (input-side definition)."""
        n, lo, hi = self.n[d], self.lo[d], self.hi[d]
        h = (hi - lo) / n if self.periodic[d] else (hi - lo) / (n - 1)
        return lo + h * np.arange(n, dtype=np.float64)

    def domain_scale(self) -> float:
        """Largest extent over the non-periodic axes (the error scale S)."""
        ext = [self.hi[d] - self.lo[d] for d in range(self.ndim) if not self.periodic[d]]
        return max(ext) if ext else max(self.hi[d] - self.lo[d] for d in range(self.ndim))


@dataclass
class DynSpec:
    """Closed dynamics family + parameters.

    Parameter layout (p[0..]) per id:
      SINGLE_INTEGRATOR: p[0] = u_max, p[1..ndim] = drift c
      DUBINS3D:          p[0] = v, p[1] = w_max
      DYNCAR4D:          p[0] = a_max, p[1] = w_max
      TWODUBINS6D:       p[0] = v_e, p[1] = u_max (evader turn),
                         p[2] = v_p, p[3] = d_max (pursuer turn)
    u_mode / d_mode: 1 = the player maximises, 0 = minimises.
    """
    id: int
    params: List[float]
    u_mode: int = MAXIMISE
    d_mode: int = MINIMISE


@dataclass
class SolveSpec:
    grid: GridSpec
    dyn: DynSpec
    tau: List[float]
    rk_order: int = 1
    cfl: float = 0.8
    mode: int = BRT
    radius: float = 1.0
    target: str = "cylinder_xy"   # or "relative_distance" (6D game), "norm"
    name: str = ""
    extra: dict = field(default_factory=dict)


PI = math.pi


def angle_axis(n: int):
    return n, -PI, PI, 1


# --------------------------------------------------------------------------
# Target functions l(z) (V0), float64 on the host
# --------------------------------------------------------------------------

def cylinder_v0(grid: GridSpec, radius: float, keep=(0, 1), center=None) -> np.ndarray:
    """sqrt(sum_{a in keep} (z_a - c_a)^2) - r broadcast over the other axes."""
    nd = grid.ndim
    center = [0.0] * nd if center is None else list(center)
    acc = None
    for a in keep:
        x = grid.axis(a) - center[a]
        shape = [1] * nd
        shape[a] = grid.n[a]
        term = (x * x).reshape(shape)
        acc = term if acc is None else acc + term
    v = np.sqrt(acc) - radius
    return np.ascontiguousarray(np.broadcast_to(v, tuple(grid.n)), dtype=np.float64)


def relative_distance_v0(grid: GridSpec, radius: float) -> np.ndarray:
    """6D game: sqrt((x_e - x_p)^2 + (y_e - y_p)^2) - r, axes (xe, ye, the, xp, yp, thp)."""
    assert grid.ndim == 6
    xe, ye, xp, yp = grid.axis(0), grid.axis(1), grid.axis(3), grid.axis(4)
    dx = xe.reshape(-1, 1, 1, 1, 1, 1) - xp.reshape(1, 1, 1, -1, 1, 1)
    dy = ye.reshape(1, -1, 1, 1, 1, 1) - yp.reshape(1, 1, 1, 1, -1, 1)
    v = np.sqrt(dx * dx + dy * dy) - radius
    return np.ascontiguousarray(np.broadcast_to(v, tuple(grid.n)), dtype=np.float64)


def make_v0(spec: SolveSpec) -> np.ndarray:
    if spec.target == "relative_distance":
        return relative_distance_v0(spec.grid, spec.radius)
    if spec.target == "norm":
        return cylinder_v0(spec.grid, spec.radius, keep=tuple(range(spec.grid.ndim)))
    return cylinder_v0(spec.grid, spec.radius, keep=(0, 1))


def reach_avoid_sets(spec: SolveSpec, t: float = 0.0):
    """Target l(z) and obstacle g(z) for the target and obstacle computation
    methods, as in the paper's reach-avoid example (a goal and an obstacle,
    both cylinders over the position axes): l is the signed distance to a
    disc (negative inside), g = minus the signed distance to another disc
    (positive inside the obstacle).  Centres sit at fixed fractions of the
    domain at t = 0 and move with t (time-varying sets: call once per tau
    point); float64 on the host."""
    g = spec.grid
    keep = (0, 1) if g.ndim >= 2 else (0,)
    at = lambda f: [g.lo[d] + f[min(d, len(f) - 1)] * (g.hi[d] - g.lo[d]) for d in range(g.ndim)]
    ext = min(g.hi[d] - g.lo[d] for d in keep)
    target = cylinder_v0(g, 0.12 * ext, keep=keep, center=at([0.7 - 0.1 * t, 0.62]))
    obstacle = -cylinder_v0(g, 0.15 * ext, keep=keep, center=at([0.35, 0.45 + 0.1 * t]))
    return target, obstacle


def moving_sets(spec: SolveSpec, tau: Sequence[float]):
    """reach_avoid_sets at every tau[k], stacked: arrays of shape
    (len(tau), *grid)."""
    ls, gs = zip(*(reach_avoid_sets(spec, float(t)) for t in tau))
    return np.stack(ls), np.stack(gs)


def make_v0_torch(spec: SolveSpec, device, dtype):
    """Same V0 as make_v0, built on `device` slab by slab (for grids too large
    for a host float64 copy, e.g. 36^6).  Evaluated in float64, then rounded."""
    import torch
    g = spec.grid
    out = torch.empty(tuple(g.n), device=device, dtype=dtype)
    ax = [torch.tensor(g.axis(d), device=device, dtype=torch.float64) for d in range(g.ndim)]
    nd = g.ndim

    def bshape(d):
        s = [1] * (nd - 1)
        s[d - 1] = g.n[d]
        return s

    for i0 in range(g.n[0]):
        if spec.target == "relative_distance":
            dx = ax[0][i0] - ax[3].reshape(bshape(3))
            dy = ax[1].reshape(bshape(1)) - ax[4].reshape(bshape(4))
            v = torch.sqrt(dx * dx + dy * dy) - spec.radius
        elif spec.target == "norm":
            acc = ax[0][i0] * ax[0][i0]
            for d in range(1, nd):
                acc = acc + (ax[d] * ax[d]).reshape(bshape(d))
            v = torch.sqrt(acc) - spec.radius
        else:
            x0 = ax[0][i0]
            v = torch.sqrt(x0 * x0 + (ax[1] * ax[1]).reshape(bshape(1))) - spec.radius
        out[i0].copy_(v.expand(tuple(g.n[1:])).to(dtype))
    return out


# --------------------------------------------------------------------------
# The five benchmark workloads
# --------------------------------------------------------------------------

def config_dubins3d(n=(60, 60, 36), T=2.0) -> SolveSpec:
    """3D Dubins car BRT: v = 1, |w| <= 1, cylinder r = 1, RK1, CFL 0.8, FP64 form."""
    g = GridSpec(list(n), [-4.0, -4.0, -PI], [4.0, 4.0, PI], [0, 0, 1])
    d = DynSpec(DYN_DUBINS3D, [1.0, 1.0], MAXIMISE, MINIMISE)
    return SolveSpec(g, d, [0.0, T], rk_order=1, cfl=0.8, mode=BRT, radius=1.0,
                     name=f"dubins3d_{n[0]}x{n[1]}x{n[2]}_rk1_brt")


def config_dyncar4d(n=80, T=3.0) -> SolveSpec:
    """4D dynamic car BRT: |a| <= 1, |w| <= 1, disc r = 0.5, RK3, CFL 0.8."""
    ns = list(n) if isinstance(n, (list, tuple)) else [n] * 4
    g = GridSpec(ns, [-5.0, -5.0, 0.0, -PI], [5.0, 5.0, 4.0, PI], [0, 0, 0, 1])
    d = DynSpec(DYN_DYNCAR4D, [1.0, 1.0], MAXIMISE, MINIMISE)
    return SolveSpec(g, d, [0.0, T], rk_order=3, cfl=0.8, mode=BRT, radius=0.5,
                     name=f"dyncar4d_{'x'.join(map(str, ns))}_rk3_brt")


def config_game6d(n=36, T=2.0) -> SolveSpec:
    """6D two-Dubins-car game: evader u maximises, pursuer d minimises,
    speeds 1/1, turn bounds 1/1, capture radius 0.5, RK2, CFL 0.8."""
    ns = list(n) if isinstance(n, (list, tuple)) else [n] * 6
    g = GridSpec(ns, [-4.0, -4.0, -PI, -4.0, -4.0, -PI], [4.0, 4.0, PI, 4.0, 4.0, PI],
                 [0, 0, 1, 0, 0, 1])
    d = DynSpec(DYN_TWODUBINS6D, [1.0, 1.0, 1.0, 1.0], MAXIMISE, MINIMISE)
    return SolveSpec(g, d, [0.0, T], rk_order=2, cfl=0.8, mode=BRT, radius=0.5,
                     target="relative_distance", name=f"game6d_{'x'.join(map(str, ns))}_rk2_brt")


def config_pe3d(n=100, T=1.5, rk_order=1) -> SolveSpec:
    """3D relative pursuit-evasion (the paper's main example and its 100^3,
    horizon 1.5 benchmark row): |x|, |y| <= 4, th in [-pi, pi), speeds
    v_a = v_b = 1, turn bounds |a|, |b| <= 1; the evader a maximises, the
    pursuer b minimises; capture radius 0.5; first order, CFL 0.8, tube."""
    ns = list(n) if isinstance(n, (list, tuple)) else [n] * 3
    g = GridSpec(ns, [-4.0, -4.0, -PI], [4.0, 4.0, PI], [0, 0, 1])
    d = DynSpec(DYN_PE3D, [1.0, 1.0, 1.0, 1.0], MAXIMISE, MINIMISE)
    return SolveSpec(g, d, [0.0, T], rk_order=rk_order, cfl=0.8, mode=BRT, radius=0.5,
                     name=f"pe3d_{'x'.join(map(str, ns))}_rk{rk_order}_brt")


def batch_dubins3d(count=512, seed=SEED_BATCH) -> List[SolveSpec]:
    """512 Dubins BRT solves with n_x, n_y ~ U{32..80}, n_th ~ U{24..48},
    v ~ U[0.5,1.5], w_max ~ U[0.5,2], r ~ U[0.3,1.2]; domain, RK1, CFL 0.8 and
    horizon 2.0 as the single 3D workload."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(32, 81, size=count)
    ny = rng.integers(32, 81, size=count)
    nt = rng.integers(24, 49, size=count)
    v = rng.uniform(0.5, 1.5, size=count)
    w = rng.uniform(0.5, 2.0, size=count)
    r = rng.uniform(0.3, 1.2, size=count)
    out = []
    for i in range(count):
        g = GridSpec([int(nx[i]), int(ny[i]), int(nt[i])], [-4.0, -4.0, -PI], [4.0, 4.0, PI], [0, 0, 1])
        d = DynSpec(DYN_DUBINS3D, [float(v[i]), float(w[i])], MAXIMISE, MINIMISE)
        out.append(SolveSpec(g, d, [0.0, 2.0], rk_order=1, cfl=0.8, mode=BRT,
                             radius=float(r[i]), name=f"batch{i}"))
    return out


@dataclass
class Request:
    arrival_s: float
    spec: SolveSpec


def serve_requests(count=2200, rate=200.0, seed=SEED_SERVE) -> List[Request]:
    """Poisson arrivals at `rate`/s: 70% 3D Dubins (n ~ U{40..80} per axis,
    v, w_max, r as the batch workload, RK1), 30% 4D car (n ~ U{40..64} per
    axis, a_max ~ U[0.5,1.5], w_max ~ U[0.5,2], r ~ U[0.3,1.2], RK3); horizon
    T ~ U[1,3]; BRT; CFL 0.8."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    reqs = []
    for i in range(count):
        T = float(rng.uniform(1.0, 3.0))
        if rng.uniform() < 0.7:
            n = [int(x) for x in rng.integers(40, 81, size=3)]
            v, w, r = float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.3, 1.2))
            g = GridSpec(n, [-4.0, -4.0, -PI], [4.0, 4.0, PI], [0, 0, 1])
            d = DynSpec(DYN_DUBINS3D, [v, w], MAXIMISE, MINIMISE)
            spec = SolveSpec(g, d, [0.0, T], rk_order=1, cfl=0.8, mode=BRT, radius=r, name=f"req{i}_3d")
        else:
            n = [int(x) for x in rng.integers(40, 65, size=4)]
            a, w, r = float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.3, 1.2))
            g = GridSpec(n, [-5.0, -5.0, 0.0, -PI], [5.0, 5.0, 4.0, PI], [0, 0, 0, 1])
            d = DynSpec(DYN_DYNCAR4D, [a, w], MAXIMISE, MINIMISE)
            spec = SolveSpec(g, d, [0.0, T], rk_order=3, cfl=0.8, mode=BRT, radius=r, name=f"req{i}_4d")
        reqs.append(Request(float(t[i]), spec))
    return reqs


def single_integrator(ndim: int, n: int, u_max: float, drift: Sequence[float], mode: int,
                      T: float, radius=1.5, periodic=False, L=4.0, rk_order=1, cfl=0.8,
                      brt=False, target="norm") -> SolveSpec:
    """Test-only N-D single integrator z' = c + u, |u| <= u_max on [-L, L]^N."""
    g = GridSpec([n] * ndim, [-L] * ndim, [L] * ndim, [1 if periodic else 0] * ndim)
    p = [u_max] + list(drift) + [0.0] * (ndim - len(drift))
    d = DynSpec(DYN_SINGLE_INTEGRATOR, p, mode, MINIMISE)
    return SolveSpec(g, d, [0.0, T], rk_order=rk_order, cfl=cfl, mode=BRT if brt else BRS,
                     radius=radius, target=target, name=f"si{ndim}d")
