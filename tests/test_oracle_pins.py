"""Pins for the float64 CPU oracle: results fixed by the mathematics, not by
the oracle's own formulas.

Each pin names what a plausible mistake would break:
  1  Hopf-Lax closed form for z' = c + u, |u| <= u_max (H, LF sign, ghosts,
     dt landing), both optimiser roles, with and without drift, 1-3D.
  2  exact discrete identities: the scheme reduces to textbook upwinding for
     pure advection (derivative indexing, LF sign, alpha); a one-cell shift
     at CFL 1 on a periodic axis; the Dubins x-axis on its th = 0 slice.
  3  tube monotonicity V(tau_k) <= V(tau_{k-1}), V <= V0, V(0) = V0.
  4  symmetries of the Dubins / car / two-car problems: mirror, quarter turn,
     heading roll (axis strides, periodic wrap, cos/sin placement).
  5  6D game with an evader-only target equals the 3D Dubins solve broadcast
     over the pursuer axes (and the pursuer-only mirror case), bitwise.
  6  4D car with a_max = 0: every v-slice is a 3D Dubins solve with v = v_k.
  7  first-order convergence of pin 1 under grid refinement.
  8  temporal order 1/2/3 of TVD-RK1/2/3 on a linear problem.
  9  computation methods (the paper's table): on a periodic advection at CFL
     1 each step is an exact one-cell shift, so every method has a closed
     form by direct recursion (V <- op(shift(V), reference)): running minima
     / maxima over time (the V^n reference), min / max with V0 or a target
     array, min / max with an obstacle array, and reach-avoid (target first,
     then obstacle); plus equivalences (target = V0 gives the V0 methods).
  -  hand-derived CFL steps of the three single-solve workloads (golden file).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2204_05520_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _grid_coords(g):
    return np.meshgrid(*[g.axis(d) for d in range(g.ndim)], indexing="ij")


# ------------------------------------------------------------------ pin 1

def hopf_lax(g, c, u_max, T, r, maximise):
    Z = _grid_coords(g)
    s = np.sqrt(sum((Z[d] + c[d] * T) ** 2 for d in range(g.ndim)))
    if maximise:
        return s + u_max * T - r
    return np.maximum(s - u_max * T, 0.0) - r


CASES_PIN1 = [
    # ndim, n, drift, maximise, brt
    (1, 161, [0.0], False, False),
    (1, 161, [0.6], False, True),
    (1, 161, [-0.4], True, False),
    (2, 81, [0.0, 0.0], False, False),
    (2, 81, [0.5, -0.3], False, True),
    (2, 81, [0.3, 0.4], True, False),
    (3, 41, [0.2, -0.3, 0.4], False, True),
    (3, 41, [0.0, 0.0, 0.0], True, False),
]


@pytest.mark.parametrize("ndim,n,drift,maximise,brt", CASES_PIN1)
def test_pin1_hopf_lax(oracle_mod, ndim, n, drift, maximise, brt):
    T, r, u_max = 0.5, 1.5, 1.0
    spec = W.single_integrator(ndim, n, u_max, drift, W.MAXIMISE if maximise else W.MINIMISE,
                               T, radius=r, brt=brt)
    V0 = W.make_v0(spec)
    res = oracle_mod.solve_spec(spec, V0)
    exact = hopf_lax(spec.grid, drift, u_max, T, r, maximise)
    band = np.abs(exact) <= 0.5
    dx = 8.0 / (n - 1)
    err = np.abs(res.V - exact)[band].max()
    # first-order scheme: error a fraction of dx in the smooth band; in 1D
    # the exact solution is piecewise linear and the scheme keeps it exactly
    # away from the kinks
    assert err <= (1e-6 if ndim == 1 else 0.75) * dx, (err, dx)
    # the whole grid (kinks included) stays within a few cells
    assert np.abs(res.V - exact).max() <= 2.5 * dx
    assert res.dt_first > 0 and math.isclose(res.dt_min, res.dt_min)


def test_pin1_wrong_sign_would_fail(oracle_mod):
    """The closed form separates maximiser and minimiser by 2 u_max T = 1."""
    spec = W.single_integrator(2, 81, 1.0, [0.0, 0.0], W.MINIMISE, 0.5)
    res = oracle_mod.solve_spec(spec)
    wrong = hopf_lax(spec.grid, [0, 0], 1.0, 0.5, 1.5, True)
    band = np.abs(wrong) <= 0.5
    assert np.abs(res.V - wrong)[band].max() > 0.5


# ----------------------------------------------------------------- pin 1b

def _arc_extreme(V0fun, x, half, maximise, periodic=True, samples=4001):
    """Hopf-Lax for x' = u, |u| <= b along one axis: the max (or min) of V0
    over [x - half, x + half], by dense sampling."""
    s = np.linspace(-half, half, samples)
    vals = V0fun(x[:, None] + s[None, :])
    return vals.max(axis=1) if maximise else vals.min(axis=1)


def _one_axis_case(dyn_id, axis, bound_index, role):
    """A target that depends on a single input axis: the other axes' terms
    vanish, and the input axis follows x' = u, |u| <= bound."""
    if dyn_id == W.DYN_DUBINS3D:
        spec = W.config_dubins3d(n=(5, 5, 96), T=0.5)
        spec.dyn = W.DynSpec(dyn_id, [0.7, 1.3], role, W.MINIMISE)
    elif dyn_id == W.DYN_DYNCAR4D:
        n = [5, 5, 5, 96] if axis == 3 else [5, 5, 161, 6]
        spec = W.config_dyncar4d(n=n, T=0.5)
        spec.dyn = W.DynSpec(dyn_id, [0.9, 1.3], role, W.MINIMISE)
    else:
        n = [4, 4, 96, 4, 4, 6] if axis == 2 else [4, 4, 6, 4, 4, 96]
        spec = W.config_game6d(n=n, T=0.5)
        spec.dyn = W.DynSpec(dyn_id, [0.6, 1.3, 0.8, 0.9],
                             role if axis == 2 else W.MAXIMISE,
                             role if axis == 5 else W.MAXIMISE)
    return spec


ONE_AXIS = [
    # dynamics, input axis, index of its bound in params, role
    (W.DYN_DUBINS3D, 2, 1, W.MAXIMISE), (W.DYN_DUBINS3D, 2, 1, W.MINIMISE),
    (W.DYN_DYNCAR4D, 3, 1, W.MAXIMISE), (W.DYN_DYNCAR4D, 3, 1, W.MINIMISE),
    (W.DYN_DYNCAR4D, 2, 0, W.MAXIMISE), (W.DYN_DYNCAR4D, 2, 0, W.MINIMISE),
    (W.DYN_TWODUBINS6D, 2, 1, W.MAXIMISE), (W.DYN_TWODUBINS6D, 2, 1, W.MINIMISE),
    (W.DYN_TWODUBINS6D, 5, 3, W.MAXIMISE), (W.DYN_TWODUBINS6D, 5, 3, W.MINIMISE),
]


@pytest.mark.parametrize("dyn_id,axis,bidx,role", ONE_AXIS)
def test_pin1b_bang_bang_axis_closed_form(oracle_mod, dyn_id, axis, bidx, role):
    spec = _one_axis_case(dyn_id, axis, bidx, role)
    g = spec.grid
    b = spec.dyn.params[bidx]
    T = spec.tau[-1]
    x = g.axis(axis)
    if g.periodic[axis]:
        f = lambda th: np.cos(th) + 0.4 * np.sin(2 * th)
    else:
        f = lambda v: 0.3 * (v - 2.0) ** 2 + 0.2 * v
    shape = [1] * g.ndim
    shape[axis] = g.n[axis]
    V0 = np.ascontiguousarray(np.broadcast_to(f(x).reshape(shape), tuple(g.n)))
    res = oracle_mod.solve(g, spec.dyn, V0, spec.tau, rk_order=1, cfl=0.8, brt=False)
    exact = _arc_extreme(f, x, b * T, role == W.MAXIMISE)
    got = np.moveaxis(res.V, axis, -1).reshape(-1, g.n[axis])
    # the result is constant across the other axes
    assert np.abs(got - got[0]).max() < 1e-12
    h = x[1] - x[0]
    keep = np.ones(x.size, dtype=bool)
    if not g.periodic[axis]:
        # stay away from the edges, where the exact solution looks past them
        keep = (x - b * T > g.lo[axis] + 4 * h) & (x + b * T < g.hi[axis] - 4 * h)
    err = np.abs(got[0] - exact)[keep].max()
    assert err < 1.5 * h, (err, h)
    # the other role is far away: the pin separates maximiser and minimiser
    other = _arc_extreme(f, x, b * T, role != W.MAXIMISE)
    assert np.abs(got[0] - other)[keep].max() > 10 * h


# ------------------------------------------------------------------ pin 2

def test_pin2_periodic_shift_at_cfl_one(oracle_mod):
    g = W.GridSpec([40], [-4.0], [4.0], [1])
    x = g.axis(0)
    V0 = np.sin(2 * np.pi * x / 8) + 0.3 * np.cos(6 * np.pi * x / 8) + 0.1 * x ** 0
    for c in (0.7, -0.45):
        d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, c], W.MINIMISE, W.MINIMISE)
        _, dt = oracle_mod.cfl_dt(g, d, 1.0)
        assert math.isclose(dt, 0.2 / abs(c), rel_tol=1e-15)
        res = oracle_mod.solve(g, d, V0, [0.0, 5 * dt], rk_order=1, cfl=1.0, brt=False)
        # V_tau = c V_x: c > 0 moves data towards -x by one cell per step
        shift = -5 if c > 0 else 5
        assert np.abs(res.V - np.roll(V0, shift)).max() < 1e-13


@pytest.mark.parametrize("c,cfl", [(0.8, 0.5), (-1.3, 0.9), (0.25, 0.3)])
def test_pin2_upwind_identity(oracle_mod, c, cfl):
    g = W.GridSpec([33], [-4.0], [4.0], [1])
    x = g.axis(0)
    rng = np.random.default_rng(7)
    V0 = np.cos(x) + 0.05 * rng.standard_normal(x.size)
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, c], W.MAXIMISE, W.MINIMISE)
    _, dt = oracle_mod.cfl_dt(g, d, cfl)
    res = oracle_mod.solve(g, d, V0, [0.0, dt], rk_order=1, cfl=cfl, brt=False)
    lam = abs(c) * dt / (8.0 / 33)
    assert math.isclose(lam, cfl, rel_tol=1e-14)
    if c > 0:
        expect = V0 + lam * (np.roll(V0, -1) - V0)
    else:
        expect = V0 + lam * (np.roll(V0, 1) - V0)
    assert np.abs(res.V - expect).max() < 1e-14


def test_pin2_dubins_x_axis_slice(oracle_mod):
    """w_max = 0: on the th = 0 slice (cos 1, sin ~0, local alpha_y ~0) the
    Dubins update is exactly upwinding along x with lambda = v dt / dx."""
    n = (30, 20, 16)
    spec = W.config_dubins3d(n=n)
    spec.dyn.params = [1.0, 0.0]
    V0 = W.make_v0(spec)
    amax, dt = oracle_mod.cfl_dt(spec.grid, spec.dyn, 0.8)
    res = oracle_mod.solve(spec.grid, spec.dyn, V0, [0.0, dt], rk_order=1, cfl=0.8, brt=False)
    k0 = n[2] // 2
    assert abs(spec.grid.axis(2)[k0]) < 1e-15
    lam = dt / (8.0 / 29)
    S0 = V0[:, :, k0]
    expect = S0[:-1] + lam * (S0[1:] - S0[:-1])
    assert np.abs(res.V[:-1, :, k0] - expect).max() < 1e-14


# ------------------------------------------------------------------ pin 3

@pytest.mark.parametrize("which,rk", [("dubins3d", 1), ("dubins3d", 2), ("dyncar4d", 3),
                                      ("game6d", 2)])
def test_pin3_brt_monotone(oracle_mod, which, rk):
    if which == "dubins3d":
        spec = W.config_dubins3d(n=(24, 24, 16), T=0.6)
    elif which == "dyncar4d":
        spec = W.config_dyncar4d(n=12, T=0.3)
    else:
        spec = W.config_game6d(n=[8, 8, 6, 7, 7, 6], T=0.3)
    _, dt = oracle_mod.cfl_dt(spec.grid, spec.dyn, spec.cfl)
    m = int(spec.tau[-1] / dt)
    tau = [k * dt for k in range(m + 1)]
    V0 = W.make_v0(spec)
    res = oracle_mod.solve(spec.grid, spec.dyn, V0, tau, rk_order=rk, cfl=spec.cfl, brt=True,
                           save_all=True)
    A = res.V_all
    assert np.array_equal(A[0], V0)
    assert (A <= V0[None] + 0.0).all()
    tol = 4 * np.finfo(np.float64).eps * np.maximum(np.abs(A[:-1]), 1.0)
    ok = A[1:] <= A[:-1] + tol
    # The order-preserving argument covers the interior; the sign-keeping
    # ghost extrapolation is not monotone in the inner node, so faces of
    # non-periodic axes are only required to stay close.
    g = spec.grid
    inner = np.ones(tuple(g.n), dtype=bool)
    for d in range(g.ndim):
        if not g.periodic[d]:
            sl = [slice(None)] * g.ndim
            sl[d] = [0, g.n[d] - 1]
            inner[tuple(sl)] = False
    assert ok[:, inner].all()
    assert (A[1:] - A[:-1]).max() < 1e-3
    # the tube grows: some point strictly decreased
    assert (A[-1] < V0 - 1e-6).any()


# ------------------------------------------------------------------ pin 4

def _solve(oracle_mod, spec, V0=None, **kw):
    V0 = W.make_v0(spec) if V0 is None else V0
    return oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order,
                            cfl=spec.cfl, brt=spec.mode == W.BRT, **kw).V


def test_pin4_dubins_symmetries(oracle_mod):
    spec = W.config_dubins3d(n=(21, 21, 16), T=0.5)
    V = _solve(oracle_mod, spec)
    n = 16
    # mirror (x, y, th) -> (x, -y, -th)
    kk = (n - np.arange(n)) % n
    Vm = V[:, ::-1, :][:, :, kk]
    assert np.abs(Vm - V).max() < 1e-12
    # quarter turn (x, y, th) -> (-y, x, th + pi/2): V[n-1-j, i, k+n/4] = V[i, j, k]
    Vr = np.empty_like(V)
    for i in range(21):
        for j in range(21):
            Vr[i, j, :] = np.roll(V[20 - j, i, :], -n // 4)
    assert np.abs(Vr - V).max() < 1e-12
    # heading roll: shift the th origin by 3 cells
    h = 2 * np.pi / n
    spec2 = W.config_dubins3d(n=(21, 21, 16), T=0.5)
    spec2.grid.lo[2] = -np.pi + 3 * h
    spec2.grid.hi[2] = np.pi + 3 * h
    V2 = _solve(oracle_mod, spec2)
    assert np.abs(V2 - np.roll(V, -3, axis=2)).max() < 1e-12


def test_pin4_symmetry_breaks_on_swapped_axes(oracle_mod):
    """Control for pin 4: exchanging the roles of x and y (cos on y) is not
    mirror-symmetric, so the mirror check does catch such a mistake."""
    spec = W.config_dubins3d(n=(21, 21, 16), T=0.5)
    V = _solve(oracle_mod, spec)
    Vt = np.transpose(V, (1, 0, 2))  # a solution with x and y exchanged
    kk = (16 - np.arange(16)) % 16
    assert np.abs(Vt[:, ::-1, :][:, :, kk] - Vt).max() > 1e-3


def test_pin4_car_and_game_mirror(oracle_mod):
    spec = W.config_dyncar4d(n=[15, 15, 6, 12], T=0.3)
    V = _solve(oracle_mod, spec)
    kk = (12 - np.arange(12)) % 12
    Vm = V[:, ::-1, :, :][:, :, :, kk]
    assert np.abs(Vm - V).max() < 1e-12

    spec = W.config_game6d(n=[7, 7, 6, 7, 7, 6], T=0.2)
    V = _solve(oracle_mod, spec)
    kk = (6 - np.arange(6)) % 6
    Vm = V[:, ::-1, :, :, ::-1, :][:, :, kk, :, :, :][:, :, :, :, :, kk]
    assert np.abs(Vm - V).max() < 1e-12


# ------------------------------------------------------------------ pin 5

@pytest.mark.parametrize("player", ["evader", "pursuer"])
def test_pin5_game_separates(oracle_mod, player):
    n6 = [11, 10, 8, 6, 5, 6]
    spec6 = W.config_game6d(n=n6, T=0.4)
    _, dt6 = oracle_mod.cfl_dt(spec6.grid, spec6.dyn, spec6.cfl)
    if player == "evader":
        keep, n3, mode, v, w = (0, 1), n6[:3], spec6.dyn.u_mode, 1.0, 1.0
        V0 = W.cylinder_v0(spec6.grid, 0.7, keep=(0, 1))
    else:
        keep, n3, mode, v, w = (3, 4), n6[3:], spec6.dyn.d_mode, 1.0, 1.0
        V0 = W.cylinder_v0(spec6.grid, 0.7, keep=(3, 4))
    V6 = oracle_mod.solve(spec6.grid, spec6.dyn, V0, spec6.tau, rk_order=2, cfl=0.8,
                          brt=True).V
    spec3 = W.config_dubins3d(n=n3, T=0.4)
    spec3.dyn = W.DynSpec(W.DYN_DUBINS3D, [v, w], mode, W.MINIMISE)
    V03 = W.cylinder_v0(spec3.grid, 0.7, keep=(0, 1))
    V3 = oracle_mod.solve(spec3.grid, spec3.dyn, V03, spec3.tau, rk_order=2, cfl=0.8,
                          brt=True, max_dt=dt6).V
    if player == "evader":
        ref = np.broadcast_to(V3[:, :, :, None, None, None], V6.shape)
    else:
        ref = np.broadcast_to(V3[None, None, None, :, :, :], V6.shape)
    assert np.array_equal(V6, ref)


# ------------------------------------------------------------------ pin 6

def test_pin6_car_reduces_to_dubins(oracle_mod):
    spec4 = W.config_dyncar4d(n=[14, 13, 5, 12], T=0.25)
    spec4.dyn.params = [0.0, 1.0]  # a_max = 0
    V0 = W.make_v0(spec4)
    _, dt4 = oracle_mod.cfl_dt(spec4.grid, spec4.dyn, spec4.cfl)
    V4 = oracle_mod.solve(spec4.grid, spec4.dyn, V0, spec4.tau, rk_order=3, cfl=0.8,
                          brt=True).V
    g4 = spec4.grid
    for k, vk in enumerate(g4.axis(2)):
        g3 = W.GridSpec([14, 13, 12], [-5.0, -5.0, -np.pi], [5.0, 5.0, np.pi], [0, 0, 1])
        d3 = W.DynSpec(W.DYN_DUBINS3D, [float(vk), 1.0], W.MAXIMISE, W.MINIMISE)
        V03 = W.cylinder_v0(g3, 0.5)
        V3 = oracle_mod.solve(g3, d3, V03, spec4.tau, rk_order=3, cfl=0.8, brt=True,
                              max_dt=dt4).V
        assert np.array_equal(V4[:, :, k, :], V3), k


# ------------------------------------------------------------------ pin 7

def test_pin7_first_order_convergence(oracle_mod):
    errs, hs = [], []
    for n in (26, 51, 101):
        spec = W.single_integrator(2, n, 1.0, [0.3, -0.2], W.MINIMISE, 0.5, brt=True)
        res = oracle_mod.solve_spec(spec)
        exact = hopf_lax(spec.grid, [0.3, -0.2], 1.0, 0.5, 1.5, False)
        band = np.abs(exact) <= 0.5
        errs.append(np.abs(res.V - exact)[band].max())
        hs.append(8.0 / (n - 1))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(2)]
    for p in orders:
        assert 0.7 <= p <= 1.3, (orders, errs)


# ------------------------------------------------------------------ pin 8

@pytest.mark.parametrize("rk", [1, 2, 3])
def test_pin8_rk_temporal_order(oracle_mod, rk):
    g = W.GridSpec([48], [0.0], [8.0], [1])
    x = g.axis(0)
    V0 = np.sin(2 * np.pi * x / 8.0)
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, 1.0], W.MAXIMISE, W.MINIMISE)
    T = 1.0
    dx = 8.0 / 48

    def run(m):
        return oracle_mod.solve(g, d, V0, [0.0, T], rk_order=rk, cfl=1.0, brt=False,
                                max_dt=T / m).V

    m0 = int(math.ceil(T / (0.5 * dx)))
    ref = run(m0 * 64)
    e = [np.abs(run(m0 * f) - ref).max() for f in (1, 2, 4)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    for r_ in rates:
        assert abs(r_ - rk) < 0.25, (rates, e)


# ------------------------------------------------------------------ pin 10
# Second-order ENO differences (the Spatial Derivatives subsection's ENO2).

def _drift_1d(n, lo=-2.0, hi=2.0, c=0.7, periodic=0):
    g = W.GridSpec([n], [lo], [hi], [periodic])
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, c], W.MAXIMISE, W.MINIMISE)
    return g, d


@pytest.mark.parametrize("ndim", [1, 3])
def test_pin10_eno2_exact_on_quadratics(oracle_mod, ndim):
    """ENO2 one-sided differences of a quadratic are its exact derivative, so
    with the drift-only Hamiltonian H = c . p the LF term vanishes and one
    step is V + dt c . grad q at every node two or more nodes from an edge.
    First-order differences miss this by dt |c_d| q_d'' dx_d / 2."""
    n = [23, 17, 19][:ndim]
    lo, hi = [-2.0, -1.0, 0.5][:ndim], [2.0, 1.5, 3.0][:ndim]
    cs = [0.7, -0.4, 0.25][:ndim]
    qa, qb = [0.8, -1.3, 0.5][:ndim], [0.3, 0.1, -0.7][:ndim]
    g = W.GridSpec(n, lo, hi, [0] * ndim)
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0] + cs, W.MAXIMISE, W.MINIMISE)
    ax = [g.axis(k) for k in range(ndim)]
    mesh = np.meshgrid(*ax, indexing="ij")
    V = sum(qa[k] * mesh[k] ** 2 + qb[k] * mesh[k] for k in range(ndim))
    grad_c = sum(cs[k] * (2 * qa[k] * mesh[k] + qb[k]) for k in range(ndim))
    inner = np.ones(V.shape, bool)
    for k in range(ndim):
        sl = [slice(None)] * ndim
        for e in (0, 1, -1, -2):
            sl[k] = e
            inner[tuple(sl)] = False
    idx = np.flatnonzero(inner.reshape(-1))
    dt = 0.01
    got = oracle_mod.step_at(g, d, V, V, dt, idx, brt=False, space_order=2)
    expect = (V + dt * grad_c).reshape(-1)[idx]
    assert np.abs(got - expect).max() < 1e-12
    first = oracle_mod.step_at(g, d, V, V, dt, idx, brt=False, space_order=1)
    assert np.abs(first - expect).max() > 1e-4


def test_pin10_eno2_picks_the_smooth_side(oracle_mod):
    """V = |x - x_k| with the kink on node k: away from the kink ENO2 takes
    the stencil that does not cross it, so both one-sided differences equal
    the exact slope +-1 and a drift step moves V by dt c sgn(x - x_k); on
    the kink node p- = -1, p+ = +1 and the step adds dt |c| (LF term)."""
    n, k = 41, 17
    for c in (0.7, -0.45):
        g, d = _drift_1d(n, c=c)
        x = g.axis(0)
        V = np.abs(x - x[k])
        idx = np.arange(2, n - 2)
        dt = 0.02
        got = oracle_mod.step_at(g, d, V, V, dt, idx, brt=False, space_order=2)
        expect = V[idx] + dt * c * np.sign(x[idx] - x[k])
        expect[idx == k] = V[k] + dt * abs(c)
        assert np.abs(got - expect).max() < 1e-12, c


def test_pin10_eno2_tie_takes_the_first_stencil(oracle_mod):
    """Equal-magnitude second differences of opposite sign around node i:
    the reading takes the first candidate (the one nearer the upwind side of
    each one-sided difference)."""
    g, d = _drift_1d(11, lo=0.0, hi=10.0, c=1.0)
    V = np.zeros(11)
    i = 5
    V[i - 2], V[i - 1], V[i], V[i + 1], V[i + 2] = 0.0, 1.0, 0.0, 1.0, 2.0
    # at i: sm = (0-1)-(1-0) = -2, s0 = (1-0)-(0-1) = 2 (tie), sp = (2-1)-(1-0) = 0
    # p- = (dm + sm/2)/dx = (-1 - 1) = -2; p+ = (dp - s0/2)/dx... s0 vs sp: |2| > 0 -> sp
    # p+ = (1 - 0)/1 = 1; with c = 1: Hh = c pbar + |c|/2 (p+ - p-) = -0.5 + 1.5 = 1
    dt = 0.1
    got = oracle_mod.step_at(g, d, V, V, dt, [i], brt=False, space_order=2)
    assert abs(got[0] - (V[i] + dt * 1.0)) < 1e-14


def test_pin10_eno2_second_ghost(oracle_mod):
    """Beyond a non-periodic edge the m-th ghost is V_b + m sgn(V_b)|V_b - V_in|.
    V = 5 - x on [1, 3] (positive, decreasing): at the lower edge the ghosts
    continue the line (the data grows away from zero there), so every node
    but the last moves by the exact drift step -dt c; at the upper edge the
    ghosts turn back up (2.1, 2.2 after 2.0), the last node's p- picks the
    line (-1) and its p+ the two ghosts (+1: the stencil through the second
    ghost is the straight one), so it moves by dt |c| (the LF term)."""
    for c in (0.6, -0.6):
        g, d = _drift_1d(21, lo=1.0, hi=3.0, c=c)
        x = g.axis(0)
        V = 5.0 - x
        dt = 0.01
        got = oracle_mod.step_at(g, d, V, V, dt, np.arange(21), brt=False, space_order=2)
        expect = V - dt * c
        expect[-1] = V[-1] + dt * abs(c)
        assert np.abs(got - expect).max() < 1e-12, c


def test_pin10_eno2_rk2_second_order_convergence(oracle_mod):
    """Periodic advection of a smooth profile with ENO2 + TVD-RK2 (the
    paper's second-order row) converges at second order; first order at
    first order."""
    def err(n, order):
        g, d = _drift_1d(n, lo=0.0, hi=8.0, c=1.0, periodic=1)
        x = g.axis(0)
        V0 = np.sin(2 * np.pi * x / 8.0) + 0.5 * np.cos(4 * np.pi * x / 8.0)
        T = 2.0
        res = oracle_mod.solve(g, d, V0, [0.0, T], rk_order=2, cfl=0.5, brt=False,
                               space_order=order)
        xe = x + T   # z' = c + u: the profile moves by -c T in tau (V(z) = V0(z + c tau))
        exact = np.sin(2 * np.pi * xe / 8.0) + 0.5 * np.cos(4 * np.pi * xe / 8.0)
        return np.abs(res.V - exact).mean()
    for order, lo_, hi_ in ((2, 1.7, 2.4), (1, 0.7, 1.3)):
        e = [err(n, order) for n in (64, 128, 256)]
        rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        for r_ in rates:
            assert lo_ <= r_ <= hi_, (order, rates, e)


# ------------------------------------------------------------------ pin 11
# Relative pursuit-evasion (the paper's main example) and the costate box.

def _pe3d_f(z, a, b, va=1.0, vb=1.0):
    """The paper's relative dynamics, for brute-force checks."""
    x, y, th = z
    return np.array([-va + vb * np.cos(th) + a * y, vb * np.sin(th) - a * x, b - a])


def test_pin11_pe3d_hamiltonian_is_max_min(oracle_mod):
    """H(z, p) = max over the evader's a in {-A, A} of min over the pursuer's
    b in {-B, B} of p . f(z, a, b) (the game's Hamiltonian; bang-bang inputs
    reach the extremes of an affine function)."""
    rng = np.random.default_rng(11)
    d = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 0.8, 1.3], W.MAXIMISE, W.MINIMISE)
    z = np.column_stack([rng.uniform(-4, 4, 400), rng.uniform(-4, 4, 400), rng.uniform(-np.pi, np.pi, 400)])
    p = rng.standard_normal((400, 3))
    H = oracle_mod.hamiltonian(d, 3, z, p)
    for j in range(400):
        best = max(min(p[j] @ _pe3d_f(z[j], a, b) for b in (-1.3, 1.3)) for a in (-0.8, 0.8))
        assert abs(H[j] - best) < 1e-12, j
    # the roles swapped: the evader minimises, the pursuer maximises
    d2 = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 0.8, 1.3], W.MINIMISE, W.MAXIMISE)
    H2 = oracle_mod.hamiltonian(d2, 3, z, p)
    for j in range(0, 400, 7):
        best = min(max(p[j] @ _pe3d_f(z[j], a, b) for b in (-1.3, 1.3)) for a in (-0.8, 0.8))
        assert abs(H2[j] - best) < 1e-12, j


def test_pin11_alpha_box_brute_force(oracle_mod):
    """alpha_d over the costate box equals its definition, the largest
    |f_d(z, a*(p), b*(p))| over p in the box, found by brute force on a dense
    sample of the box; for Dubins, the 4D car and the 6D game the box gives
    the all-inputs alpha (every input drives one axis at its bound)."""
    rng = np.random.default_rng(5)
    d = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)
    ticks = np.linspace(0.0, 1.0, 25)
    smaller = 0
    for case in range(80):
        lo = rng.uniform(-1.0, 0.6, 3)
        hi = lo + rng.uniform(0.05, 1.5, 3)
        # half of the states near the origin, where the p_th term decides
        # the evader's switching function and the split of the box on the
        # sign of p_th (the pursuer's) matters
        r = 4.0 if case < 40 else 0.25
        z = np.array([rng.uniform(-r, r), rng.uniform(-r, r), rng.uniform(-np.pi, np.pi)])
        ab, aa = oracle_mod.alpha_box(d, 3, z, lo, hi)
        P = np.stack(np.meshgrid(*[lo[k] + ticks * (hi[k] - lo[k]) for k in range(3)],
                                 indexing="ij"), -1).reshape(-1, 3)
        if lo[2] < 0 < hi[2]:
            P = np.vstack([P, np.column_stack([P[:, 0], P[:, 1], np.zeros(len(P))])])
        s_a = P[:, 0] * z[1] - P[:, 1] * z[0] - P[:, 2]
        a = np.where(s_a >= 0, 1.0, -1.0)
        b = np.where(P[:, 2] >= 0, -1.0, 1.0)
        F = np.abs(np.stack([-1 + np.cos(z[2]) + a * z[1], np.sin(z[2]) - a * z[0], b - a], 1))
        brute = F.max(0)
        assert np.abs(ab[0] - brute).max() < 1e-12, (case, ab, brute, lo, hi, z)
        assert np.all(ab[0] <= aa[0] + 1e-15)
        smaller += int(np.any(ab[0] < aa[0] - 1e-9))
    assert smaller >= 5  # the box matters for this game
    for dyn, nd in ((W.DynSpec(W.DYN_DUBINS3D, [1.0, 1.3], W.MAXIMISE, W.MINIMISE), 3),
                    (W.DynSpec(W.DYN_DYNCAR4D, [0.7, 1.1], W.MAXIMISE, W.MINIMISE), 4),
                    (W.DynSpec(W.DYN_TWODUBINS6D, [1.0, 1.2, 0.9, 0.8], W.MAXIMISE, W.MINIMISE), 6)):
        for case in range(20):
            lo = rng.uniform(-1.0, 0.6, nd)
            hi = lo + rng.uniform(0.05, 1.5, nd)
            z = rng.uniform(-3, 3, nd)
            ab, aa = oracle_mod.alpha_box(dyn, nd, z, lo, hi)
            assert np.array_equal(ab, aa)


def test_pin11_pe3d_without_turning_is_drift(oracle_mod):
    """With both turn bounds 0 the game is a drift (-v_a + v_b cos th,
    v_b sin th, 0): every heading slice is a 2D drift solve with that
    velocity (same step sizes)."""
    ns = [21, 19, 12]
    g = W.GridSpec(ns, [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_PE3D, [0.7, 1.2, 0.0, 0.0], W.MAXIMISE, W.MINIMISE)
    V0 = W.cylinder_v0(g, 1.0)
    tau = [0.0, 0.6]
    res = oracle_mod.solve(g, d, V0, tau, rk_order=2, cfl=0.8, brt=True, max_dt=0.04)
    g2 = W.GridSpec(ns[:2], [-4.0, -4.0], [4.0, 4.0], [0, 0])
    th = g.axis(2)
    for k in (0, 3, 7, 11):
        d2 = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, -0.7 + 1.2 * np.cos(th[k]), 1.2 * np.sin(th[k])],
                       W.MAXIMISE, W.MINIMISE)
        r2 = oracle_mod.solve(g2, d2, V0[:, :, k], tau, rk_order=2, cfl=0.8, brt=True, max_dt=0.04)
        assert r2.steps == res.steps
        assert np.abs(r2.V - res.V[:, :, k]).max() < 1e-12, k


def test_pin11_pe3d_one_step_with_known_box(oracle_mod):
    """V = x + c |y - y0| (kink on the node row y = y0): pbar = (1, +-c or 0,
    0) everywhere, edges included, so the costate box is {1} x [-c, c] x {0}.
    One step at every node off the y edges, written out from Algorithm 1:
    H = pbar . f with the optimal inputs, plus the LF term, which only the
    kink row has (p+_y - p-_y = 2c) with alpha_y from the box: the pursuer's
    b = -B (p_th = 0), the evader's a = +A always and a = -A only where
    y0 - c |x| < 0."""
    c, y0, A, B, dt = 0.3, 0.5, 1.0, 1.0, 0.01
    g = W.GridSpec([33, 17, 12], [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, A, B], W.MAXIMISE, W.MINIMISE)
    x, y, th = (g.axis(k) for k in range(3))
    X, Y, TH = np.meshgrid(x, y, th, indexing="ij")
    V = X + c * np.abs(Y - y0)
    rows = np.arange(1, 16)
    idx = np.ravel_multi_index(np.meshgrid(np.arange(33), rows, np.arange(12), indexing="ij"),
                               (33, 17, 12)).reshape(-1)
    got = oracle_mod.step_at(g, d, V, V, dt, idx, brt=False)
    Xs, Ys, Ts = X.reshape(-1)[idx], Y.reshape(-1)[idx], TH.reshape(-1)[idx]
    kink = np.abs(Ys - y0) < 1e-12
    py = np.where(kink, 0.0, c * np.sign(Ys - y0))
    a = np.where(Ys - py * Xs >= 0, A, -A)
    H = (-1.0 + np.cos(Ts) + a * Ys) + py * (np.sin(Ts) - a * Xs)
    both = y0 - c * np.abs(Xs) < 0
    alpha_y = np.where(both, np.abs(np.sin(Ts)) + A * np.abs(Xs), np.abs(np.sin(Ts) - A * Xs))
    expect = V.reshape(-1)[idx] + dt * (H + np.where(kink, alpha_y * c, 0.0))
    assert np.abs(got - expect).max() < 1e-12
    # the all-inputs alpha would differ on the kink row
    assert np.any(kink & ~both & (np.abs(np.sin(Ts) - A * Xs) < np.abs(np.sin(Ts)) + A * np.abs(Xs) - 1e-6))


def _narrow_box_case():
    g = W.GridSpec([33, 17, 12], [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)
    X, Y, _ = np.meshgrid(g.axis(0), g.axis(1), g.axis(2), indexing="ij")
    return g, d, X + 0.3 * np.abs(Y - 0.5)


def test_pin11_pe3d_cfl_step_from_the_box(oracle_mod):
    """Algorithm 1 takes the CFL step from alpha^max, the largest alpha_i of
    the dissipation loop, each alpha_i over the costate box.  Worked out by
    hand for V0 = x + 0.3 |y - 0.5| on 33 x 17 x 12 nodes over [-4,4]^2 x
    [-pi,pi): the box is {1} x [-0.3, 0.3] x {0} (edges included: a ghost
    keeps the edge node's sign, which leaves pbar_y in [-0.3, 0.3]).  The
    pursuer's switching function p_th is 0 (b = -B); the evader's, y - x p_y,
    ranges over [y - 0.3|x|, y + 0.3|x|], so rows with |y| > 0.3|x| realise
    only a = sign(y) A.  Then alpha_x = max |-1 + cos th + a y| = 4 (|y| = 4,
    th = 0), where all inputs give |-1 + cos pi| + 4 = 6; alpha_y = |sin th|
    + |x| = 5 (x = +-4 with both signs realised, th = +-pi/2); alpha_th =
    |b - a| = 2.  The first step is therefore 0.8 / (4/dx + 5/dy + 2/dth),
    1.27 times the all-inputs step, and a horizon of 8 all-inputs steps takes
    7 (the box stays narrow)."""
    g, d, V0 = _narrow_box_case()
    (dmin, dmax), amax = oracle_mod.box_alpha_max(g, d, V0)
    assert np.allclose(dmin, [1.0, -0.3, 0.0], atol=1e-12) and np.allclose(dmax, [1.0, 0.3, 0.0], atol=1e-12)
    assert np.abs(amax - [4.0, 5.0, 2.0]).max() < 1e-12
    all_inputs, dt_all = oracle_mod.cfl_dt(g, d, 0.8)
    assert np.abs(all_inputs - [6.0, 5.0, 2.0]).max() < 1e-12
    dx, dy, dth = 8.0 / 32, 8.0 / 16, 2 * np.pi / 12
    dt_box = 0.8 / (4.0 / dx + 5.0 / dy + 2.0 / dth)
    assert abs(dt_all - 0.8 / (6.0 / dx + 5.0 / dy + 2.0 / dth)) < 1e-15
    tau = [0.0, 8 * dt_all * (1 - 1e-12)]
    for rk in (1, 2):
        res = oracle_mod.solve(g, d, V0, tau, rk_order=rk, cfl=0.8, brt=False)
        assert abs(res.dt_first - dt_box) < 1e-15 * dt_box, (res.dt_first, dt_box)
        assert res.steps == 7, res.steps
    # the global-alpha approximation has no box: the all-inputs step
    res = oracle_mod.solve(g, d, V0, tau, rk_order=1, cfl=0.8, brt=False, global_alpha=True)
    assert abs(res.dt_first - dt_all) < 1e-15 * dt_all and res.steps == 8


def test_pin11_pe3d_capture_box_is_all_inputs(oracle_mod):
    """For the capture target (relative distance - 0.5) the costate box
    spans both signs of both switching functions at every node, so the box
    alpha equals the all-inputs alpha everywhere and the CFL step is the
    all-inputs step: pbar_x and pbar_y take both signs (the distance
    gradient points every way) and so does pbar_th after one step."""
    spec = W.config_pe3d(n=[23, 21, 16], T=0.5)
    V0 = W.make_v0(spec)
    all_inputs, dt_all = oracle_mod.cfl_dt(spec.grid, spec.dyn, spec.cfl)
    (dmin, dmax), amax = oracle_mod.box_alpha_max(spec.grid, spec.dyn, V0)
    assert dmin[0] < 0 < dmax[0] and dmin[1] < 0 < dmax[1]
    assert np.array_equal(amax, all_inputs)
    res = oracle_mod.solve_spec(spec)
    assert res.dt_max == dt_all


def test_pin11_pe3d_mirror_symmetry(oracle_mod):
    """(x, y, th) -> (x, -y, -th) with (a, b) -> (-a, -b) maps the game to
    itself and the capture target to itself, so the tube is symmetric."""
    spec = W.config_pe3d(n=[23, 21, 16], T=0.5)
    res = oracle_mod.solve_spec(spec)
    V = res.V
    k = (16 - np.arange(16)) % 16
    M = V[:, ::-1, :][:, :, k]
    assert np.abs(M - V).max() < 1e-12
    # and the solve is not trivial
    assert np.abs(V - W.make_v0(spec)).max() > 0.1


# ------------------------------------------------------------------ pin 12
# Time-to-reach by Lax-Friedrichs sweeping (Algorithm 2).

def _ball_ttr(nn, u_max=1.0, r=1.0):
    g = W.GridSpec([nn, nn], [-4.0, -4.0], [4.0, 4.0], [0, 0])
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [u_max, 0.0, 0.0], W.MINIMISE, W.MAXIMISE)
    return g, d, W.cylinder_v0(g, r)


def test_pin12_ttr_ball_closed_form_first_order(oracle_mod):
    """|u| <= u_max in 2D, disc target of radius 1: the time to reach is
    max(|z| - 1, 0) / u_max.  The sweeping solution converges to it at first
    order (max and mean error)."""
    errs = []
    for nn in (41, 81, 161):
        g, d, l = _ball_ttr(nn)
        r = oracle_mod.ttr_solve(g, d, l, eps=1e-10)
        assert r.change < 1e-10
        exact = np.maximum(l, 0.0)
        errs.append((np.abs(r.phi - exact).max(), np.abs(r.phi - exact).mean()))
        assert np.all(r.phi[l <= 0] == 0.0)
    for k in (0, 1):
        rates = [math.log2(errs[i][k] / errs[i + 1][k]) for i in range(2)]
        for rt in rates:
            assert 0.7 <= rt <= 1.3, (k, rates, errs)
    assert errs[-1][0] < 0.08


def test_pin12_ttr_speed_scaling(oracle_mod):
    """Doubling the speed bound halves the time to reach: every term of the
    update scales by a power of two, so the converged fields agree to the
    stopping tolerance."""
    g, d1, l = _ball_ttr(61, 1.0)
    _, d2, _ = _ball_ttr(61, 2.0)
    a = oracle_mod.ttr_solve(g, d1, l, eps=1e-11).phi
    b = oracle_mod.ttr_solve(g, d2, l, eps=1e-11).phi
    assert np.abs(b - 0.5 * a).max() < 1e-8


def test_pin12_ttr_monotone_in_target(oracle_mod):
    """A larger target is reached no later, node by node."""
    g, d, l1 = _ball_ttr(61, 1.0, r=1.0)
    l2 = W.cylinder_v0(g, 1.5)
    a = oracle_mod.ttr_solve(g, d, l1, eps=1e-10).phi
    b = oracle_mod.ttr_solve(g, d, l2, eps=1e-10).phi
    assert np.all(b <= a + 1e-9)
    assert np.abs(a - b).max() > 0.3


def test_pin12_ttr_iteration_orders(oracle_mod):
    """The Gauss-Seidel sweep and the parallel (Jacobi) iteration reach the
    same fixed point where the non-periodic edges are outflow edges with
    values growing outward (the 2D disc target); the parallel form takes
    more iterations and satisfies the same closed-form band."""
    g, d, l = _ball_ttr(61)
    a = oracle_mod.ttr_solve(g, d, l, eps=1e-12)
    b = oracle_mod.ttr_solve(g, d, l, eps=1e-12, jacobi=True)
    assert b.iters > a.iters
    assert np.abs(a.phi - b.phi).max() < 1e-9
    exact = np.maximum(l, 0.0)
    assert np.abs(b.phi - exact).max() < 0.25


def test_pin12_ttr_dubins_straight_ahead(oracle_mod):
    """Dubins car (v = 1, |w| <= 1, time-minimising turn), disc target of
    radius 1: from a state on the x axis heading straight at the target the
    time to reach is (|x| - 1) / v; the sweeping solution sits within a
    first-order band of it, and no state is reached faster than its
    straight-line distance allows."""
    g = W.GridSpec([41, 41, 32], [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_DUBINS3D, [1.0, 1.0], W.MINIMISE, W.MAXIMISE)
    l = W.cylinder_v0(g, 1.0)
    r = oracle_mod.ttr_solve(g, d, l, eps=1e-9)
    x = g.axis(0)
    # heading pi (index 0: -pi) from x > 1 on y = 0 drives straight at the target
    j0 = 20
    sel = (x > 1.2) & (x < 3.6)
    got = r.phi[sel, j0, 0]
    exact = x[sel] - 1.0
    assert np.abs(got - exact).max() < 0.2, np.abs(got - exact).max()
    assert np.all(r.phi >= np.maximum(l, 0.0) - 1e-9)


# ------------------------------------------------------------------ golden

def test_golden_cfl_steps(oracle_mod):
    gold = json.load(open(os.path.join(HERE, "golden", "cfl_steps.json")))
    # the full 36^6 reduction is too slow for a plain CPU loop; the reduced
    # game grid keeps the heading axes and therefore alpha^max
    specs = {"dubins3d_60x60x36": W.config_dubins3d(),
             "dyncar4d_80": W.config_dyncar4d(),
             "game6d_8x8x36x8x8x36": W.config_game6d(n=[8, 8, 36, 8, 8, 36])}
    for key, spec in specs.items():
        amax, dt = oracle_mod.cfl_dt(spec.grid, spec.dyn, spec.cfl)
        assert np.allclose(amax, gold[key]["alpha_max"], rtol=0, atol=1e-15), key
        assert math.isclose(dt, gold[key]["dt"], rel_tol=1e-13), key


def test_golden_step_count_3d(oracle_mod):
    gold = json.load(open(os.path.join(HERE, "golden", "cfl_steps.json")))["dubins3d_60x60x36"]
    res = oracle_mod.solve_spec(W.config_dubins3d())
    assert res.steps == gold["steps"]
    assert math.isclose(res.dt_first, gold["dt"], rel_tol=1e-13)
    # the clipped last step lands exactly on T
    assert math.isclose(res.dt_min, gold["T"] - (gold["steps"] - 1) * gold["dt"], rel_tol=1e-9)


# ------------------------------------------------------------------ sampled evaluator

def test_step_at_matches_full_step(oracle_mod):
    """The on-demand evaluator (used for sampled checks of huge grids) agrees
    with the whole-grid solver for one step, for every RK order."""
    spec = W.config_dyncar4d(n=[9, 8, 6, 10], T=0.02)
    V0 = W.make_v0(spec)
    rng = np.random.default_rng(3)
    Vs = V0 + 0.05 * rng.standard_normal(V0.shape)
    idx = rng.choice(V0.size, 60, replace=False)
    idx = np.concatenate([idx, [0, V0.size - 1]])
    for rk in (1, 2, 3):
        full = oracle_mod.solve(spec.grid, spec.dyn, V0, [0.0, 0.004], rk_order=rk, cfl=0.8,
                                brt=True, V_init=Vs)
        assert full.steps == 1
        pts = oracle_mod.step_at(spec.grid, spec.dyn, Vs, V0, 0.004, idx, rk_order=rk, brt=True)
        assert np.array_equal(pts, full.V.reshape(-1)[idx])


def test_restart_equals_single_call(oracle_mod):
    spec = W.config_dubins3d(n=(20, 18, 12), T=1.0)
    V0 = W.make_v0(spec)
    one = oracle_mod.solve(spec.grid, spec.dyn, V0, [0.0, 0.37, 1.0], save_all=True)
    a = oracle_mod.solve(spec.grid, spec.dyn, V0, [0.0, 0.37])
    b = oracle_mod.solve(spec.grid, spec.dyn, V0, [0.37, 1.0], V_init=a.V)
    assert np.array_equal(one.V_all[1], a.V)
    assert np.array_equal(one.V, b.V)
    assert one.steps == a.steps + b.steps


# ------------------------------------------------------------------ pin 9

def _advection_case():
    """Periodic 1D advection z' = c (c > 0 moves data towards -x): at CFL
    lambda one step is V_i + lambda (V_{i+1} - V_i) (pin 2), an exact
    one-cell shift at lambda = 1; 9 steps to the horizon."""
    g = W.GridSpec([30], [-4.0], [4.0], [1])
    x = g.axis(0)
    V0 = np.sin(2 * np.pi * x / 8) + 0.4 * np.cos(6 * np.pi * x / 8)
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, 0.6], W.MINIMISE, W.MINIMISE)
    rng = np.random.default_rng(99)
    target = 0.6 * np.cos(2 * np.pi * x / 8 + 1.0) + 0.1 * rng.standard_normal(x.size)
    obstacle = np.where(np.abs(x - 1.5) < 1.0, 0.3, -5.0) + 0.05 * rng.standard_normal(x.size)
    return g, d, V0, target, obstacle, 9


def _recursion(V0, steps, op, lam=1.0):
    V = V0.copy()
    for _ in range(steps):
        V = op(V + lam * (np.roll(V, -1) - V), V)
    return V


CASES_PIN9 = [
    # tmode, omode, per-step operation op(shifted, V^n) with target l / obstacle g
    ("minVWithV0", "none", lambda s, vn, V0, l, g: np.minimum(s, V0)),
    ("maxVWithV0", "none", lambda s, vn, V0, l, g: np.maximum(s, V0)),
    ("minVWithVInit", "none", lambda s, vn, V0, l, g: np.minimum(s, vn)),
    ("maxVWithVInit", "none", lambda s, vn, V0, l, g: np.maximum(s, vn)),
    ("minVWithVTarget", "none", lambda s, vn, V0, l, g: np.minimum(s, l)),
    ("maxVWithVTarget", "none", lambda s, vn, V0, l, g: np.maximum(s, l)),
    ("none", "minVWithObstacle", lambda s, vn, V0, l, g: np.minimum(s, g)),
    ("none", "maxVWithObstacle", lambda s, vn, V0, l, g: np.maximum(s, g)),
    ("minVWithVTarget", "maxVWithObstacle", lambda s, vn, V0, l, g: np.maximum(np.minimum(s, l), g)),
    ("minVWithV0", "maxVWithObstacle", lambda s, vn, V0, l, g: np.maximum(np.minimum(s, V0), g)),
]


@pytest.mark.parametrize("tmode,omode,op", CASES_PIN9, ids=[f"{a}+{b}" for a, b, _ in CASES_PIN9])
@pytest.mark.parametrize("cfl", [1.0, 0.5])
def test_pin9_computation_methods_closed_form(oracle_mod, tmode, omode, op, cfl):
    g, d, V0, l, ob, steps = _advection_case()
    _, dt = oracle_mod.cfl_dt(g, d, cfl)
    res = oracle_mod.solve(g, d, V0, [0.0, steps * dt * (1 - 1e-12)], rk_order=1, cfl=cfl,
                           tmode=tmode, omode=omode, target=l, obstacle=ob)
    assert res.steps == steps
    expect = _recursion(V0, steps, lambda s, vn: op(s, vn, V0, l, ob), lam=cfl)
    # the horizon sits 1e-12 short of 9 CFL steps, so the last step has
    # lambda short by O(1e-11): hence the tolerance
    assert np.abs(res.V - expect).max() < 1e-10
    # every method changes the plain transport somewhere
    plain = _recursion(V0, steps, lambda s, vn: s, lam=cfl)
    assert np.abs(expect - plain).max() > 0.05


@pytest.mark.parametrize("tmode,npop", [("minVWithVInit", np.minimum), ("maxVWithVInit", np.maximum),
                                         ("minVWithV0", None)])
def test_pin9_restart_reference(oracle_mod, tmode, npop):
    """From a restart value V_init != V0 the value-over-time methods take
    min/max with the previous step's value (which starts at V_init), the V0
    method keeps using V0.  (From V_init = V0 a monotone scheme makes
    min(S V^n, V^n) equal to min(S V^n, V0) by induction, so only a restart
    tells the two references apart.)"""
    g, d, V0, l, ob, steps = _advection_case()
    x = np.arange(V0.size) / V0.size
    Vi = V0 + 0.4 * np.cos(6 * np.pi * x) + 0.2
    for cfl in (1.0, 0.5):
        _, dt = oracle_mod.cfl_dt(g, d, cfl)
        res = oracle_mod.solve(g, d, V0, [0.0, steps * dt * (1 - 1e-12)], rk_order=1, cfl=cfl,
                               tmode=tmode, V_init=Vi)
        if npop is None:
            expect = _recursion(Vi, steps, lambda s_, vn: np.minimum(s_, V0), lam=cfl)
        else:
            expect = _recursion(Vi, steps, lambda s_, vn: npop(s_, vn), lam=cfl)
        assert np.abs(res.V - expect).max() < 1e-10
        other = _recursion(Vi, steps, lambda s_, vn: np.minimum(s_, Vi if npop is None else V0),
                           lam=cfl)
        assert np.abs(expect - other).max() > 0.05


@pytest.mark.parametrize("cfl", [1.0, 0.5])
def test_pin9_time_varying_sets(oracle_mod, cfl):
    """Time-varying target and obstacle: slice k holds the sets at tau[k];
    the steps from tau[k-1] to tau[k] compare with slice k-1.  Three output
    intervals of three steps each, slices that differ from one another."""
    g, d, V0, l, ob, steps = _advection_case()
    _, dt = oracle_mod.cfl_dt(g, d, cfl)
    tau = [3 * k * dt * (1 - 1e-12) for k in range(4)]
    L = np.stack([np.roll(l, 4 * k) - 0.1 * k for k in range(4)])
    G = np.stack([np.roll(ob, -3 * k) + 0.05 * k for k in range(4)])
    res = oracle_mod.solve(g, d, V0, tau, rk_order=1, cfl=cfl, tmode="minVWithVTarget",
                           omode="maxVWithObstacle", target=L, obstacle=G)
    assert res.steps == 9
    V = V0.copy()
    for st in range(9):
        k = st // 3
        V = np.maximum(np.minimum(V + cfl * (np.roll(V, -1) - V), L[k]), G[k])
    assert np.abs(res.V - V).max() < 1e-10
    # a static set (slice 0 throughout) gives another answer
    static = oracle_mod.solve(g, d, V0, tau, rk_order=1, cfl=cfl, tmode="minVWithVTarget",
                              omode="maxVWithObstacle", target=L[0], obstacle=G[0])
    assert np.abs(static.V - V).max() > 0.05


def test_pin9_target_equal_to_v0_is_the_v0_method(oracle_mod):
    spec = W.config_dubins3d(n=(17, 15, 12), T=0.6)
    V0 = W.make_v0(spec)
    for a, b in (("minVWithVTarget", "minVWithV0"), ("maxVWithVTarget", "maxVWithV0")):
        ra = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=2, tmode=a, target=V0).V
        rb = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=2, tmode=b).V
        assert np.array_equal(ra, rb)


def test_pin9_value_over_time_monotone(oracle_mod):
    """min / max with V^n: V(tau_k) is exactly non-increasing / non-decreasing."""
    spec = W.config_dubins3d(n=(17, 15, 12), T=0.6)
    V0 = W.make_v0(spec)
    tau = [0.0, 0.15, 0.3, 0.45, 0.6]
    lo = oracle_mod.solve(spec.grid, spec.dyn, V0, tau, rk_order=3, tmode="minVWithVInit",
                          save_all=True).V_all
    hi = oracle_mod.solve(spec.grid, spec.dyn, V0, tau, rk_order=3, tmode="maxVWithVInit",
                          save_all=True).V_all
    assert (lo[1:] <= lo[:-1]).all() and (hi[1:] >= hi[:-1]).all()
    assert (lo[-1] < V0 - 1e-6).any() and (hi[-1] > V0 + 1e-6).any()


def test_pin9_obstacle_bounds(oracle_mod):
    """An obstacle below every value (max) or above every value (min) changes
    nothing; max with a large constant gives that constant everywhere."""
    spec = W.config_dubins3d(n=(17, 15, 12), T=0.6)
    V0 = W.make_v0(spec)
    ref = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=1, brt=True).V
    lo = np.full(V0.shape, -1e30)
    hi = np.full(V0.shape, 1e30)
    a = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=1, brt=True,
                         omode="maxVWithObstacle", obstacle=lo).V
    b = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=1, brt=True,
                         omode="minVWithObstacle", obstacle=hi).V
    c = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=1, brt=True,
                         omode="maxVWithObstacle", obstacle=np.full(V0.shape, 7.0)).V
    assert np.array_equal(a, ref) and np.array_equal(b, ref) and (c == 7.0).all()


# ------------------------------------------------------------------ pin 13
# The global-alpha approximation (Algorithm 1's note that the per-point alpha
# may be replaced by the largest rate of change over the grid).

def _dubins_no_turn(n_xy, n_th, v=1.0, w=0.3, T=0.4):
    g = W.GridSpec([n_xy, n_xy, n_th], [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_DUBINS3D, [v, w], W.MAXIMISE, W.MINIMISE)
    return g, d


def test_pin13_global_alpha_heat_step_where_the_drift_vanishes(oracle_mod):
    """Dubins car with V = x^2 (no y or heading dependence).  On the heading
    slice th = pi/2 the x-velocity v cos th vanishes (to rounding), so with
    per-point alpha the x term is zero and V does not move, while the global
    approximation dissipates with alpha^max_x = v: one step is the discrete
    heat step V_i + dt (v / 2dx)(V_{i+1} - 2 V_i + V_{i-1}) = x^2 + dt v dx at
    interior nodes (worked out by hand).  On th = 0 both forms are the
    upwind step x^2 + dt v (2x + dx) (forward difference, v > 0).  The
    heading term (alpha_th = w) and y terms see zero differences."""
    v, w, dt = 1.3, 0.3, 0.01
    g, d = _dubins_no_turn(41, 4, v=v, w=w)  # headings -pi, -pi/2, 0, pi/2
    x = g.axis(0)
    X = np.broadcast_to(x[:, None, None], tuple(g.n))
    V = np.ascontiguousarray(X * X)
    dx = x[1] - x[0]
    amax, _ = oracle_mod.cfl_dt(g, d, 0.8)
    assert abs(amax[0] - v) < 1e-15 and abs(amax[2] - w) < 1e-15
    ix = np.arange(1, 40)
    for k, expect_local, expect_global in (
            (3, x[ix] ** 2, x[ix] ** 2 + dt * v * dx),                       # th = pi/2
            (2, x[ix] ** 2 + dt * v * (2 * x[ix] + dx), x[ix] ** 2 + dt * v * (2 * x[ix] + dx))):  # th = 0
        idx = np.ravel_multi_index((ix, np.full_like(ix, 2), np.full_like(ix, k)), tuple(g.n))
        loc = oracle_mod.step_at(g, d, V, V, dt, idx, brt=False)
        glo = oracle_mod.step_at(g, d, V, V, dt, idx, brt=False, alpha_glob=amax)
        assert np.abs(loc - expect_local).max() < 1e-12, k
        assert np.abs(glo - expect_global).max() < 1e-12, k
    # the whole solve takes the same global-alpha dissipation
    res = oracle_mod.solve(g, d, V, [0.0, dt], rk_order=1, cfl=0.8, brt=False, global_alpha=True)
    got = res.V[ix, 2, 3]
    assert np.abs(got - (x[ix] ** 2 + dt * v * dx)).max() < 1e-12


def _advected(g, v, T, r=1.0):
    """Dubins with w = 0 is a constant-velocity advection on every heading
    slice: V(z, T) = V0(x + v cos th T, y + v sin th T) for V0 = |(x, y)| - r."""
    X, Y, TH = np.meshgrid(g.axis(0), g.axis(1), g.axis(2), indexing="ij")
    return np.sqrt((X + v * np.cos(TH) * T) ** 2 + (Y + v * np.sin(TH) * T) ** 2) - r


def test_pin13_global_alpha_converges_at_first_order(oracle_mod):
    """With the turn bound 0 every heading slice is an advection whose exact
    solution is the advected cone; the global-alpha scheme (more diffusive
    where |v cos th| < v) still converges to it at first order in the band
    |V| <= 0.5 (observed order in [0.7, 1.3]) and differs from the
    per-point form by O(dx)."""
    errs, hs = [], []
    for n in (26, 51, 101):
        g, d = _dubins_no_turn(n, 8, v=1.0, w=0.0)
        V0 = W.cylinder_v0(g, 1.0)
        T = 0.5
        res = oracle_mod.solve(g, d, V0, [0.0, T], rk_order=1, cfl=0.8, brt=False, global_alpha=True)
        exact = _advected(g, 1.0, T)
        band = np.abs(exact) <= 0.5
        errs.append(np.abs(res.V - exact)[band].max())
        hs.append(8.0 / (n - 1))
        loc = oracle_mod.solve(g, d, V0, [0.0, T], rk_order=1, cfl=0.8, brt=False)
        diff = np.abs(res.V - loc.V)[band].max()
        assert 0.01 * hs[-1] < diff < 2.0 * hs[-1], (n, diff)
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(2)]
    assert all(0.7 <= o <= 1.3 for o in orders), (errs, orders)


def test_pin13_global_alpha_tube_monotone(oracle_mod):
    """Pin 3 with the global approximation: the scheme stays monotone (alpha
    only grows), so the tube never grows back inside and V <= V0."""
    spec = W.config_dubins3d(n=(24, 24, 16), T=0.6)
    V0 = W.make_v0(spec)
    res = oracle_mod.solve(spec.grid, spec.dyn, V0, [0.0, 0.3, 0.6], rk_order=1, cfl=0.8, brt=True,
                           global_alpha=True, save_all=True)
    A = res.V_all
    assert np.all(A[1] <= V0 + 1e-12) and np.all(A[2] <= V0 + 1e-12)
    inner = (slice(1, -1), slice(1, -1), slice(None))
    assert np.all(A[2][inner] <= A[1][inner] + 1e-12)
    assert np.abs(A[2] - V0).max() > 0.1


# ------------------------------------------------------------------ pin 14
# ENO2 stencil choices taken in float32 (as a float32 solve takes them).

def test_pin14_eno_f32_choices_agree_with_margins(oracle_mod):
    """Where the two candidate second differences differ by far more than
    float32 rounding (V = exp(x/2): consecutive second differences differ by
    a factor e^{dx/2}), taking the choices in float32 changes nothing: the
    step is the same, bit for bit, on float32-representable data."""
    for c in (0.8, -0.6):
        g, d = _drift_1d(41, c=c)
        V = np.exp(g.axis(0) / 2).astype(np.float32).astype(np.float64)
        idx = np.arange(41)
        a = oracle_mod.step_at(g, d, V, V, 0.01, idx, brt=False, space_order=2, eno_f32=True)
        b = oracle_mod.step_at(g, d, V, V, 0.01, idx, brt=False, space_order=2, eno_f32=False)
        assert np.array_equal(a, b), c


def test_pin14_eno_f32_near_tie_built_by_hand(oracle_mod):
    """A stencil (V_{i-2}, V_{i-1}, V_i, V_{i+1}) = (2^-30, 0, 1, 3) on unit
    spacing: the minus side's candidates are sm = 1 + 2^-30 and s0 = 1.  In
    float64 |sm| > |s0|, so p- = dm + s0/2 = 1.5; in float32 the difference
    1 + 2^-30 rounds to 1, a tie, which takes the first candidate: p- = 1 +
    (1 + 2^-30)/2 (the correction itself in float64).  With drift c = -1
    (alpha = 1) the step is V_i - dt p-, so the two forms differ by exactly
    dt 2^-31."""
    g = W.GridSpec([8], [0.0], [7.0], [0])
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [0.0, -1.0], W.MAXIMISE, W.MINIMISE)
    V = np.array([5.0, 4.0, 2.0 ** -30, 0.0, 1.0, 3.0, 6.0, 10.0])
    dt = 0.25
    i = 4
    f64 = oracle_mod.step_at(g, d, V, V, dt, [i], brt=False, space_order=2, eno_f32=False)[0]
    f32 = oracle_mod.step_at(g, d, V, V, dt, [i], brt=False, space_order=2, eno_f32=True)[0]
    # plus side (s0 = 1 against sp = 3 - 2 = 1, a tie in both: first) is the
    # same in both forms; with c = -1 the LF form uses p- only
    assert f64 == 1.0 - dt * 1.5
    assert f32 == 1.0 - dt * (1.5 + 2.0 ** -31)


# ------------------------------------------------------------------ pin 15
# The parallel (Jacobi) time-to-reach iteration, derived by hand.

def test_pin15_ttr_jacobi_front_in_1d(oracle_mod):
    """1D, |u| <= 1 (sigma = 1), target = node 0, unit spacing.  The point
    update reduces to phi_i <- min(phi_i, 1 + min(phi_{i-1}, phi_{i+1})) (the
    centred costate's |pbar| term cancels the neighbour mean's difference),
    so in the parallel form the front advances exactly one node per
    iteration: after k iterations phi_i = i for i <= k and the start value
    beyond.  The far edge node takes max(2 phi_a - phi_b, phi_b) from the
    previous iterate, one iteration after its inner neighbour is reached,
    giving n - 1.  (A forward Gauss-Seidel sweep finishes the interior in one
    iteration.)"""
    n, big = 12, 1e4
    g = W.GridSpec([n], [0.0], [float(n - 1)], [0])
    d = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [1.0, 0.0], W.MINIMISE, W.MAXIMISE)
    l = np.arange(n, dtype=np.float64) - 0.5  # only node 0 has l <= 0
    for k in (1, 4, n - 3, n - 2, n - 1):
        r = oracle_mod.ttr_solve(g, d, l, eps=1e-300, max_iters=k, big=big, jacobi=True)
        expect = np.where(np.arange(n) <= k, np.arange(n, dtype=np.float64), big)
        expect[n - 1] = n - 1.0 if k >= n - 1 else big
        assert np.array_equal(r.phi, expect), (k, r.phi)
    conv = oracle_mod.ttr_solve(g, d, l, eps=1e-12, jacobi=True, big=big)
    assert np.array_equal(conv.phi, np.arange(n, dtype=np.float64)) and conv.iters == n
    gs = oracle_mod.ttr_solve(g, d, l, eps=1e-300, max_iters=1, big=big)
    assert np.array_equal(gs.phi[:n - 1], np.arange(n - 1, dtype=np.float64))
