"""GPU parity of the computation methods (the paper's table of computation
methods): the six target methods, both obstacle methods alone and the
reach-avoid pairs, through the C ABI against the float64 oracle.

Bars as for the plain solve: float64 within 1e-9 S, float32 within 1e-4 S of
the oracle, the same step count.  The grids reach every kernel form that the
methods touch: the scalar 1D kernel, the 2D vector kernel without the LDS
exchange, and the 3D and 4D kernels with it, in all three Runge-Kutta orders
(the last stage reads V^n, which the value-over-time methods compare with).
"""
import math

import numpy as np
import pytest

from paper_2204_05520_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {64: 1e-9, 32: 1e-4}

METHODS = [
    ("minVWithV0", "None"), ("maxVWithV0", "None"), ("minVWithVInit", "None"),
    ("maxVWithVInit", "None"), ("minVWithVTarget", "None"), ("maxVWithVTarget", "None"),
    ("None", "minVWithObstacle"), ("None", "maxVWithObstacle"),
    ("minVWithVTarget", "maxVWithObstacle"), ("minVWithV0", "maxVWithObstacle"),
    ("maxVWithVInit", "minVWithObstacle"),
]

GRIDS = {
    "si1d_300_rk1": lambda: W.single_integrator(1, 300, 1.0, [0.6], W.MINIMISE, 0.4, rk_order=1),
    "si2d_61_rk2": lambda: W.single_integrator(2, 61, 0.2, [0.5, -0.3], W.MAXIMISE, 0.4, rk_order=2),
    "dubins3d_37x29x22_rk1": lambda: W.config_dubins3d(n=(37, 29, 22), T=0.8),
    "dyncar4d_13x12x9x16_rk3": lambda: W.config_dyncar4d(n=[13, 12, 9, 16], T=0.3),
    # six dimensions: the far axes' neighbours and the pointwise operands
    # (V^n, the target or V0, the obstacle) reach LDS by direct copies
    "game6d_7x6x6x5x6x8_rk1": lambda: _rk(W.config_game6d(n=[7, 6, 6, 5, 6, 8], T=0.2), 1),
    "game6d_7x6x6x5x6x8_rk2": lambda: W.config_game6d(n=[7, 6, 6, 5, 6, 8], T=0.2),
    "game6d_6x7x5x6x5x8_rk3": lambda: _rk(W.config_game6d(n=[6, 7, 5, 6, 5, 8], T=0.2), 3),
}


def _rk(spec, order):
    spec.rk_order = order
    return spec


@pytest.fixture(scope="module")
def odp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_05520_amd as odp
    odp.lib()
    return odp


def _dev(x, prec):
    import torch
    return torch.tensor(x, dtype=torch.float64 if prec == 64 else torch.float32, device="cuda:0")


def _oracle_names(tm, om):
    return ("none" if tm == "None" else tm), ("none" if om == "None" else om)


@pytest.mark.parametrize("gname", list(GRIDS))
def test_methods_parity(odp, oracle_mod, gname):
    import torch
    spec = GRIDS[gname]()
    V0 = W.make_v0(spec)
    target, obstacle = W.reach_avoid_sets(spec)
    S = spec.grid.domain_scale()
    plain = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order,
                             cfl=spec.cfl, tmode="none")
    for tm, om in METHODS:
        otm, oom = _oracle_names(tm, om)
        uses_t = tm in ("minVWithVTarget", "maxVWithVTarget")
        uses_o = om != "None"
        ref = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order,
                               cfl=spec.cfl, tmode=otm, omode=oom, target=target,
                               obstacle=obstacle)
        # the method changes the plain solve: the comparison is exercised
        assert np.abs(ref.V - plain.V).max() > 1e-3, (tm, om)
        for prec in (64, 32):
            print(f"[gpu] methods {gname} {tm}+{om} fp{prec}", flush=True)
            res = odp.solve(spec, _dev(V0, prec), precision=prec, mode=tm, obstacle_mode=om,
                            target=_dev(target, prec) if uses_t else None,
                            obstacle=_dev(obstacle, prec) if uses_o else None)
            torch.cuda.synchronize()
            got = res.V.double().cpu().numpy()
            err = float(np.abs(got - ref.V).max())
            print(f"    steps gpu={res.stats['steps']} oracle={ref.steps} max|err|/S={err / S:.3e}",
                  flush=True)
            assert res.stats["steps"] == ref.steps
            assert err <= TOL[prec] * S, (tm, om, prec, err / S)


@pytest.mark.parametrize("tm", ["minVWithVInit", "maxVWithVInit", "minVWithV0"])
def test_methods_from_restart(odp, oracle_mod, tm):
    """From V_init != V0 the value-over-time methods compare with the value
    before each step (which starts at V_init), the V0 method with V0."""
    import torch
    for spec in (W.config_dubins3d(n=(37, 29, 22), T=0.8),
                 W.config_dyncar4d(n=[13, 12, 9, 16], T=0.3)):
        V0 = W.make_v0(spec)
        target, _ = W.reach_avoid_sets(spec)
        Vi = np.minimum(V0, target) + 0.05
        ref = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order,
                               cfl=spec.cfl, tmode=tm, V_init=Vi)
        S = spec.grid.domain_scale()
        for prec in (64, 32):
            print(f"[gpu] restart {spec.name} {tm} fp{prec}", flush=True)
            res = odp.solve(spec, _dev(V0, prec), precision=prec, V_init=_dev(Vi, prec), mode=tm)
            torch.cuda.synchronize()
            err = float(np.abs(res.V.double().cpu().numpy() - ref.V).max())
            assert res.stats["steps"] == ref.steps
            assert err <= TOL[prec] * S, (tm, prec, err / S)


def test_methods_alg_bytes(odp):
    """Algorithmic bytes per step count the arrays a method reads: V0 or the
    target (one array), the obstacle (one more), none for value over time."""
    import torch
    spec = W.config_dubins3d(n=(37, 29, 22), T=0.4)
    V0 = W.make_v0(spec)
    target, obstacle = W.reach_avoid_sets(spec)
    P = V0.size
    per = {}
    for tm, om in [("None", "None"), ("minVWithV0", "None"), ("maxVWithVInit", "None"),
                   ("minVWithVTarget", "maxVWithObstacle")]:
        res = odp.solve(spec, _dev(V0, 32), precision=32, mode=tm, obstacle_mode=om,
                        target=_dev(target, 32) if tm == "minVWithVTarget" else None,
                        obstacle=_dev(obstacle, 32) if om != "None" else None)
        torch.cuda.synchronize()
        per[(tm, om)] = res.stats["alg_bytes"] / res.stats["steps"] / (4 * P)
    assert per[("None", "None")] == 2
    assert per[("minVWithV0", "None")] == 3
    assert per[("maxVWithVInit", "None")] == 2
    assert per[("minVWithVTarget", "maxVWithObstacle")] == 4


def test_batch_methods_equal_single_bitwise(odp):
    """Batches take the methods without arrays: each member equals its single
    solve bit for bit (one member padded: its last axis is not a whole
    number of 16-byte vectors)."""
    import torch
    for tm in ("maxVWithV0", "minVWithVInit", "maxVWithVInit"):
        specs = [W.config_dubins3d(n=(21, 19, 16), T=0.5), W.config_dubins3d(n=(17, 23, 13), T=0.7)]
        for s in specs:
            s.mode = odp.method_code(tm)
        V0s = [_dev(W.make_v0(s), 32) for s in specs]
        outs, _ = odp.batch(specs, V0s, precision=32)
        for s, v0, o in zip(specs, V0s, outs):
            print(f"[gpu] batch {tm} {s.grid.n}", flush=True)
            one = odp.solve(s, v0, precision=32, mode=tm).V
            torch.cuda.synchronize()
            assert torch.equal(o, one), (tm, s.grid.n)


@pytest.mark.parametrize("spec_fn", [lambda: W.config_dubins3d(n=(37, 29, 22), T=0.8),
                                     lambda: W.config_dyncar4d(n=[13, 12, 9, 16], T=0.3)],
                         ids=["dubins3d_rk1", "dyncar4d_rk3"])
def test_time_varying_sets(odp, oracle_mod, spec_fn):
    """Time-varying target and obstacle (moving discs, one grid per tau
    point): the steps from tau[k-1] to tau[k] compare with the sets at
    tau[k-1]; the reach-avoid pair and the obstacle method alone."""
    import torch
    spec = spec_fn()
    tau = list(np.linspace(0.0, spec.tau[-1], 5))
    V0 = W.make_v0(spec)
    L, G = W.moving_sets(spec, tau)
    S = spec.grid.domain_scale()
    for tm, om in [("minVWithVTarget", "maxVWithObstacle"), ("None", "maxVWithObstacle")]:
        uses_t = tm != "None"
        ref = oracle_mod.solve(spec.grid, spec.dyn, V0, tau, rk_order=spec.rk_order, cfl=spec.cfl,
                               tmode="none" if tm == "None" else tm, omode=om,
                               target=L if uses_t else None, obstacle=G)
        static = oracle_mod.solve(spec.grid, spec.dyn, V0, tau, rk_order=spec.rk_order,
                                  cfl=spec.cfl, tmode="none" if tm == "None" else tm, omode=om,
                                  target=L[0] if uses_t else None, obstacle=G[0])
        assert np.abs(ref.V - static.V).max() > 1e-3
        for prec in (64, 32):
            print(f"[gpu] time-varying {spec.name} {tm}+{om} fp{prec}", flush=True)
            res = odp.solve(spec, _dev(V0, prec), precision=prec, tau=tau, mode=tm, obstacle_mode=om,
                            target=_dev(L, prec) if uses_t else None, obstacle=_dev(G, prec))
            torch.cuda.synchronize()
            err = float(np.abs(res.V.double().cpu().numpy() - ref.V).max())
            print(f"    steps gpu={res.stats['steps']} oracle={ref.steps} max|err|/S={err / S:.3e}",
                  flush=True)
            assert res.stats["steps"] == ref.steps
            assert err <= TOL[prec] * S, (tm, om, prec, err / S)


def test_time_varying_sets_graph_equals_eager(odp):
    """The slice switches between steps are ordinary stream work: recorded in
    the HIP graph they give the eager result bit for bit."""
    import torch
    spec = W.config_dubins3d(n=(37, 29, 22), T=0.8)
    tau = list(np.linspace(0.0, 0.8, 5))
    V0 = _dev(W.make_v0(spec), 32)
    L, G = W.moving_sets(spec, tau)
    L, G = _dev(L, 32), _dev(G, 32)
    st = torch.cuda.Stream()
    outs = []
    for graph in (2, 1, 1):
        with torch.cuda.stream(st):
            r = odp.solve(spec, V0, precision=32, tau=tau, mode="minVWithVTarget",
                          obstacle_mode="maxVWithObstacle", target=L, obstacle=G, stream=st,
                          graph=graph)
        st.synchronize()
        outs.append(r.V.clone())
        torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_paper_interface_hjsolver_ttrsolver(odp, oracle_mod):
    """The paper's HJSolver / TTRSolver calls map onto the entry points:
    reach-avoid with [goal, obstacle] and compMethods, save_all, and the time
    to reach, against the oracle."""
    spec = W.config_dubins3d(n=(37, 29, 22), T=0.8)
    g, d = spec.grid, spec.dyn
    goal, obstacle = W.reach_avoid_sets(spec)
    tau = [0.0, 0.4, 0.8]
    V = odp.HJSolver(d, g, [goal, obstacle], tau,
                     {"TargetSetMode": "minVWithVTarget", "ObstacleSetMode": "maxVWithObstacle"},
                     save_all=True, precision=64)
    ref = oracle_mod.solve(g, d, goal, tau, rk_order=1, cfl=0.8, tmode="minVWithVTarget",
                           omode="maxVWithObstacle", target=goal, obstacle=obstacle, save_all=True)
    assert V.shape == (3,) + tuple(g.n)
    assert np.abs(V - ref.V_all).max() < 1e-9 * g.domain_scale()
    brs = odp.HJSolver(d, g, W.make_v0(spec), tau, precision=64)
    ref = oracle_mod.solve(g, d, W.make_v0(spec), tau, rk_order=1, cfl=0.8, brt=False)
    assert np.abs(brs - ref.V).max() < 1e-9 * g.domain_scale()
    g2 = W.GridSpec([61, 57], [-4.0, -4.0], [4.0, 4.0], [0, 0])
    d2 = W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [1.0, 0.0, 0.0], W.MINIMISE, W.MAXIMISE)
    l2 = W.cylinder_v0(g2, 1.0)
    phi, st = odp.TTRSolver(d2, g2, l2, epsilon=1e-11, precision=64)
    ref = oracle_mod.ttr_solve(g2, d2, l2, eps=1e-12, jacobi=True)
    assert st["converged"] == 1
    assert np.abs(phi - ref.phi).max() < 1e-7 * g2.domain_scale()
