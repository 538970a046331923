"""GPU parity of the relative pursuit-evasion model (the paper's main
example) with the costate box of Algorithm 1: a grid-wide reduction of the
stage input's costate before every stage update, the dissipation taken over
the input pairs the box realises.  Through the C ABI against the float64
oracle; bars as elsewhere (float64 1e-9 S, float32 1e-4 S), the same step
count; non-cubic grids with ragged tails.
"""
import numpy as np
import pytest

from paper_2204_05520_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {64: 1e-9, 32: 1e-4}


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


def _check(odp, oracle_mod, spec, space_order=1, dissipation=0, precs=(64, 32)):
    import torch
    V0 = W.make_v0(spec)
    ref = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order, cfl=spec.cfl,
                           brt=spec.mode == W.BRT, space_order=space_order,
                           global_alpha=bool(dissipation))
    S = spec.grid.domain_scale()
    for prec in precs:
        print(f"[gpu] pe3d {spec.name} order={space_order} diss={dissipation} fp{prec}", flush=True)
        res = odp.solve(spec, _dev(V0, prec), precision=prec, space_order=space_order,
                        dissipation=dissipation)
        torch.cuda.synchronize()
        err = float(np.abs(res.V.double().cpu().numpy() - ref.V).max())
        print(f"    steps gpu={res.stats['steps']} oracle={ref.steps} max|err|/S={err / S:.3e}", flush=True)
        assert res.stats["steps"] == ref.steps
        # float64 boxes round like the oracle's; a float32 box may differ in
        # its last bits, which moves the step only at a pattern threshold
        if prec == 64:
            assert res.stats["dt_max"] == ref.dt_max
        else:
            assert abs(res.stats["dt_max"] - ref.dt_max) <= 1e-12 * ref.dt_max
        assert err <= TOL[prec] * S, (prec, err / S)
    return ref


@pytest.mark.parametrize("n,rk,order", [([23, 21, 16], 1, 1), ([31, 27, 24], 2, 1),
                                        ([19, 23, 18], 3, 1), ([23, 21, 16], 2, 2),
                                        ([40, 40, 36], 1, 1)])
def test_pe3d_parity(odp, oracle_mod, n, rk, order):
    spec = W.config_pe3d(n=n, T=0.6, rk_order=rk)
    ref = _check(odp, oracle_mod, spec, space_order=order)
    assert np.abs(ref.V - W.make_v0(spec)).max() > 0.1


def test_pe3d_global_alpha(odp, oracle_mod):
    _check(odp, oracle_mod, W.config_pe3d(n=[23, 21, 16], T=0.6), dissipation=1)


@pytest.mark.parametrize("rk", [1, 2])
def test_pe3d_narrow_box(odp, oracle_mod, rk):
    """V0 = x + 0.3 |y - 0.5|: the costate box stays narrow for the first
    steps, so its dissipation and Algorithm 1's CFL step (from the largest box
    alpha, (4, 5, 2) against the all-inputs (6, 5, 2) at the start) differ
    from the all-inputs ones: a horizon of 8 all-inputs steps takes 7.  The
    GPU machine reduction, the per-step box alpha^max and the box dissipation are
    what is compared."""
    import torch
    g = W.GridSpec([33, 17, 12], [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)
    X, Y, _ = np.meshgrid(g.axis(0), g.axis(1), g.axis(2), indexing="ij")
    V0 = X + 0.3 * np.abs(Y - 0.5)
    _, dt = oracle_mod.cfl_dt(g, d, 0.8)
    spec = W.SolveSpec(g, d, [0.0, 8 * dt * (1 - 1e-12)], rk_order=rk, cfl=0.8, mode=W.BRS,
                       name=f"pe3d_narrow_box_rk{rk}")
    ref = oracle_mod.solve(g, d, V0, spec.tau, rk_order=rk, cfl=0.8, brt=False)
    assert ref.steps == 7
    for prec in (64, 32):
        res = odp.solve(spec, _dev(V0, prec), precision=prec)
        torch.cuda.synchronize()
        err = float(np.abs(res.V.double().cpu().numpy() - ref.V).max())
        print(f"    narrow box rk{rk} fp{prec}: steps {res.stats['steps']} dt_max {res.stats['dt_max']:.6e} "
              f"(oracle {ref.dt_max:.6e}) max|err| {err:.3e}", flush=True)
        assert res.stats["steps"] == ref.steps
        assert abs(res.stats["dt_max"] - ref.dt_max) <= 1e-12 * ref.dt_max
        assert err <= TOL[prec] * 8.0, (prec, err)


def test_pe3d_narrow_box_save_all_and_odd_steps(odp, oracle_mod):
    """save_all on a solve whose landings the device decides (the box step),
    with output times chosen so that the step count is odd and even across
    intervals (first-order results then end in either ping-pong buffer):
    every saved slice matches the oracle's."""
    import torch
    g = W.GridSpec([33, 17, 12], [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
    d = W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)
    X, Y, _ = np.meshgrid(g.axis(0), g.axis(1), g.axis(2), indexing="ij")
    V0 = X + 0.3 * np.abs(Y - 0.5)
    _, dt = oracle_mod.cfl_dt(g, d, 0.8)
    tau = [0.0, 2.5 * dt, 5.2 * dt, 8.1 * dt]
    spec = W.SolveSpec(g, d, tau, rk_order=1, cfl=0.8, mode=W.BRS, name="pe3d_narrow_box_save_all")
    ref = oracle_mod.solve(g, d, V0, tau, rk_order=1, cfl=0.8, brt=False, save_all=True)
    for prec in (64, 32):
        res = odp.solve(spec, _dev(V0, prec), precision=prec, save_all=True)
        torch.cuda.synchronize()
        assert res.stats["steps"] == ref.steps
        allv = res.V_all.double().cpu().numpy()
        for k in range(len(tau)):
            err = float(np.abs(allv[k] - ref.V_all[k]).max())
            assert err <= TOL[prec] * 8.0, (prec, k, err)
        assert np.array_equal(res.V.cpu().numpy(), res.V_all[-1].cpu().numpy())


def test_pe3d_capture_100_full_size(odp, oracle_mod):
    """The benchmark workload itself (100^3, horizon 1.5, first order, tube):
    the costate box spans both signs of the evader's switching function at
    every node from the first step on, so Algorithm 1's box alpha^max is the
    all-inputs bound at every step (all 315 steps take the all-inputs dt, the
    last one clipped), and the whole grid matches the oracle."""
    import torch
    spec = W.config_pe3d(n=100)
    V0 = W.make_v0(spec)
    _, dt_all = oracle_mod.cfl_dt(spec.grid, spec.dyn, spec.cfl)
    print("[gpu] pe3d 100^3 full size: oracle solve (float64, CPU)", flush=True)
    ref = oracle_mod.solve_spec(spec, V0)
    assert ref.dt_max == dt_all and ref.steps == 315
    S = spec.grid.domain_scale()
    for prec in (64, 32):
        res = odp.solve(spec, _dev(V0, prec), precision=prec)
        torch.cuda.synchronize()
        err = float(np.abs(res.V.double().cpu().numpy() - ref.V).max())
        print(f"    100^3 fp{prec}: steps {res.stats['steps']} dt_max {res.stats['dt_max']!r} "
              f"max|err|/S {err / S:.3e}", flush=True)
        assert res.stats["steps"] == 315
        assert res.stats["dt_max"] == dt_all
        assert err <= TOL[prec] * S


def test_pe3d_launch_shapes_and_batch_bitwise(odp):
    import torch
    spec = W.config_pe3d(n=[23, 21, 16], T=0.4)
    V0 = _dev(W.make_v0(spec), 32)
    outs = [odp.solve(spec, V0, precision=32, tile_chunk=c).V.cpu() for c in (1, 5, 23)]
    assert all(torch.equal(o, outs[0]) for o in outs[1:])
    specs = [W.config_pe3d(n=[23, 21, 16], T=0.4), W.config_pe3d(n=[17, 19, 14], T=0.7),
             W.config_dubins3d(n=(21, 19, 16), T=0.5)]
    V0s = [_dev(W.make_v0(s), 32) for s in specs]
    bouts, _ = odp.batch(specs, V0s, precision=32)
    for s, v0, o in zip(specs, V0s, bouts):
        one = odp.solve(s, v0, precision=32).V
        torch.cuda.synchronize()
        assert torch.equal(o, one), s.name


def test_pe3d_served_equals_alone(odp):
    """Served pursuit-evasion requests (each tick runs the box pass of every
    active solve before its update, each solve's own step counter choosing
    its box buffer) equal the same solves alone, bit for bit, also mixed with
    Dubins requests and with staggered horizons."""
    import time
    import torch
    srv = odp.Server(1 << 30, 4, precision=32, rk_order=1)
    try:
        specs = [W.config_pe3d(n=[23, 21, 16], T=0.4), W.config_dubins3d(n=(21, 19, 16), T=0.5),
                 W.config_pe3d(n=[17, 19, 14], T=0.7)]
        tickets = [srv.submit(s, W.make_v0(s)) for s in specs]
        for s, t in zip(specs, tickets):
            out = np.empty(tuple(s.grid.n), np.float32)
            t0 = time.time()
            while True:
                rc, _ = srv.poll(t, out)
                if rc != odp.ODP_PENDING:
                    break
                assert time.time() - t0 < 60
                time.sleep(0.002)
            assert rc == odp.ODP_OK
            one = odp.solve(s, _dev(W.make_v0(s), 32), precision=32).V
            torch.cuda.synchronize()
            assert np.array_equal(out, one.cpu().numpy()), s.name
    finally:
        srv.close()
