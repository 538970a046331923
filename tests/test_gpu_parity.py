"""GPU parity: the HIP path (through the C ABI) against the float64 oracle.

Bars: float64 GPU within 1e-9 * S of the oracle, float32 GPU within 1e-4 * S
(S = largest non-periodic extent), the same step count, element by element
on the whole grid.  Sizes span several 256-point tiles with ragged tails and
axis-0 chunks that do not divide the axis.
"""
import math

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


def _dtype(prec):
    import torch
    return torch.float64 if prec == 64 else torch.float32


def gpu_solve(odp, spec, V0, prec, **kw):
    import torch
    print(f"[gpu] {spec.name} fp{prec} n={spec.grid.n} rk={spec.rk_order} {kw}", flush=True)
    dev = torch.device("cuda:0")
    t = torch.tensor(V0, dtype=_dtype(prec), device=dev)
    vi = kw.pop("V_init", None)
    if vi is not None:
        vi = torch.tensor(vi, dtype=_dtype(prec), device=dev)
    res = odp.solve(spec, t, precision=prec, V_init=vi, **kw)
    torch.cuda.synchronize()
    return res


def compare(odp, oracle_mod, spec, prec, V0=None, oracle_kw=None, **kw):
    V0 = W.make_v0(spec) if V0 is None else V0
    okw = dict(oracle_kw or {})
    ref = oracle_mod.solve(spec.grid, spec.dyn, V0, spec.tau, rk_order=spec.rk_order,
                           cfl=spec.cfl, brt=spec.mode == W.BRT, **okw)
    res = gpu_solve(odp, spec, V0, prec, **kw)
    got = res.V.double().cpu().numpy()
    S = spec.grid.domain_scale()
    err = float(np.abs(got - ref.V).max())
    loc = np.unravel_index(int(np.abs(got - ref.V).argmax()), got.shape)
    print(f"    steps gpu={res.stats['steps']} oracle={ref.steps} max|err|={err:.3e} at {loc} "
          f"(/S = {err / S:.3e}, limit {TOL[prec]:.0e})", flush=True)
    assert res.stats["steps"] == ref.steps
    assert math.isclose(res.stats["dt_max"], ref.dt_max, rel_tol=0, abs_tol=0)
    assert err <= TOL[prec] * S
    return res, ref


CASES = [
    ("dubins3d_60x60x36", lambda: W.config_dubins3d(), (64, 32)),
    ("dubins3d_ragged", lambda: W.config_dubins3d(n=(37, 29, 22), T=1.3), (64, 32)),
    ("dyncar4d_22x21x19x24_rk3", lambda: W.config_dyncar4d(n=[22, 21, 19, 24], T=0.6), (64, 32)),
    ("game6d_9x8x8x7x9x8_rk2", lambda: W.config_game6d(n=[9, 8, 8, 7, 9, 8], T=0.5), (64, 32)),
    # axis N-2 periodic: its rows wrapped across the edge are not in a
    # block's LDS tile; in 6D they are copied into LDS with the plane's other
    # memory-loaded neighbours
    ("game6d_periodic_axis4", lambda: _periodic4(W.config_game6d(n=[8, 7, 6, 5, 9, 12], T=0.4)),
     (64, 32)),
    # axes 1 and 2 in 6 x 6 squares, cubes of axes 3..5 of 11200 points:
    # quad tiles (a block's waves are 2x2 axis-1/axis-2 neighbours; ragged
    # last tile of every cube)
    ("game6d_brick_5x6x6x20x20x28", lambda: W.config_game6d(n=[5, 6, 6, 20, 20, 28], T=0.25), (64, 32)),
    # axes 1 and 2 in 3 x 3 squares only: brick tiles of whole blocks
    ("game6d_brick3_4x9x3x24x24x36", lambda: W.config_game6d(n=[4, 9, 3, 24, 24, 36], T=0.2), (64, 32)),
]


def _periodic4(spec):
    spec.grid.periodic[4] = 1
    spec.name += "_periodic4"
    return spec


@pytest.mark.parametrize("name,mk,precs", CASES, ids=[c[0] for c in CASES])
def test_parity_workloads(odp, oracle_mod, name, mk, precs):
    for prec in precs:
        compare(odp, oracle_mod, mk(), prec)


@pytest.mark.parametrize("ndim,n,drift,role,brt,periodic,rk", [
    (1, 300, [0.6], W.MINIMISE, True, False, 1),
    (1, 257, [-0.3], W.MAXIMISE, False, True, 3),
    (2, 61, [0.5, -0.3], W.MINIMISE, True, False, 2),
    (3, 23, [0.2, -0.3, 0.4], W.MAXIMISE, False, False, 3),
    (4, 11, [0.1, 0.0, -0.2, 0.3], W.MINIMISE, True, True, 1),
    (5, 7, [0.0] * 5, W.MAXIMISE, True, False, 2),
    (6, 6, [0.1] * 6, W.MINIMISE, True, False, 1),
])
def test_parity_single_integrator(odp, oracle_mod, ndim, n, drift, role, brt, periodic, rk):
    spec = W.single_integrator(ndim, n, 1.0, drift, role, 0.4, brt=brt, periodic=periodic,
                               rk_order=rk)
    for prec in (64, 32):
        compare(odp, oracle_mod, spec, prec)


def test_parity_global_alpha(odp, oracle_mod):
    spec = W.config_dyncar4d(n=[15, 14, 9, 16], T=0.4)
    for prec in (64, 32):
        compare(odp, oracle_mod, spec, prec, oracle_kw={"global_alpha": True}, dissipation=1)


def _chunk_specs():
    g6 = W.config_game6d(n=[7, 6, 6, 5, 6, 8], T=0.2)
    return [("dyncar4d_13x17x9x20", W.config_dyncar4d(n=[13, 17, 9, 20], T=0.2)),
            ("dubins3d_15x22x16", W.config_dubins3d(n=(15, 22, 16), T=0.3)),
            ("game6d_7x6x6x5x6x8", g6),
            ("game6d_brick_5x6x6x20x20x28", W.config_game6d(n=[5, 6, 6, 20, 20, 28], T=0.1)),
            ("game6d_brick3_4x9x3x24x24x36", W.config_game6d(n=[4, 9, 3, 24, 24, 36], T=0.1))]


@pytest.mark.parametrize("name,spec", _chunk_specs(), ids=[c[0] for c in _chunk_specs()])
def test_parity_tile_chunks_bitwise(odp, name, spec):
    """Every chunking of axis 0 gives the same bits (the arithmetic per point
    does not depend on the launch shape): runs shorter than the march's
    4-plane cycle and ragged last runs, which end the march early up to four
    dimensions and compute unstored planes from five on."""
    import torch
    V0 = W.make_v0(spec)
    for prec in (64, 32):
        outs = [gpu_solve(odp, spec, V0, prec, tile_chunk=c).V.cpu() for c in (1, 2, 3, 5, 13)]
        same = [bool(torch.equal(o, outs[0])) for o in outs[1:]]
        assert all(same), same


def test_autotuned_tiles_bitwise(odp):
    """The autotuner times candidate tilings in the real workspace (and the
    caller's output array) before the solve: the result equals the default
    tiling's bit for bit, on the first call (tuning) and the second (cache)."""
    import torch
    spec = W.config_dyncar4d(n=[21, 17, 12, 20], T=0.3)
    V0 = W.make_v0(spec)
    for prec in (32, 64):
        ref = gpu_solve(odp, spec, V0, prec).V.cpu()
        for _ in range(2):
            got = gpu_solve(odp, spec, V0, prec, tile_chunk=odp.ODP_TILE_AUTOTUNE).V.cpu()
            assert bool(torch.equal(got, ref))


def test_parity_save_all_and_restart(odp, oracle_mod):
    import torch
    spec = W.config_dubins3d(n=(26, 24, 18), T=1.0)
    V0 = W.make_v0(spec)
    tau = [0.0, 0.23, 0.6, 1.0]
    ref = oracle_mod.solve(spec.grid, spec.dyn, V0, tau, rk_order=1, cfl=0.8, brt=True,
                           save_all=True)
    res = gpu_solve(odp, spec, V0, 64, tau=tau, save_all=True)
    allv = res.V_all.cpu().numpy()
    assert np.abs(allv - ref.V_all).max() <= 1e-9 * 8
    assert res.stats["steps"] == ref.steps
    # restart from tau = 0.23 equals the single call, bit for bit
    first = gpu_solve(odp, spec, V0, 64, tau=[0.0, 0.23])
    second = gpu_solve(odp, spec, V0, 64, tau=[0.23, 0.6, 1.0], V_init=first.V.cpu().numpy())
    same_final = torch.equal(second.V.cpu(), res.V.cpu())
    same_mid = torch.equal(first.V.cpu(), res.V_all[1].cpu())
    assert same_final and same_mid


def test_parity_max_dt_and_rk_orders(odp, oracle_mod):
    for rk in (1, 2, 3):
        spec = W.config_dubins3d(n=(20, 19, 12), T=0.35)
        spec.rk_order = rk
        compare(odp, oracle_mod, spec, 64, oracle_kw={"max_dt": 0.013}, max_dt=0.013)


def test_nonfinite_reported(odp):
    import torch
    spec = W.config_dubins3d(n=(12, 11, 8), T=0.2)
    V0 = W.make_v0(spec)
    V0[3, 4, 5] = np.nan
    t = torch.tensor(V0, dtype=torch.float32, device="cuda:0")
    with pytest.raises(odp.OdpError) as ei:
        odp.solve(spec, t, precision=32)
    assert ei.value.code == odp.ODP_ENONFINITE


def test_graph_replays_equal_eager(odp):
    """The time stepping recorded into a HIP graph (small grids on a stream)
    gives the eager launches' bits, call after call, with eager work and
    synchronisations in between."""
    import torch
    stream = torch.cuda.Stream()
    for spec in (W.config_dubins3d(n=(30, 28, 20), T=0.8), W.config_dyncar4d(n=[12, 11, 9, 16], T=0.3)):
        V0 = W.make_v0(spec)
        for prec in (64, 32):
            eager = gpu_solve(odp, spec, V0, prec, graph=2, stream=stream).V.cpu()
            for rep in range(3):
                g = gpu_solve(odp, spec, V0, prec, graph=1, stream=stream).V.cpu()
                e = gpu_solve(odp, spec, V0, prec, graph=2, stream=stream).V.cpu()
                same = bool(torch.equal(g, eager)) and bool(torch.equal(e, eager))
                assert same, (spec.name, prec, rep)


def test_solve_is_stream_ordered(odp, oracle_mod):
    """odp_hj_solve without stats returns once its work is enqueued: the step
    count is worked out on the host, so nothing waits for the device.  Right
    after the call the stream still runs the 4D solve (about 0.1 s of
    kernels); once it drains, the result equals the same solve with stats
    (which synchronises) bit for bit."""
    import time
    import torch
    spec = W.config_dyncar4d(n=80)
    V0 = torch.tensor(W.make_v0(spec), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.Stream()
    grid = odp.Grid.from_spec(spec.grid)
    opts = odp.make_opts(32, spec.rk_order, spec.cfl, spec.mode, 0, 0.0, 0, 0, odp._stream_handle(stream))
    ws = torch.empty(odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, opts), dtype=torch.uint8,
                     device="cuda:0")
    out = torch.empty_like(V0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    odp.odp_hj_solve(grid, spec.dyn, V0, None, spec.tau, opts, ws, out, want_stats=False)
    t_call = time.perf_counter() - t0
    busy = not stream.query()
    stream.synchronize()
    t_all = time.perf_counter() - t0
    print(f"    call returned after {t_call * 1e3:.1f} ms, stream busy: {busy}, done after {t_all * 1e3:.1f} ms",
          flush=True)
    assert busy and t_call < 0.5 * t_all
    ref = torch.empty_like(V0)
    st = odp.odp_hj_solve(grid, spec.dyn, V0, None, spec.tau, opts, ws, ref, want_stats=True)
    assert st.steps == 359
    assert torch.equal(out, ref)


def test_cached_graph_replays_new_inputs(odp, oracle_mod):
    """A repeated solve of one shape on one workspace replays its cached HIP
    graph; the graph reads V0 and V_out through the descriptors the prologue
    uploads, so new inputs and outputs give the eager results."""
    import torch
    stream = torch.cuda.Stream()
    spec = W.config_dubins3d(n=(30, 28, 20), T=0.8)
    grid = odp.Grid.from_spec(spec.grid)
    for prec in (64, 32):
        dt = _dtype(prec)
        V0a = torch.tensor(W.make_v0(spec), dtype=dt, device="cuda:0")
        V0b = V0a * 0.5 - 0.25
        opts_g = odp.make_opts(prec, 1, spec.cfl, spec.mode, 0, 0.0, 0, 0, odp._stream_handle(stream), 0, 1)
        opts_e = odp.make_opts(prec, 1, spec.cfl, spec.mode, 0, 0.0, 0, 0, odp._stream_handle(stream), 0, 2)
        ws = torch.empty(odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, opts_g), dtype=torch.uint8,
                         device="cuda:0")
        outs = {}
        for name, v0 in (("a", V0a), ("b", V0b), ("a2", V0a)):
            og, oe = torch.empty_like(v0), torch.empty_like(v0)
            odp.odp_hj_solve(grid, spec.dyn, v0, None, spec.tau, opts_g, ws, og, want_stats=False)
            odp.odp_hj_solve(grid, spec.dyn, v0, None, spec.tau, opts_e, ws, oe, want_stats=True)
            stream.synchronize()
            assert torch.equal(og, oe), (prec, name)
            outs[name] = og
        assert torch.equal(outs["a"], outs["a2"]) and not torch.equal(outs["a"], outs["b"])
