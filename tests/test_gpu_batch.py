"""GPU batch (odp_hj_batch): every member equals the same solve run alone
through odp_hj_solve, bit for bit, and the float64 batch matches the oracle.
Sizes are small, uneven, with ragged tails and every vector width."""
import numpy as np
import pytest

from paper_2204_05520_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def odp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_05520_amd as odp
    odp.lib()
    return odp


def small_batch(count, seed, T=0.6):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = [int(rng.integers(9, 27)), int(rng.integers(9, 27)), int(rng.integers(6, 21))]
        g = W.GridSpec(n, [-4.0, -4.0, -np.pi], [4.0, 4.0, np.pi], [0, 0, 1])
        d = W.DynSpec(W.DYN_DUBINS3D, [float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.5, 2.0))],
                      W.MAXIMISE, W.MINIMISE)
        specs.append(W.SolveSpec(g, d, [0.0, float(rng.uniform(0.2, T))], rk_order=1, cfl=0.8,
                                 mode=W.BRT, radius=float(rng.uniform(0.3, 1.2)), name=f"b{i}"))
    return specs


def _dev(V0, prec):
    import torch
    return torch.tensor(V0, dtype=torch.float32 if prec == 32 else torch.float64, device="cuda:0")


@pytest.mark.parametrize("prec", [32, 64])
def test_batch_equals_single(odp, prec):
    import torch
    specs = small_batch(23, 11 + prec)
    V0s = [_dev(W.make_v0(s), prec) for s in specs]
    print(f"[gpu] batch of {len(specs)} dubins3d fp{prec}", flush=True)
    outs, stats = odp.batch(specs, V0s, precision=prec)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        single = odp.solve(s, V0s[i], precision=prec)
        same = bool(torch.equal(single.V, outs[i]))
        assert same, (i, s.grid.n, float((single.V - outs[i]).abs().max()))
        assert stats[i]["steps"] == single.stats["steps"]


def test_batch_autotuned_equals_default(odp):
    """Autotuned batch tiles (first call tunes, second hits the cache) give
    the default tiling's bits for every member."""
    import torch
    specs = small_batch(17, 5)
    V0s = [_dev(W.make_v0(s), 32) for s in specs]
    ref, _ = odp.batch(specs, V0s, precision=32)
    for _ in range(2):
        got, st = odp.batch(specs, V0s, precision=32, tile_chunk=odp.ODP_TILE_AUTOTUNE)
        torch.cuda.synchronize()
        for i in range(len(specs)):
            assert bool(torch.equal(got[i], ref[i])), i


def test_batch_fp64_matches_oracle(odp, oracle_mod):
    import torch
    specs = small_batch(6, 5)
    V0n = [W.make_v0(s) for s in specs]
    outs, stats = odp.batch(specs, [_dev(v, 64) for v in V0n], precision=64)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        ref = oracle_mod.solve(s.grid, s.dyn, V0n[i], s.tau, rk_order=1, cfl=0.8, brt=True)
        err = float(np.abs(outs[i].cpu().numpy() - ref.V).max())
        print(f"    member {i} n={s.grid.n} steps={stats[i]['steps']} err={err:.2e}", flush=True)
        assert stats[i]["steps"] == ref.steps
        assert err <= 1e-9 * 8


def test_batch_mixed_dynamics_rk3(odp, oracle_mod):
    """Different dynamics and dimensions in one batch (several kernel groups)."""
    import torch
    specs = [W.config_dyncar4d(n=[11, 10, 7, 12], T=0.3),
             W.config_dubins3d(n=(13, 12, 10), T=0.3),
             W.config_dyncar4d(n=[9, 12, 6, 9], T=0.2),
             W.single_integrator(2, 21, 1.0, [0.2, -0.1], W.MINIMISE, 0.3, brt=True),
             W.config_game6d(n=[6, 5, 6, 5, 6, 4], T=0.2)]
    for s in specs:
        s.rk_order = 3
    V0n = [W.make_v0(s) for s in specs]
    outs, stats = odp.batch(specs, [_dev(v, 64) for v in V0n], precision=64)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        ref = oracle_mod.solve(s.grid, s.dyn, V0n[i], s.tau, rk_order=3, cfl=0.8,
                               brt=s.mode == W.BRT)
        err = float(np.abs(outs[i].cpu().numpy() - ref.V).max())
        print(f"    {s.name} steps={stats[i]['steps']} err={err:.2e}", flush=True)
        assert stats[i]["steps"] == ref.steps
        assert err <= 1e-9 * s.grid.domain_scale()


def test_batch_rejects_bad_entry(odp):
    import torch
    specs = small_batch(3, 1)
    V0s = [_dev(W.make_v0(s), 32) for s in specs]
    specs[1].tau = [0.5, 0.1]
    with pytest.raises(odp.OdpError) as ei:
        odp.batch(specs, V0s, precision=32)
    assert ei.value.code == odp.ODP_EINVAL
