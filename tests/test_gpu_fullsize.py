"""Parity at the full workload sizes, in the launch configuration bench.py
uses (default tiles), on outputs the oracle can compute one by one: one CFL
step from V0 with dt fixed by the output time (below the CFL step), checked
at sampled points (corners, faces, random) against the oracle's on-demand
evaluator.  Whole-solve properties at full size: the tube stays below V0,
shrinks monotonically in time, and the float32 solve stays within 1e-4 S of
the float64 solve (whose parity with the oracle is checked on smaller grids).
"""
import itertools

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


def sample_indices(shape, count, seed):
    rng = np.random.default_rng(seed)
    corners = [np.ravel_multi_index(c, shape)
               for c in itertools.product(*[(0, n - 1) for n in shape])]
    faces = []
    for d in range(len(shape)):
        for side in (0, shape[d] - 1):
            idx = [int(rng.integers(0, n)) for n in shape]
            idx[d] = side
            faces.append(np.ravel_multi_index(idx, shape))
    rnd = rng.integers(0, int(np.prod(shape, dtype=np.int64)), size=count)
    return np.unique(np.concatenate([corners, faces, rnd]).astype(np.int64))


def one_step_check(odp, oracle_mod, spec, prec, t1, V0_np, V0_dev, seed):
    import torch
    print(f"[gpu] full-size one step {spec.name} fp{prec} dt={t1}", flush=True)
    res = odp.solve(spec, V0_dev, precision=prec, tau=[0.0, t1])
    torch.cuda.synchronize()
    assert res.stats["steps"] == 1
    idx = sample_indices(tuple(spec.grid.n), 3000, seed)
    got = res.V.reshape(-1)[torch.tensor(idx, device=res.V.device)].double().cpu().numpy()
    ref = oracle_mod.step_at(spec.grid, spec.dyn, V0_np, V0_np, t1, idx, rk_order=spec.rk_order,
                             brt=True)
    S = spec.grid.domain_scale()
    err = float(np.abs(got - ref).max())
    print(f"    {idx.size} sampled points, max|err| = {err:.3e} (/S {err / S:.2e})", flush=True)
    assert err <= (1e-9 if prec == 64 else 1e-4) * S
    return res


def test_dyncar4d_80_full_size(odp, oracle_mod):
    import torch
    spec = W.config_dyncar4d()
    V0_np = W.make_v0(spec)
    outs = {}
    for prec, dt in ((32, torch.float32), (64, torch.float64)):
        V0 = torch.tensor(V0_np, dtype=dt, device="cuda:0")
        one_step_check(odp, oracle_mod, spec, prec, 0.005, V0_np, V0, 7)
        print(f"[gpu] full solve {spec.name} fp{prec}", flush=True)
        res = odp.solve(spec, V0, precision=prec, tau=[0.0, 1.5, 3.0], save_all=True)
        torch.cuda.synchronize()
        A = res.V_all
        assert bool((A[1] <= V0).all()) and bool((A[2] <= V0).all())
        # the tube only grows: V(3.0) <= V(1.5) up to small departures (the
        # sign-keeping ghost is not monotone at non-periodic faces and what it
        # does there spreads inwards over ~180 steps; the oracle shows the
        # same at faces), bounded here, not proven
        # (observed: 1.05e-5 in float32, 2.2e-8 in float64; bounds about 10x)
        inc = (A[2] - A[1])
        bound = {32: 1.5e-4, 64: 3e-7}[prec]
        print(f"    max increase V(3.0) - V(1.5): {float(inc.max()):.2e} (bound {bound:.0e}), "
              f"max decrease {float(-inc.min()):.2e}", flush=True)
        assert float(inc.max()) <= bound
        assert bool((A[2] < V0 - 0.05).any())  # the tube grew beyond the target
        outs[prec] = A[2].double().cpu()
        del V0, A, res
        torch.cuda.empty_cache()
    err = float((outs[32] - outs[64]).abs().max())
    print(f"    fp32 vs fp64 full 80^4 solve: max|err| = {err:.3e} (limit {1e-4 * 10:.0e})", flush=True)
    assert err <= 1e-4 * spec.grid.domain_scale()


def test_game6d_36_full_size(odp, oracle_mod):
    import torch
    spec = W.config_game6d()
    print("[gpu] building the 36^6 float64 target on the host", flush=True)
    V0_np = W.make_v0(spec)
    V0 = W.make_v0_torch(spec, torch.device("cuda:0"), torch.float32)
    res = one_step_check(odp, oracle_mod, spec, 32, 0.01, V0_np, V0, 11)
    del res
    torch.cuda.empty_cache()
    print(f"[gpu] full solve {spec.name} fp32 (tube below V0)", flush=True)
    out = odp.solve(spec, V0, precision=32)
    torch.cuda.synchronize()
    assert out.stats["steps"] == 73
    assert bool((out.V <= V0).all())
    assert out.stats["nonfinite"] == 0


def _max_abs_diff(a, b, chunk=1 << 26):
    """max |a - b| in float64 over two device arrays, in chunks."""
    a, b = a.reshape(-1), b.reshape(-1)
    m = 0.0
    for i in range(0, a.numel(), chunk):
        m = max(m, float((a[i:i + chunk].double() - b[i:i + chunk].double()).abs().max()))
    return m


def test_game6d_36_full_horizon_fp32_vs_fp64(odp):
    """The 36^6 game over the whole horizon (T = 2, 73 RK2 steps) in float32
    and in the float64 plain form (3 x 17.4 GB): the float32 solve stays
    within 1e-4 S of the float64 one (whose parity with the oracle is checked
    on smaller grids: the chain of the 6D row)."""
    import torch
    spec = W.config_game6d()
    dev = torch.device("cuda:0")
    print("[gpu] 36^6 full horizon fp32", flush=True)
    V0 = W.make_v0_torch(spec, dev, torch.float32)
    r32 = odp.solve(spec, V0, precision=32)
    torch.cuda.synchronize()
    out32 = r32.V
    del V0, r32
    torch.cuda.empty_cache()
    print("[gpu] 36^6 full horizon fp64", flush=True)
    V0 = W.make_v0_torch(spec, dev, torch.float64)
    r64 = odp.solve(spec, V0, precision=64)
    torch.cuda.synchronize()
    assert r64.stats["steps"] == 73
    err = _max_abs_diff(out32, r64.V)
    S = spec.grid.domain_scale()
    print(f"    fp32 vs fp64, 36^6, T=2: max|err| = {err:.3e} (/S {err / S:.2e}, limit 1e-4)", flush=True)
    assert err <= 1e-4 * S
    del V0, r64, out32
    torch.cuda.empty_cache()


def test_dyncar4d_80_eno2_full_horizon_fp32_vs_fp64(odp):
    """The second-order solve the benchmark times (ENO2 + TVD-RK2, 80^4,
    T = 3, 359 steps) in float32 against float64: within 1e-4 S over the
    whole horizon."""
    import torch
    spec = W.config_dyncar4d()
    spec.rk_order = 2
    V0_np = W.make_v0(spec)
    outs = {}
    for prec, dt in ((32, torch.float32), (64, torch.float64)):
        print(f"[gpu] 80^4 ENO2 RK2 full horizon fp{prec}", flush=True)
        V0 = torch.tensor(V0_np, dtype=dt, device="cuda:0")
        r = odp.solve(spec, V0, precision=prec, space_order=2)
        torch.cuda.synchronize()
        assert r.stats["steps"] == 359
        outs[prec] = r.V
        del V0, r
    err = _max_abs_diff(outs[32], outs[64])
    S = spec.grid.domain_scale()
    print(f"    fp32 vs fp64, ENO2 80^4, T=3: max|err| = {err:.3e} (/S {err / S:.2e}, limit 1e-4)", flush=True)
    assert err <= 1e-4 * S
