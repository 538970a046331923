"""Tile coverage on the GPU: one step of negligible size (tau = 1e-30, far
below every value's rounding) on index-valued data (point i holds i + 1,
exact in float32 up to 2^24) must leave every output point holding its own
value: a point that no tile wrote keeps the output buffer's fill (NaN), one
written from the wrong place holds another index.  Every launch form: single
solves with several axis-0 chunkings (runs shorter than the 4-plane cycle,
ragged last runs), both spatial orders, row-major, brick and quad tiles, the
point-per-lane kernel, batches with padded rows, the server."""
import time

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


def _spec(name, n, dyn):
    nd = len(n)
    per = [0] * nd
    if dyn.id in (W.DYN_DUBINS3D, W.DYN_PE3D):
        per[2] = 1
    elif dyn.id == W.DYN_DYNCAR4D:
        per[3] = 1
    elif dyn.id == W.DYN_TWODUBINS6D:
        per[2] = per[5] = 1
    g = W.GridSpec(list(n), [-4.0] * nd, [4.0] * nd, per)
    return W.SolveSpec(g, dyn, [0.0, 1e-30], rk_order=1, cfl=0.8, mode=W.BRS, name=name)


CASES = [
    ("si2d", [37, 45], W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [1.0, 0.3, -0.2], W.MAXIMISE, W.MINIMISE)),
    ("dubins3d", [23, 29, 22], W.DynSpec(W.DYN_DUBINS3D, [1.0, 1.0], W.MAXIMISE, W.MINIMISE)),
    ("dyncar4d", [13, 11, 9, 18], W.DynSpec(W.DYN_DYNCAR4D, [1.0, 1.0], W.MAXIMISE, W.MINIMISE)),
    ("si5d", [7, 6, 5, 9, 11], W.DynSpec(W.DYN_SINGLE_INTEGRATOR, [1.0], W.MINIMISE, W.MINIMISE)),
    ("game6d", [7, 6, 5, 6, 7, 10], W.DynSpec(W.DYN_TWODUBINS6D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)),
    # cubes of axes 3..5 of 11200 and 20736 points: first order takes quad
    # tiles (6x6 squares of axes 1 and 2) and brick tiles (3x3 squares)
    ("game6d_quad", [4, 6, 6, 20, 20, 28],
     W.DynSpec(W.DYN_TWODUBINS6D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)),
    ("game6d_brick3", [3, 9, 3, 24, 24, 36],
     W.DynSpec(W.DYN_TWODUBINS6D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)),
    ("pe3d", [21, 19, 14], W.DynSpec(W.DYN_PE3D, [1.0, 1.0, 1.0, 1.0], W.MAXIMISE, W.MINIMISE)),
]


def _index_field(spec, dtype):
    import torch
    return (torch.arange(spec.grid.npts, dtype=torch.float64) + 1.0).to(dtype).reshape(tuple(spec.grid.n)).cuda()


@pytest.mark.parametrize("name,n,dyn", CASES, ids=[c[0] for c in CASES])
def test_every_point_written_once_with_its_value(odp, name, n, dyn):
    import torch
    spec = _spec(name, n, dyn)
    for prec, dt in ((32, torch.float32), (64, torch.float64)):
        V = _index_field(spec, dt)
        for order in (1, 2):
            for chunk in (0, 1, 2, 3, 5, 13):
                print(f"[gpu] coverage {name} {n} fp{prec} order {order} chunk {chunk}", flush=True)
                res = odp.solve(spec, V, precision=prec, tile_chunk=chunk, space_order=order)
                torch.cuda.synchronize()
                assert res.stats["steps"] == 1
                assert torch.equal(res.V, V), (name, prec, order, chunk)


def test_batch_and_server_cover_every_point(odp):
    """Members with rows that are not whole 16-byte vectors run on padded
    copies (batch) or padded pitches (server); their dense results hold
    every point's own value."""
    import torch
    specs = [_spec("b0", [19, 23, 13], CASES[1][2]), _spec("b1", [11, 9, 7, 10], CASES[2][2]),
             _spec("b2", [17, 21, 15], CASES[1][2]), _spec("b3", [9, 8, 6, 5], CASES[2][2])]
    V = [_index_field(s, torch.float32) for s in specs]
    outs, _ = odp.batch(specs, V, precision=32)
    torch.cuda.synchronize()
    for s, v, o in zip(specs, V, outs):
        assert torch.equal(o, v), s.name
    srv = odp.Server(1 << 30, 4, precision=32, rk_order=1)
    try:
        tickets = [srv.submit(s, v.cpu().numpy()) for s, v in zip(specs, V)]
        for s, v, t in zip(specs, V, tickets):
            out = np.full(tuple(s.grid.n), np.nan, np.float32)
            t0 = time.time()
            while True:
                rc, _ = srv.poll(t, out)
                if rc != odp.ODP_PENDING:
                    break
                assert time.time() - t0 < 60
                time.sleep(0.002)
            assert rc == odp.ODP_OK
            assert np.array_equal(out, v.cpu().numpy()), s.name
    finally:
        srv.close()
