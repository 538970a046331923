"""CPU checks of the C ABI: the library loads, exports every function that
include/odp.h declares, and rejects bad arguments before any GPU work.
(No compute call is made here: there is no GPU in this environment.)"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2204_05520_amd as odp
from paper_2204_05520_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "odp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(odp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(odp.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return odp.lib()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 15, names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(odp.SYMBOLS) == names


def test_strerror_covers_codes(lib):
    for code in range(-7, 2):
        assert odp.odp_strerror(code) != "unknown error code"
    assert odp.odp_strerror(-99) == "unknown error code"


@pytest.mark.parametrize("n,lo,hi,msg", [
    ([2, 5], [0, 0], [1, 1], "nodes"),
    ([5, 5], [0, 1], [1, 1], "lo < hi"),
    ([5] * 7, [0] * 7, [1] * 7, "ndim"),
    ([5, 5], [0, float("nan")], [1, 1], "finite"),
])
def test_grid_create_rejects(lib, n, lo, hi, msg):
    with pytest.raises(odp.OdpError) as ei:
        odp.Grid(n, lo, hi, [0] * len(n))
    assert ei.value.code == odp.ODP_EINVAL
    assert msg in str(ei.value)


def test_grid_points_and_limits(lib):
    g = odp.Grid([80, 80, 80, 80], [-5, -5, 0, -3.14], [5, 5, 4, 3.14], [0, 0, 0, 1])
    assert g.npts == 80 ** 4
    with pytest.raises(odp.OdpError):
        odp.Grid([3, 1 << 16, 1 << 16], [0, 0, 0], [1, 1, 1], [0, 0, 0])  # hyperplane >= 2^31


def _solve_rc(spec, precision=32, **kw):
    """odp_hj_solve with fake (never dereferenced) device pointers: every case
    here must fail validation before touching the GPU."""
    grid = odp.Grid.from_spec(spec.grid)
    d = odp.make_dynamics(spec.dyn)
    tau = kw.pop("tau", spec.tau)
    t = (ctypes.c_double * len(tau))(*tau)
    opts = odp.make_opts(precision, kw.pop("rk", spec.rk_order), kw.pop("cfl", spec.cfl),
                         kw.pop("mode", spec.mode), kw.pop("diss", 0), kw.pop("max_dt", 0.0),
                         kw.pop("save_all", 0), kw.pop("tile_chunk", 0), None,
                         obstacle_mode=kw.pop("obstacle_mode", 0), target=kw.pop("target", None),
                         obstacle=kw.pop("obstacle", None), set_slices=kw.pop("set_slices", 0),
                         space_order=kw.pop("space_order", 1))
    V0 = kw.pop("V0", ctypes.c_void_p(0x1000))
    Vout = kw.pop("Vout", ctypes.c_void_p(0x2000))
    rc = odp.lib().odp_hj_solve(grid.handle, ctypes.byref(d), V0, None, t, len(tau),
                                ctypes.byref(opts), None, Vout, None, None)
    return rc, odp.odp_last_error()


@pytest.mark.parametrize("kw,msg", [
    ({"precision": 16}, "precision"),
    ({"rk": 4}, "rk_order"),
    ({"cfl": 1.5}, "cfl"),
    ({"cfl": 0.0}, "cfl"),
    ({"diss": 2}, "dissipation"),
    ({"max_dt": -1.0}, "max_dt"),
    ({"tau": [0.0]}, "tau"),
    ({"tau": [0.0, 1.0, 1.0]}, "increasing"),
    ({"tau": [-1.0, 1.0]}, "tau[0]"),
    ({"save_all": 1}, "V_all"),
    ({"V0": None}, "V0"),
    ({"Vout": ctypes.c_void_p(0x1000)}, "alias"),
    ({"mode": 7}, "mode"),
    ({"mode": -1}, "mode"),
    ({"obstacle_mode": 3, "obstacle": 0x3000}, "obstacle_mode"),
    ({"mode": "minVWithVTarget"}, "needs target_dev"),
    ({"mode": "maxVWithVTarget"}, "needs target_dev"),
    ({"mode": "minVWithV0", "target": 0x3000}, "target_dev is set"),
    ({"obstacle_mode": "maxVWithObstacle"}, "needs obstacle_dev"),
    ({"obstacle": 0x3000}, "obstacle_dev is set"),
    ({"mode": "minVWithVTarget", "target": 0x2000}, "alias"),
    ({"obstacle_mode": 2, "obstacle": 0x2000}, "alias"),
    ({"set_slices": 2}, "set_slices needs"),
    ({"set_slices": -1}, "set_slices needs"),
    ({"mode": 5, "target": 0x3000, "set_slices": 3}, "set_slices must be"),
    ({"space_order": 3}, "space_order"),
    ({"space_order": -1}, "space_order"),
])
def test_solve_rejects_before_gpu(lib, kw, msg):
    spec = W.config_dubins3d(n=(10, 10, 8))
    rc, err = _solve_rc(spec, **kw)
    assert rc == odp.ODP_EINVAL
    assert msg in err


def test_dynamics_checks(lib):
    spec = W.config_dubins3d(n=(10, 10, 8))
    spec.dyn.params = [1.0, -1.0]
    rc, err = _solve_rc(spec)
    assert rc == odp.ODP_EINVAL and "w_max" in err
    spec = W.config_dubins3d(n=(10, 10, 8))
    spec.grid.periodic = [0, 0, 0]
    rc, err = _solve_rc(spec)
    assert rc == odp.ODP_EINVAL and "periodic" in err
    spec = W.config_dubins3d(n=(10, 10, 8))
    spec.dyn.id = W.DYN_DYNCAR4D
    rc, err = _solve_rc(spec)
    assert rc == odp.ODP_EINVAL and "dimension" in err
    spec.dyn.id = 7
    rc, err = _solve_rc(spec)
    assert rc == odp.ODP_EINVAL


def test_workspace_bytes(lib):
    spec = W.config_dyncar4d()
    grid = odp.Grid.from_spec(spec.grid)
    o32 = odp.make_opts(32, 3)
    o64 = odp.make_opts(64, 3)
    b32 = odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, o32)
    b64 = odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, o64)
    P = 80 ** 4
    # RK3: two stage buffers beside the caller's arrays, plus schedule/tables
    assert 2 * 4 * P <= b32 < 2 * 4 * P + (8 << 20)
    assert 2 * 8 * P <= b64 < 2 * 8 * P + (8 << 20)
    o1 = odp.make_opts(32, 1)
    b1 = odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, o1)
    assert 4 * P <= b1 < 4 * P + (8 << 20)
    assert odp.odp_hj_workspace_bytes(grid, spec.dyn, [1.0, 0.5], o32) == 0


def test_tile_chunk_values(lib):
    """tile_chunk: >= 0 or the autotune sentinel; with autotune the workspace
    query covers every candidate tiling."""
    spec = W.config_dyncar4d(n=(24, 20, 16, 12))
    grid = odp.Grid.from_spec(spec.grid)
    fixed = odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau, odp.make_opts(32, 3, tile_chunk=4))
    auto = odp.odp_hj_workspace_bytes(grid, spec.dyn, spec.tau,
                                      odp.make_opts(32, 3, tile_chunk=odp.ODP_TILE_AUTOTUNE))
    assert fixed > 0 and auto >= fixed
    rc, err = _solve_rc(spec, tile_chunk=-2)
    assert rc == odp.ODP_EINVAL and "tile_chunk" in err


def test_batch_and_server_reject(lib):
    specs = [W.config_dubins3d(n=(10, 10, 8))]
    descs = (odp.odp_solve_desc * 1)()
    grid = odp.Grid.from_spec(specs[0].grid)
    descs[0].grid = grid.handle
    descs[0].dyn = odp.make_dynamics(specs[0].dyn)
    descs[0].V0_dev = 0x1000
    t = (ctypes.c_double * 2)(0.0, 1.0)
    descs[0].tau = ctypes.cast(t, ctypes.POINTER(ctypes.c_double))
    descs[0].ntau = 2
    descs[0].V_out_dev = 0x1000  # aliases V0
    opts = odp.make_opts(32, 1)
    rc = lib.odp_hj_batch(1, descs, ctypes.byref(opts), None, 0, None)
    assert rc == odp.ODP_EINVAL
    assert lib.odp_hj_batch(0, descs, ctypes.byref(opts), None, 0, None) == odp.ODP_EINVAL
    bad = odp.make_opts(32, 1, save_all=1)
    h = ctypes.c_void_p()
    assert lib.odp_server_create(1 << 20, 4, ctypes.byref(bad), ctypes.byref(h)) == odp.ODP_EUNSUPPORTED
    assert lib.odp_server_create(1 << 20, 0, ctypes.byref(opts), ctypes.byref(h)) == odp.ODP_EINVAL
    assert lib.odp_server_create(0, 4, ctypes.byref(opts), ctypes.byref(h)) == odp.ODP_EINVAL


def test_fastdiv_magic_numbers():
    """The round-up magic-number division the kernels use for the in-plane
    index (host formula, checked against integer division)."""
    rng = np.random.default_rng(0)
    for d in list(range(1, 300)) + [36 ** 4, 80 ** 3, 6400, 46656]:
        s = 0
        while (1 << s) < d:
            s += 1
        m = ((1 << 32) * ((1 << s) - d)) // d + 1
        for n in [0, d - 1, d, d + 1, (1 << 31) - 1] + list(rng.integers(0, 1 << 31, 50)):
            assert ((((int(n) * m) >> 32) + int(n)) >> s) == int(n) // d


def test_product_path_has_no_oracle_import():
    """The library binding never imports the oracle (test infrastructure)."""
    for f in ("__init__.py", "workloads.py", "build.py"):
        src = open(os.path.join(ROOT, "paper_2204_05520_amd", f)).read()
        assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2204_05520_amd", "csrc")):
        src = open(os.path.join(ROOT, "paper_2204_05520_amd", "csrc", f)).read()
        assert "oracle" not in src.lower(), f


def test_struct_layout_matches_header(lib, tmp_path):
    """The ctypes mirrors have the C structs' sizes and field offsets (checked
    by compiling the header with gcc)."""
    structs = {"odp_solve_opts": odp.odp_solve_opts, "odp_solve_stats": odp.odp_solve_stats,
               "odp_dynamics": odp.odp_dynamics, "odp_solve_desc": odp.odp_solve_desc,
               "odp_ttr_opts": odp.odp_ttr_opts, "odp_ttr_stats": odp.odp_ttr_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "odp.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])


def test_method_names(lib):
    assert odp.method_code("None") == odp.ODP_BRS
    assert odp.method_code("minVWithV0") == odp.ODP_BRT
    assert [odp.method_code(m) for m in ("maxVWithV0", "minVWithVInit", "maxVWithVInit",
                                         "minVWithVTarget", "maxVWithVTarget")] == [2, 3, 4, 5, 6]
    assert odp.obstacle_code("maxVWithObstacle") == 2 and odp.obstacle_code("minVWithObstacle") == 1


def test_batch_and_server_reject_method_arrays(lib):
    spec = W.config_dubins3d(n=(10, 10, 8))
    grid = odp.Grid.from_spec(spec.grid)
    t = (ctypes.c_double * len(spec.tau))(*spec.tau)
    desc = odp.odp_solve_desc()
    desc.grid = grid.handle
    desc.dyn = odp.make_dynamics(spec.dyn)
    desc.V0_dev = 0x1000
    desc.tau = ctypes.cast(t, ctypes.POINTER(ctypes.c_double))
    desc.ntau = len(spec.tau)
    desc.V_out_dev = 0x2000
    for kw in ({"mode": 5, "target": 0x3000}, {"obstacle_mode": 2, "obstacle": 0x3000}):
        opts = odp.make_opts(32, 1, 0.8, kw.get("mode", 1), obstacle_mode=kw.get("obstacle_mode", 0),
                             target=kw.get("target"), obstacle=kw.get("obstacle"))
        rc = odp.lib().odp_hj_batch(1, ctypes.byref(desc), ctypes.byref(opts), None, 0, None)
        assert rc == odp.ODP_EUNSUPPORTED and "one grid" in odp.odp_last_error()
        assert odp.lib().odp_hj_batch_workspace_bytes(1, ctypes.byref(desc), ctypes.byref(opts)) == 0
        srv = ctypes.c_void_p()
        rc = odp.lib().odp_server_create(1 << 30, 4, ctypes.byref(opts), ctypes.byref(srv))
        assert rc == odp.ODP_EUNSUPPORTED and not srv.value


@pytest.mark.parametrize("kw,code,msg", [
    ({"precision": 16}, -1, "precision"),
    ({"eps": 0.0}, -1, "eps"),
    ({"max_iters": 0}, -1, "max_iters"),
    ({"check_every": -1}, -1, "check_every"),
    ({"big": -1.0}, -1, "big"),
    ({"alias": True}, -1, "alias"),
    ({"pe3d": True}, -4, "pursuit-evasion"),
])
def test_ttr_rejects_before_gpu(lib, kw, code, msg):
    spec = W.config_dubins3d(n=(10, 10, 8))
    if kw.pop("pe3d", False):
        spec = W.config_pe3d(n=[10, 10, 8])
    grid = odp.Grid.from_spec(spec.grid)
    d = odp.make_dynamics(spec.dyn)
    alias = kw.pop("alias", False)
    o = odp.make_ttr_opts(**kw)
    rc = odp.lib().odp_ttr_solve(grid.handle, ctypes.byref(d), ctypes.c_void_p(0x1000), ctypes.byref(o),
                                 None, 0, ctypes.c_void_p(0x1000 if alias else 0x2000), None)
    assert rc == code and msg in odp.odp_last_error()


def test_ttr_workspace_bytes(lib):
    spec = W.config_dubins3d(n=(100, 100, 100))
    grid = odp.Grid.from_spec(spec.grid)
    b32 = odp.lib().odp_ttr_workspace_bytes(grid.handle, ctypes.byref(odp.make_ttr_opts(32)))
    b64 = odp.lib().odp_ttr_workspace_bytes(grid.handle, ctypes.byref(odp.make_ttr_opts(64)))
    assert 4 * 10**6 <= b32 < 4 * 10**6 + (1 << 20)
    assert 8 * 10**6 <= b64 < 8 * 10**6 + (1 << 20)
