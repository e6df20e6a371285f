"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pbgpu.h declares, the ctypes structs match the C
layout, workspace queries are sane and bad arguments are rejected before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbgpu.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pb_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def pbgpu():
    import paper_1704_02745_amd as m
    return m


def test_every_declared_symbol_is_exported(pbgpu):
    names = _declared()
    assert "pb_solve" in names and "pb_setup" in names and "pb_energy" in names
    lib = ctypes.CDLL(pbgpu.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pbgpu.EXPORTS)


def test_struct_layouts(pbgpu):
    assert ctypes.sizeof(pbgpu.Grid) == 48
    assert ctypes.sizeof(pbgpu.SolveOpts) == 40
    assert ctypes.sizeof(pbgpu.Info) == 56 and pbgpu.Info.coded_launches.offset == 48
    assert pbgpu.SolveOpts.inner_tol.offset == 24
    assert pbgpu.Info.relres_recur.offset == 16
    assert ctypes.sizeof(pbgpu.Tuning) == 40
    assert pbgpu.Tuning.us_per_iter.offset == 16 and pbgpu.Tuning.scheme.offset == 28
    assert pbgpu.Tuning.streaming.offset == 32


def test_version(pbgpu):
    assert "gfx950" in pbgpu.version()


def test_workspace_queries(pbgpu):
    lib = pbgpu.lib
    g = pbgpu.make_grid(33, 33, 33, 0.5, (0, 0, 0))
    assert lib.pb_setup_workspace_bytes(ctypes.byref(g), 50) > 33 ** 3 * 8
    bad = pbgpu.make_grid(1, 33, 33, 0.5, (0, 0, 0))
    assert lib.pb_setup_workspace_bytes(ctypes.byref(bad), 50) == 0
    assert lib.pb_setup_workspace_bytes(ctypes.byref(g), -1) == 0
    n32 = pbgpu.solve_workspace_bytes(257, 257, 257, "f32")
    n64 = pbgpu.solve_workspace_bytes(257, 257, 257, "f64")
    dia = pbgpu.solve_workspace_bytes(257, 257, 257, "f32", op="dia")
    assert 257 ** 3 * 80 < n32 < 257 ** 3 * 120
    assert n64 > 257 ** 3 * 80 and dia > n32 + 5 * 4 * 257 ** 3
    assert pbgpu.solve_workspace_bytes(0, 5, 5) == 0
    o = pbgpu.SolveOpts()
    o.tol = -1.0
    assert lib.pb_solve_workspace_bytes(5, 5, 5, ctypes.byref(o)) == 0
    assert lib.pb_energy_workspace_bytes(10) > 0 and lib.pb_energy_workspace_bytes(-3) == 0


def test_bad_arguments_rejected_on_host(pbgpu):
    lib = pbgpu.lib
    o = pbgpu.SolveOpts()
    o.tol = 1e-6
    info = pbgpu.Info()
    dummy = ctypes.c_void_p(256)
    st = lib.pb_solve(0, 4, 4, 0.5, dummy, dummy, dummy, dummy, dummy, dummy, ctypes.byref(o), dummy, 1 << 20,
                      None, ctypes.byref(info))
    assert st == pbgpu.PB_ERR_ARG and "dims" in pbgpu.last_error()
    st = lib.pb_solve(4, 4, 4, -0.5, dummy, dummy, dummy, dummy, dummy, dummy, ctypes.byref(o), dummy, 1 << 20,
                      None, ctypes.byref(info))
    assert st == pbgpu.PB_ERR_ARG
    o.tol = 0.0
    st = lib.pb_solve(4, 4, 4, 0.5, dummy, dummy, dummy, dummy, dummy, dummy, ctypes.byref(o), dummy, 1 << 20,
                      None, ctypes.byref(info))
    assert st == pbgpu.PB_ERR_ARG
    o.tol = 1e-6
    st = lib.pb_solve(4, 4, 4, 0.5, dummy, None, dummy, dummy, dummy, dummy, ctypes.byref(o), dummy, 1 << 20,
                      None, ctypes.byref(info))
    assert st == pbgpu.PB_ERR_ARG
    # misaligned workspace
    st = lib.pb_solve(4, 4, 4, 0.5, dummy, dummy, dummy, dummy, dummy, dummy, ctypes.byref(o),
                      ctypes.c_void_p(1000), 1 << 20, None, ctypes.byref(info))
    assert st == pbgpu.PB_ERR_ARG
    # workspace too small is reported before any launch
    st = lib.pb_solve(4, 4, 4, 0.5, dummy, dummy, dummy, dummy, dummy, dummy, ctypes.byref(o), dummy, 16,
                      None, ctypes.byref(info))
    assert st == pbgpu.PB_ERR_NOMEM
    g = pbgpu.make_grid(5, 5, 5, 0.5, (0, 0, 0))
    st = lib.pb_setup(ctypes.byref(g), 1, dummy, dummy, dummy, -1.0, 80.0, 0.0, dummy, dummy, dummy, dummy,
                      dummy, None, None, dummy, 1 << 30, None)
    assert st == pbgpu.PB_ERR_ARG and "dielectric" in pbgpu.last_error()
    e = ctypes.c_double()
    st = lib.pb_energy(ctypes.byref(g), 3, dummy, dummy, dummy, None, ctypes.byref(e), dummy, 8, None)
    assert st == pbgpu.PB_ERR_NOMEM


def test_tuning_queries_reject_bad_arguments_on_host(pbgpu):
    lib = pbgpu.lib
    t = pbgpu.Tuning()
    n = ctypes.c_int32(-1)
    assert lib.pb_get_tuning(33, 33, 33, pbgpu.PRECISIONS["f32"], None) == pbgpu.PB_ERR_ARG
    assert lib.pb_get_tuning(0, 33, 33, pbgpu.PRECISIONS["f32"], ctypes.byref(t)) == pbgpu.PB_ERR_ARG
    assert lib.pb_get_tuning(33, 33, 33, 7, ctypes.byref(t)) == pbgpu.PB_ERR_ARG
    assert lib.pb_tiling_candidates(33, 33, 33, pbgpu.PRECISIONS["f32"], None, 0, None) == pbgpu.PB_ERR_ARG
    assert lib.pb_tiling_candidates(33, 33, 33, pbgpu.PRECISIONS["f32"], None, 4, ctypes.byref(n)) == pbgpu.PB_ERR_ARG
    assert lib.pb_set_tuning(33, 33, 33, pbgpu.PRECISIONS["f32"], None) == pbgpu.PB_ERR_ARG
    assert n.value == -1


def test_coded_coefficient_switch(pbgpu):
    """The process-wide switch of the coded pass is host state: on by default,
    off and on again without a device."""
    assert pbgpu.get_coded_coefficients() is True
    try:
        pbgpu.set_coded_coefficients(False)
        assert pbgpu.get_coded_coefficients() is False
        assert pbgpu.lib.pb_get_coded_coefficients() == 0
    finally:
        pbgpu.set_coded_coefficients(True)
    assert pbgpu.lib.pb_get_coded_coefficients() == 1
