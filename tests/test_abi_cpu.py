"""CPU tests of the C ABI library: it loads, exports every symbol the header
declares, validates hierarchies on the host and lays them out the way the oracle's
independent plan does.  No compute calls (no GPU here)."""

import ctypes
import os
import re

import numpy as np
import pytest

import apm_workloads as W
from apm_workloads import GridSpec
from oracle import apm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apm.h")

P = pytest.importorskip("paper_1410_0010_amd")
from paper_1410_0010_amd import _apm  # noqa: E402


def _declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(apm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_apm.LIB_PATH)
    syms = _declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(_apm.SIGNATURES), set(syms) ^ set(_apm.SIGNATURES)


def test_library_is_gfx950_code_object():
    data = open(_apm.LIB_PATH, "rb").read()
    assert b"gfx950" in data


@pytest.mark.parametrize("wl", [
    lambda: W.workload_root32_uniform_gas(),
    lambda: W.workload_plummer_nested(root_n=128, sub_n=64, nlevels=2, npart=10),
    lambda: W.workload_clumps(ngrids=12, per_clump=10),
    lambda: W.workload_large_nested(npart=10, with_velocities=False),
    lambda: W.workload_sine_wave(ntracer=10),
    lambda: W.workload_plummer_periodic(npart=10),
])
def test_layout_matches_oracle_plan(wl):
    w = wl()
    plan = P.Plan(w.root_n, w.grids, boundary=w.boundary)
    op = O.OraclePlan(w.root_n, w.grids, boundary=w.boundary)
    assert plan.ngrids == len(op.grids)
    assert plan.nlevels == op.nlevels
    for g, og in zip(plan.grids, op.grids):
        assert list(og.gmf_lo) == g["gmf_lo"] and list(og.gmf_n) == g["gmf_n"]
        assert list(og.fld_lo) == g["fld_lo"] and list(og.fld_n) == g["fld_n"]
        assert list(og.M) == g["fft_n"]
        assert g["dx"] == og.dx
    for l in range(plan.nlevels):
        gs = op.level_grids(l)
        assert plan.levels[l]["gmf_elems"] == sum(int(np.prod(g.gmf_n)) for g in gs)
        assert plan.levels[l]["fld_cells"] == sum(int(np.prod(g.fld_n)) for g in gs)


def test_bench_workload_fft_sizes():
    """Root 128^3 uses the 256^3 doubled mesh; 64^3 subgrids (70^3 GMF + 5 padding)
    use 128^3 (Sec. 2.2 padding of 0.65 R a/dx cells, power-of-two lengths)."""
    plan = P.Plan(128, W.centred_nested_grids(128, 64, 2))
    assert plan.grids[0]["fft_n"] == [256] * 3
    assert plan.grids[1]["fft_n"] == [128] * 3 and plan.grids[1]["gmf_n"] == [70] * 3


def test_periodic_root_fft_is_not_doubled():
    """A periodic root needs no zero padding (Sec. 2.1): its FFT is root_n long, so a
    1024^3 periodic root is accepted while an isolated one (2048) is not."""
    plan = P.Plan(128, W.centred_nested_grids(128, 64, 2), boundary="periodic")
    assert plan.grids[0]["fft_n"] == [128] * 3
    assert plan.grids[1]["fft_n"] == [128] * 3
    big = P.Plan(1024, [GridSpec(0, -1, (0, 0, 0), (1024,) * 3)], boundary="periodic")
    assert big.grids[0]["fft_n"] == [1024] * 3
    assert _bad([GridSpec(0, -1, (0, 0, 0), (1024,) * 3)], root_n=1024) == _apm.APM_ERR_RANGE
    cfg = _apm.apm_config()
    P.lib().apm_config_default(ctypes.byref(cfg))
    assert cfg.boundary == _apm.APM_BC_ISOLATED
    cfg.root_n = 16
    cfg.boundary = 7
    arr = (_apm.apm_grid * 1)()
    arr[0].level, arr[0].parent = 0, -1
    for a in range(3):
        arr[0].n[a] = 16
    h = ctypes.c_void_p()
    assert P.lib().apm_plan_create(ctypes.byref(cfg), arr, 1, ctypes.byref(h)) == _apm.APM_ERR_INVALID
    cfg.boundary = _apm.APM_BC_ISOLATED
    cfg.strict = 2
    assert P.lib().apm_plan_create(ctypes.byref(cfg), arr, 1, ctypes.byref(h)) == _apm.APM_ERR_INVALID
    cfg.strict = 1
    cfg.deposit_accum = 2
    assert P.lib().apm_plan_create(ctypes.byref(cfg), arr, 1, ctypes.byref(h)) == _apm.APM_ERR_INVALID
    cfg.deposit_accum = _apm.APM_ACC_F32_COMP
    assert P.lib().apm_plan_create(ctypes.byref(cfg), arr, 1, ctypes.byref(h)) == _apm.APM_OK
    P.lib().apm_plan_destroy(h)


def _bad(grids, root_n=16, **kw):
    with pytest.raises(P.APMError) as e:
        P.Plan(root_n, grids, **kw)
    return e.value.status


def test_plan_validation_errors():
    root = GridSpec(0, -1, (0, 0, 0), (16,) * 3)
    assert _bad([root], root_n=12) == _apm.APM_ERR_INVALID           # not a power of two
    assert _bad([root], root_n=1024) == _apm.APM_ERR_RANGE           # 2048 FFT
    assert _bad([GridSpec(0, -1, (0, 0, 0), (8,) * 3)]) == _apm.APM_ERR_INVALID
    assert _bad([root, GridSpec(1, 0, (3, 8, 8), (8, 8, 8))]) == _apm.APM_ERR_INVALID   # odd lo
    assert _bad([root, GridSpec(1, 0, (8, 8, 8), (7, 8, 8))]) == _apm.APM_ERR_INVALID   # odd n
    assert _bad([root, GridSpec(1, 0, (2, 8, 8), (8, 8, 8))]) == _apm.APM_ERR_INVALID   # margin
    assert _bad([root, GridSpec(1, 0, (8, 8, 8), (22, 8, 8))]) == _apm.APM_ERR_INVALID  # margin hi
    assert _bad([root, GridSpec(2, 0, (8, 8, 8), (8, 8, 8))]) == _apm.APM_ERR_INVALID   # level jump
    assert _bad([root, GridSpec(1, 1, (8, 8, 8), (8, 8, 8))]) == _apm.APM_ERR_INVALID   # self parent
    assert _bad([root], G=-1.0) == _apm.APM_ERR_INVALID
    assert _bad([root], ghost=1) == _apm.APM_ERR_INVALID
    # subgrid FFT length beyond 1024
    big = [GridSpec(0, -1, (0, 0, 0), (512,) * 3), GridSpec(1, 0, (4, 8, 8), (1014, 8, 8))]
    assert _bad(big, root_n=512) == _apm.APM_ERR_RANGE
    # the particle sort keys 8^3 tiles of the finest level in 64 bits: at most 2^24
    # cells per axis there (root 32 and 19 levels of refinement), one level more fails
    P.Plan(32, W.centred_nested_grids(32, 16, 19))
    assert _bad(W.centred_nested_grids(32, 16, 20), root_n=32) == _apm.APM_ERR_RANGE


def test_plan_accepts_paper_geometries():
    for w in (W.workload_self_force(), W.workload_orbit(2), W.workload_orbit(4),
              W.workload_point_source(False, ntest=3), W.workload_point_source(True, ntest=3),
              W.workload_uniform_sphere()):
        P.Plan(w.root_n, w.grids)


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    plan = P.Plan(16, [GridSpec(0, -1, (0, 0, 0), (16,) * 3)])
    h = ctypes.c_void_p()
    st = P.lib().apm_create(plan.handle, 0, None, ctypes.byref(h))
    assert st == _apm.APM_ERR_DEVICE
    assert b"device" in P.lib().apm_last_error()


def test_null_arguments_rejected_on_host():
    lib = P.lib()
    assert lib.apm_plan_create(None, None, 0, None) == _apm.APM_ERR_INVALID
    assert lib.apm_plan_nlevels(None) == -1
    assert lib.apm_owner(None, _apm.APM_F32, None, None, None, 0, None) == _apm.APM_ERR_INVALID
    assert lib.apm_solve(None, _apm.APM_F64, None, None, None, None, 0, None, None, None, None,
                         None) == _apm.APM_ERR_INVALID
    assert lib.apm_field_ptr(None, _apm.APM_F32, 0) is None
