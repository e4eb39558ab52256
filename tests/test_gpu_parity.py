"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every stage is compared on the same seeded inputs: the GMF of every grid, the own
(short-range) field, the composed field, the owner grid (exact), the particle
accelerations and potentials, and the FP64 totals.  Tolerances (relative L2 of
acceleration and potential): 1e-12 in FP64, 1e-5 in FP32; deposited mass 1e-6.
FP32 runs feed the FP32-rounded inputs to both sides.
"""

import math
import sys

import numpy as np
import pytest

import apm_workloads as W
from apm_workloads import GridSpec
from oracle import apm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_1410_0010_amd")

DEV = torch.device("cuda", 0)
TOL = {np.float64: dict(gmf=1e-13, field=1e-12, acc=1e-12, pot=1e-12, mass=1e-12),
       np.float32: dict(gmf=1e-6, field=1e-5, acc=1e-5, pot=1e-5, mass=1e-6)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype))).to(DEV)


def run_staged(w, dtype, gradient="spectral", accum="f64"):
    plan = P.Plan(w.root_n, w.grids, gradient=gradient, boundary=w.boundary, deposit_accum=accum)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, dtype) for a in (w.x, w.y, w.z, w.m))
    tdt = x.dtype
    gas = [ctx.pack_gas(l, w.gas, tdt) for l in range(plan.nlevels)]
    owner = ctx.owner(x, y, z)
    gmf = [ctx.deposit(l, x, y, z, m, gas[l], gas[l - 1] if l > 0 else None)
           for l in range(plan.nlevels)]
    own = [ctx.solve_level(l, gmf[l]) for l in range(plan.nlevels)]
    fld = []
    for l in range(plan.nlevels):
        fld.append(ctx.accel(l, own[l], fld[l - 1] if l > 0 else None))
    n = w.npart
    ax, ay, az, pot = (torch.zeros(n, dtype=tdt, device=DEV) for _ in range(4))
    for l in range(plan.nlevels):
        ctx.interp(l, fld[l], x, y, z, owner, ax, ay, az, pot)
    tot = ctx.totals(gmf, m, owner, ax, ay, az, pot)
    torch.cuda.synchronize()
    out = dict(plan=plan, ctx=ctx,
               gmf=[ctx.gmf_view(gmf[g["level"]], g["index"]).cpu().numpy() for g in plan.grids],
               own=[ctx.field_view(own[g["level"]], g["index"]).cpu().numpy() for g in plan.grids],
               field=[ctx.field_view(fld[g["level"]], g["index"]).cpu().numpy() for g in plan.grids],
               owner=owner.cpu().numpy(),
               acc=np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], 1),
               pot=pot.cpu().numpy(), totals=tot, tensors=(x, y, z, m, gas))
    return out


def run_oracle(w, dtype, gradient="spectral", cache=None):
    cast = lambda a: None if a is None else np.asarray(a, dtype).astype(np.float64)
    plan = O.OraclePlan(w.root_n, w.grids, gradient=gradient, boundary=w.boundary)
    return O.solve(plan, cast(w.x), cast(w.y), cast(w.z), cast(w.m),
                   [cast(g) for g in w.gas], cache=cache)


def compare(name, w, dtype, got, ref):
    t = TOL[dtype]
    assert np.array_equal(got["owner"], ref["owner"]), f"{name}: owner grids differ"
    for i in range(len(ref["gmf"])):
        e = rel(got["gmf"][i], ref["gmf"][i])
        assert e <= t["gmf"], f"{name}: grid {i} GMF rel L2 {e:.3e}"
        for key in ("own", "field"):
            refk = ref["short"][i] if key == "own" else ref["field"][i]
            ea = rel(got[key][i][..., :3], refk[..., :3])
            ep = rel(got[key][i][..., 3], refk[..., 3])
            assert ea <= t["field"] and ep <= t["field"], \
                f"{name}: grid {i} {key} rel L2 acc {ea:.3e} pot {ep:.3e}"
    if w.npart:
        own = ref["owner"] >= 0
        ea = rel(got["acc"][own], ref["acc"][own])
        ep = rel(got["pot"][own], ref["pot"][own])
        assert ea <= t["acc"], f"{name}: particle acc rel L2 {ea:.3e}"
        assert ep <= t["pot"], f"{name}: particle pot rel L2 {ep:.3e}"
        assert np.all(got["acc"][~own] == 0)
    nl = got["plan"].nlevels
    plan = O.OraclePlan(w.root_n, w.grids)
    for l in range(nl):
        mref = sum(ref["mass"][g.index] for g in plan.level_grids(l))
        assert abs(got["totals"][l] - mref) <= t["mass"] * abs(mref), f"{name}: level {l} mass"
    if w.npart:
        m64 = np.asarray(w.m, dtype).astype(np.float64)
        own = ref["owner"] >= 0
        wref = 0.5 * np.sum(m64[own] * ref["pot"][own])
        assert abs(got["totals"][nl] - wref) <= 10 * t["pot"] * abs(wref)
        fref = (m64[own, None] * ref["acc"][own]).sum(0)
        scale = np.abs(m64[own, None] * ref["acc"][own]).sum()
        assert np.abs(got["totals"][nl + 1:nl + 4] - fref).max() <= 10 * t["acc"] * scale


def slab_workload(npart=3000, seed=77, axis=0):
    """Root 64^3 and a chain of thin slab grids (8 cells thick) reaching level 4 with
    FFT lengths 256, 512 and 1024 along `axis` and 32 across: axis 0 runs the row
    passes at those lengths, axis 1 the y column passes, axis 2 the z pass."""
    grids = [GridSpec(0, -1, (0, 0, 0), (64,) * 3)]
    spans = [(4, 120), (12, 232), (28, 456), (60, 904)]
    for lev, (lo, n) in enumerate(spans, start=1):
        c = 32 * 2 ** lev
        los, ns = [c - 4] * 3, [8] * 3
        los[axis], ns[axis] = lo, n
        grids.append(GridSpec(lev, lev - 1, tuple(los), tuple(ns)))
    rng = np.random.default_rng(seed)
    p = [0.5 + rng.normal(0, 0.002, npart) for _ in range(3)]
    p[axis] = rng.uniform(0.08, 0.92, npart)
    m = rng.uniform(0.5, 1.5, npart) / npart
    return W.Workload(f"slab_chain_axis{axis}", 64, grids, p[0], p[1], p[2], m,
                      [None] * len(grids))


def tiny_grid_workload():
    """Root 16^3 plus subgrids of 4, 6 and 10 cells per axis (FFT lengths 16 and 32)."""
    grids = [GridSpec(0, -1, (0, 0, 0), (16,) * 3),
             GridSpec(1, 0, (8, 10, 12), (4, 6, 10)),
             GridSpec(1, 0, (18, 16, 8), (10, 4, 4))]
    rng = np.random.default_rng(5)
    p = rng.uniform(0.2, 0.8, (3000, 3))
    return W.Workload("tiny_grids", 16, grids, p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(),
                      np.full(3000, 1.0 / 3000), [None] * 3)


def edge_workload():
    """Particles outside the domain, NaN, on the last cell, and exactly on cell
    corners; a particle at x = 0."""
    grids = W.centred_nested_grids(16, 8, 1)
    x = np.array([0.5, 0.5, -0.01, np.nan, 0.999999, 0.0, 0.25, 1.0, 0.53125])
    y = np.array([0.5, 0.47, 0.5, 0.5, 0.5, 0.3, 0.25, 0.5, 0.46875])
    z = np.array([0.5, 0.52, 0.5, 0.5, 0.5, 0.7, 0.25, 0.5, 0.5])
    m = np.array([1.0, 0.5, 1.0, 1.0, 0.1, 0.2, 0.3, 1.0, 0.7])
    return W.Workload("edge", 16, grids, x, y, z, m, [None] * 2)


def clustered_workload(seed=80, boundary="isolated"):
    """Extreme clustering: 5000 particles at one point and 5000 inside one cell of the
    subgrid, 3000 at one point of the root outside it, 500 spread out.  The hot tiles
    hold several deposit chunks whose entries all share a cell."""
    grids = W.centred_nested_grids(16, 8, 1)
    rng = np.random.default_rng(seed)
    p = np.concatenate([np.tile([0.5 + 0.3 / 32, 0.5 - 0.1 / 32, 0.5 + 0.7 / 32], (5000, 1)),
                        0.5 + rng.uniform(0, 1.0 / 32, (5000, 3)),
                        np.tile([0.2, 0.3, 0.7], (3000, 1)),
                        rng.uniform(0.1, 0.9, (500, 3))])
    m = rng.uniform(0.5, 1.5, p.shape[0]) / p.shape[0]
    return W.Workload("clustered", 16, grids, p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(),
                      m, [None] * 2, boundary=boundary)


def periodic_edge_workload(seed=78):
    """Periodic root 16^3 with one subgrid: particles within a cell of every face and
    corner (clouds and stencils that wrap), exactly at 0, just below 1, outside the
    box and NaN, plus a clump on the subgrid; gas on both grids."""
    grids = W.centred_nested_grids(16, 8, 1)
    rng = np.random.default_rng(seed)
    d = 1.0 / 16
    near = np.where(rng.uniform(0, 1, (600, 3)) < 0.5, rng.uniform(0, d, (600, 3)),
                    rng.uniform(1 - d, 1, (600, 3)))
    mix = rng.uniform(0, 1, (600, 3))
    pick = rng.uniform(0, 1, (600, 3)) < 0.6
    p = np.concatenate([np.where(pick, near, mix), rng.uniform(0.45, 0.55, (300, 3)),
                        np.array([[0.0, 0.0, 0.0], [np.nextafter(1.0, 0.0), 0.5, 0.0],
                                  [0.0, np.nextafter(np.float32(1.0), np.float32(0.0)), 0.5],
                                  [-0.01, 0.5, 0.5], [np.nan, 0.5, 0.5], [1.0, 0.2, 0.2]])])
    m = rng.uniform(0.5, 1.5, p.shape[0]) / p.shape[0]
    gas = [W.root_uniform_gas(16, lambda x, y, z: 1.0 + 0.5 * np.sin(2 * np.pi * (x + 2 * y))),
           None]
    gas[1] = W.inject_gas(gas[0], grids[0], grids[1]) * 1.1
    return W.Workload("periodic_edges", 16, grids, p[:, 0].copy(), p[:, 1].copy(),
                      p[:, 2].copy(), m, gas, boundary="periodic")


def periodic_sine_particles():
    """The sine wave geometry on a 32^3 periodic root (P = 0.2) with 3000 massive
    particles uniform in the box besides the gas."""
    w = W.workload_sine_wave(period=0.2, root_n=32, ntracer=3000)
    rng = np.random.default_rng(79)
    w.m = rng.lognormal(0.0, 1.0, w.npart) * 1e-4
    return w


CASES = {
    "periodic_edges16": periodic_edge_workload,
    "periodic_sine32_P0.2": periodic_sine_particles,
    "periodic_sine64_tracers": lambda: W.workload_sine_wave(period=1.0, ntracer=2000),
    "periodic_plummer32": lambda: W.workload_plummer_periodic(root_n=32, sub_n=16, nlevels=2,
                                                              npart=20000),
    "root32_gas_4096": W.workload_root32_uniform_gas,
    "nested32_2x16_plummer": lambda: W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=2,
                                                                npart=20000),
    "clumps32_24grids": lambda: W.workload_clumps(root_n=32, ngrids=24, per_clump=400,
                                                   side_lo=4, side_hi=20),
    "gas_nested32": lambda: W.workload_plummer_gas(root_n=32, sub_n=16, nlevels=2, npart=5000),
    "slab_chain_L1024": slab_workload,
    "slab_chain_L1024_y": lambda: slab_workload(axis=1),
    "slab_chain_L1024_z": lambda: slab_workload(axis=2),
    "tiny_grids_L16": tiny_grid_workload,
    "edge_particles": edge_workload,
    "clustered_one_cell": clustered_workload,
    "clustered_one_cell_periodic": lambda: clustered_workload(boundary="periodic"),
    "uniform_sphere_gas_only": W.workload_uniform_sphere,
}


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_parity_small(case, dtype):
    w = CASES[case]()
    say(f"[parity] case={case} dtype={dtype.__name__} npart={w.npart} grids={len(w.grids)}")
    ref = run_oracle(w, dtype)
    got = run_staged(w, dtype)
    compare(case, w, dtype, got, ref)


# The compensated FP32 deposit (FP32 weights and (sum, error) pairs in registers, LDS
# and the key-box grid) meets the same FP32 bar as the FP64-accumulated one.
COMP_CASES = ("nested32_2x16_plummer", "gas_nested32", "periodic_edges16", "edge_particles",
              "clumps32_24grids", "slab_chain_L1024_z", "tiny_grids_L16", "clustered_one_cell")


@pytest.mark.parametrize("case", COMP_CASES)
def test_parity_compensated_fp32_deposit(case):
    w = CASES[case]()
    say(f"[parity] compensated FP32 deposit case={case} npart={w.npart}")
    ref = run_oracle(w, np.float32)
    got = run_staged(w, np.float32, accum="f32_comp")
    compare(case + "_comp", w, np.float32, got, ref)
    ctx = got["ctx"]
    x, y, z, m, gas = got["tensors"]
    ax, ay, az, pot = ctx.solve(x, y, z, m, gas)
    torch.cuda.synchronize()
    acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], 1)
    if w.npart:
        own = ref["owner"] >= 0
        assert rel(acc[own], ref["acc"][own]) <= TOL[np.float32]["acc"]
        assert rel(pot.cpu().numpy()[own], ref["pot"][own]) <= TOL[np.float32]["pot"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_fd2_gradient(dtype):
    w = W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=2, npart=8000)
    say(f"[parity] two-point gradient dtype={dtype.__name__}")
    compare("fd2", w, dtype, run_staged(w, dtype, "fd2"), run_oracle(w, dtype, "fd2"))


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("boundary", ["isolated", "periodic"])
def test_one_call_solve_matches_staged(dtype, boundary):
    if boundary == "isolated":
        w = W.workload_plummer_gas(root_n=32, sub_n=16, nlevels=2, npart=5000)
    else:
        w = periodic_sine_particles()
    say(f"[parity] apm_solve vs staged boundary={boundary} dtype={dtype.__name__}")
    got = run_staged(w, dtype)
    ctx = got["ctx"]
    x, y, z, m, gas = got["tensors"]
    ax, ay, az, pot = ctx.solve(x, y, z, m, gas)
    torch.cuda.synchronize()
    acc = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()], 1)
    tol = 1e-13 if dtype == np.float64 else 1e-6
    assert rel(acc, got["acc"]) <= tol and rel(pot.cpu().numpy(), got["pot"]) <= tol
    for l in range(got["plan"].nlevels):
        f = ctx.solved_field(l, x.dtype).cpu().numpy()
        ref = np.concatenate([got["field"][g["index"]].reshape(-1, 4)
                              for g in got["plan"].level_grids(l)])
        assert rel(f, ref) <= tol


# ---- the benchmarked workload at full size: root 128^3 + 2 x 64^3, 2^20 Plummer -------

@pytest.fixture(scope="module")
def bench_oracle():
    w = W.workload_plummer_nested()
    say("[parity] building oracle for the full bench workload (about a minute)")
    plan = O.OraclePlan(w.root_n, w.grids)
    cache = {g.index: O.greens(plan, g) for g in plan.grids}
    return w, cache


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype,accum", [(np.float64, "f64"), (np.float32, "f64"),
                                         (np.float32, "f32_comp")],
                         ids=["f64", "f32", "f32_comp"])
def test_parity_bench_workload_full_size(bench_oracle, dtype, accum):
    w, cache = bench_oracle
    say(f"[parity] full bench workload dtype={dtype.__name__} accum={accum} npart={w.npart}")
    ref = run_oracle(w, dtype, cache=cache)
    got = run_staged(w, dtype, accum=accum)
    compare("bench_full", w, dtype, got, ref)


# ---- batched level at full size: root 64^3 + 256 uneven level-1 grids, 2^21 particles --
# The oracle deposits every particle once per grid, so it is run on the root and on a
# sample of the 256 grids (each sampled grid in full: GMF, own and composed field, and
# every particle it owns); the owner grid of every particle is compared exactly.

CLUMP_SAMPLE = (0, 1, 37, 101, 128, 200, 254, 255)


@pytest.fixture(scope="module")
def clumps_oracle():
    w = W.workload_clumps()
    return w, O.OraclePlan(w.root_n, w.grids)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_clumps_workload_full_size(clumps_oracle, dtype):
    w, oplan = clumps_oracle
    say(f"[parity] full clumps workload dtype={dtype.__name__} npart={w.npart} "
        f"grids={len(w.grids)}")
    got = run_staged(w, dtype)
    t = TOL[dtype]
    cast = lambda a: np.asarray(a, dtype).astype(np.float64)
    x, y, z, m = (cast(a) for a in (w.x, w.y, w.z, w.m))
    say("[parity] oracle: owners of the rounded positions, root and sampled grids")
    own_ref = O.owner_of(oplan, x, y, z)
    assert np.array_equal(got["owner"], own_ref), "owner grids differ"
    gas = [None] * len(w.grids)
    root = oplan.grids[0]
    rho0 = O.deposit_grid(oplan, root, x, y, z, m, gas)
    f0 = O.compose(oplan, root, O.convolve(oplan, root, rho0), None)
    sample = [1 + (i % (len(w.grids) - 1)) for i in CLUMP_SAMPLE]
    fields = {0: f0}
    for gi in sample:
        g = oplan.grids[gi]
        rho = O.deposit_grid(oplan, g, x, y, z, m, gas)
        short = O.convolve(oplan, g, rho)
        fields[gi] = O.compose(oplan, g, short, f0)
        for key, ref in (("gmf", rho), ("own", short), ("field", fields[gi])):
            e = rel(got[key][gi], ref)
            assert e <= (t["gmf"] if key == "gmf" else t["field"]), \
                f"grid {gi} {key} rel L2 {e:.3e}"
    assert rel(got["gmf"][0], rho0) <= t["gmf"] and rel(got["field"][0], f0) <= t["field"]
    sel = np.nonzero(np.isin(own_ref, list(fields)))[0]
    flist = [fields.get(i, np.zeros((1, 1, 1, 4))) for i in range(len(w.grids))]
    pa = O.interp(oplan, flist, own_ref[sel], x[sel], y[sel], z[sel])
    say(f"[parity] clumps: {sel.size} particles on the root and the sampled grids")
    assert rel(got["acc"][sel], pa[:, :3]) <= t["acc"]
    assert rel(got["pot"][sel], pa[:, 3]) <= t["pot"]


# ---- periodic root at full size: 128^3 periodic + 2 x 64^3, 2^20 Plummer -------------

@pytest.fixture(scope="module")
def periodic_oracle():
    w = W.workload_plummer_periodic()
    say("[parity] building oracle kernels for the full periodic workload")
    plan = O.OraclePlan(w.root_n, w.grids, boundary="periodic")
    cache = {g.index: O.greens(plan, g) for g in plan.grids}
    return w, cache


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_parity_periodic_workload_full_size(periodic_oracle, dtype):
    w, cache = periodic_oracle
    say(f"[parity] full periodic workload dtype={dtype.__name__} npart={w.npart}")
    ref = run_oracle(w, dtype, cache=cache)
    got = run_staged(w, dtype)
    compare("periodic_full", w, dtype, got, ref)


def test_periodic_subgrid_solve_needs_the_average_density():
    """A periodic subgrid level cannot be solved before a level-0 deposit (or a solve)
    has recorded the average density."""
    import ctypes
    from paper_1410_0010_amd import _apm
    w = W.workload_sine_wave(period=1.0, root_n=32, ntracer=100)
    plan = P.Plan(w.root_n, w.grids, boundary="periodic")
    ctx = P.Context(plan, 0)
    lib = P.lib()
    gmf = ctx.empty_gmf(1, torch.float32)
    fld = ctx.empty_field(1, torch.float32)
    st = lib.apm_solve_level(ctx.handle, _apm.APM_F32, 1, ctypes.c_void_p(gmf.data_ptr()),
                             ctypes.c_void_p(fld.data_ptr()))
    assert st == _apm.APM_ERR_STATE
    x, y, z, m = (dev(a, np.float32) for a in (w.x, w.y, w.z, w.m))
    gas = [ctx.pack_gas(l, w.gas, torch.float32) for l in range(plan.nlevels)]
    ctx.solve(x, y, z, m, gas)
    torch.cuda.synchronize()
    st = lib.apm_solve_level(ctx.handle, _apm.APM_F32, 1, ctypes.c_void_p(gmf.data_ptr()),
                             ctypes.c_void_p(fld.data_ptr()))
    assert st == _apm.APM_OK
    torch.cuda.synchronize()


# ---- error paths through the device entry points ------------------------------------

def test_device_error_paths():
    import ctypes
    from paper_1410_0010_amd import _apm
    w = W.workload_plummer_nested(root_n=16, sub_n=8, nlevels=1, npart=100)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    lib = P.lib()
    x = dev(w.x, np.float64)
    assert lib.apm_deposit(ctx.handle, _apm.APM_F64, 5, None, None, None, None, 0, None, None,
                           None) == _apm.APM_ERR_INVALID
    f = ctx.empty_field(1, torch.float64)
    assert lib.apm_accel(ctx.handle, _apm.APM_F64, 1, ctypes.c_void_p(f.data_ptr()), None,
                         ctypes.c_void_p(f.data_ptr())) == _apm.APM_ERR_STATE
    assert lib.apm_deposit(ctx.handle, 7, 0, None, None, None, None, 0, None, None,
                           None) == _apm.APM_ERR_INVALID
    small = P.Plan(w.root_n, w.grids, workspace_limit=1024)
    c2 = P.Context(small, 0)
    with pytest.raises(P.APMError) as e:
        c2.deposit(0, x, x, x, x)
    assert e.value.status == _apm.APM_ERR_OOM


# ---- batched launches, graph replay and autotuning ------------------------------------

def _solve_np(ctx, t, gas=None):
    ax, ay, az, pot = ctx.solve(*t, gas)
    torch.cuda.synchronize()
    return np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy(),
                     pot.cpu().numpy()], 1).astype(np.float64)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_graph_replays_match_eager(dtype):
    """apm_solve is captured on its second identical call and replayed after; every
    replay, with eager torch work and synchronisations in between, matches the
    eager result and the oracle."""
    w = W.workload_clumps(root_n=32, ngrids=12, per_clump=600, side_lo=6, side_hi=18)
    say(f"[graph] clumps32 dtype={dtype.__name__}")
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    t = [dev(a, dtype) for a in (w.x, w.y, w.z, w.m)]
    ctx.set_graph(False)
    ref = _solve_np(ctx, t)
    ctx.set_graph(True)
    tol = 1e-12 if dtype == np.float64 else 2e-6
    scratch = torch.zeros(1 << 20, device=DEV)
    outs = [torch.empty(w.npart, dtype=t[0].dtype, device=DEV) for _ in range(4)]
    for rep in range(5):
        ctx.solve(*t, None, *outs)
        scratch.add_(1.0)                       # eager work on the same stream
        torch.cuda.synchronize()
        got = np.stack([o.cpu().numpy() for o in outs], 1).astype(np.float64)
        e = rel(got, ref)
        assert e <= tol, f"replay {rep}: rel {e:.3e}"
        outs[0].fill_(np.nan)                   # a replay must rewrite its outputs
    oref = run_oracle(w, dtype)
    own = oref["owner"] >= 0
    assert rel(got[own, :3], oref["acc"][own]) <= TOL[dtype]["acc"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_graph_replays_periodic_recompute_the_mean(dtype):
    """A periodic solve with root and subgrid gas under graph replay: the average
    density is taken inside the graph, so rewriting the masses in place between
    replays changes the result exactly as an eager solve on the new masses does."""
    w = periodic_sine_particles()
    say(f"[graph] periodic sine32 dtype={dtype.__name__}")
    plan = P.Plan(w.root_n, w.grids, boundary="periodic")
    ctx = P.Context(plan, 0)
    t = [dev(a, dtype) for a in (w.x, w.y, w.z, w.m)]
    gas = [ctx.pack_gas(l, w.gas, t[0].dtype) for l in range(plan.nlevels)]
    ctx.set_graph(False)
    ref1 = _solve_np(ctx, t, gas)
    m2 = np.asarray(w.m) * 3.0 + 1e-4
    eager2 = P.Context(plan, 0)
    eager2.set_graph(False)
    ref2 = _solve_np(eager2, t[:3] + [dev(m2, dtype)], gas)
    ctx.set_graph(True)
    tol = 1e-12 if dtype == np.float64 else 2e-6
    outs = [torch.empty(w.npart, dtype=t[0].dtype, device=DEV) for _ in range(4)]
    m1 = t[3].clone()
    for rep in range(6):
        ref = ref1 if rep % 2 == 0 else ref2
        t[3].copy_(m1 if rep % 2 == 0 else dev(m2, dtype))
        ctx.solve(*t, gas, *outs)
        torch.cuda.synchronize()
        got = np.stack([o.cpu().numpy() for o in outs], 1).astype(np.float64)
        e = rel(got, ref)
        assert e <= tol, f"replay {rep}: rel {e:.3e}"
        for o in outs:
            o.fill_(np.nan)
    assert rel(ref1, ref2) > 0.1                 # the two mass sets differ in the result
    w2 = periodic_sine_particles()
    w2.m = m2
    oref = run_oracle(w2, dtype)
    own = oref["owner"] >= 0
    assert rel(ref2[own, :3], oref["acc"][own]) <= TOL[dtype]["acc"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_autotune_keeps_parity(dtype):
    w = W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=2, npart=20000)
    say(f"[autotune] nested32 dtype={dtype.__name__}")
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    t = [dev(a, dtype) for a in (w.x, w.y, w.z, w.m)]
    _solve_np(ctx, t)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    report = ctx.autotune(tdt, reps=3)
    assert len(report) >= 5 and all("lines" in v for v in report.values())
    got = _solve_np(ctx, t)
    ref = run_oracle(w, dtype)
    own = ref["owner"] >= 0
    assert rel(got[own, :3], ref["acc"][own]) <= TOL[dtype]["acc"]
    assert rel(got[own, 3], ref["pot"][own]) <= TOL[dtype]["pot"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_dropped_particles_and_strict_mode(dtype):
    """apm_dropped counts the particles a deposit leaves out (outside [0, 1)^3 or NaN)
    and their mass; in strict mode apm_solve and apm_deposit report them as
    APM_ERR_RANGE, and accept the same hierarchy with those particles removed."""
    w = edge_workload()
    say(f"[dropped] edge particles dtype={dtype.__name__}")
    cast = lambda a: np.asarray(a, dtype).astype(np.float64)
    bad = ~O.valid_particles(cast(w.x), cast(w.y), cast(w.z))
    assert bad.sum() == 3
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, dtype) for a in (w.x, w.y, w.z, w.m))
    cnt, mass = ctx.dropped(x, y, z, m)
    assert cnt == 3 and abs(mass - cast(w.m)[bad].sum()) <= 1e-12
    assert ctx.dropped(x[:2], y[:2], z[:2], m[:2]) == (0, 0.0)
    strict = P.Context(P.Plan(w.root_n, w.grids, strict=True), 0)
    from paper_1410_0010_amd import _apm
    for call in (lambda: strict.solve(x, y, z, m), lambda: strict.deposit(0, x, y, z, m)):
        with pytest.raises(P.APMError) as e:
            call()
        assert e.value.status == _apm.APM_ERR_RANGE
    ok = torch.from_numpy(np.nonzero(~bad)[0]).to(DEV)
    sx, sy, sz, sm = (t[ok].contiguous() for t in (x, y, z, m))
    got = strict.solve(sx, sy, sz, sm)
    ref = ctx.solve(sx, sy, sz, sm)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_repeat_runs_agree_within_rounding(dtype):
    """The deposit sums with atomics in an order that varies between runs, so repeated
    solves of the same input need not be bit-identical; they agree to the rounding of
    the working precision (bound: 1e-6 relative L2 in FP32, 1e-14 in FP64, far inside
    the parity tolerances)."""
    w = W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=2, npart=50000)
    say(f"[repeat] nested32 npart={w.npart} dtype={dtype.__name__}")
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    ctx.set_graph(False)
    t = [dev(a, dtype) for a in (w.x, w.y, w.z, w.m)]
    runs = [_solve_np(ctx, t) for _ in range(4)]
    bound = 1e-6 if dtype == np.float32 else 1e-14
    worst = max(rel(r, runs[0]) for r in runs[1:])
    say(f"[repeat] largest relative L2 difference between runs: {worst:.3e}")
    assert worst <= bound
