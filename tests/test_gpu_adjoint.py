"""GPU parity of the reverse sweep (apm_solve_adjoint through the C ABI) against the
FP64 oracle adjoint (oracle/apm_adjoint.py, itself pinned by finite differences and
transpose identities), and a finite-difference check of the autograd wrappers on
the GPU.  Tolerances: relative L2 1e-11 in FP64 and 1e-5 in FP32 (FP32-rounded
inputs on both sides)."""

import dataclasses
import sys

import numpy as np
import pytest

import apm_workloads as W
from oracle import apm_adjoint as A
from oracle import apm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_1410_0010_amd")
from paper_1410_0010_amd import autograd as AG  # noqa: E402

DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype))).to(DEV)


def rounded(w, dtype):
    f = lambda a: None if a is None else np.asarray(a, dtype).astype(np.float64)
    return f(w.x), f(w.y), f(w.z), f(w.m), [f(g) for g in w.gas]


def gas_clumps():
    """24 overlapping level-1 grids (several grids per tile, restriction from many
    children) with gas on the root injected into every grid."""
    w = W.workload_clumps(root_n=32, ngrids=24, per_clump=300, side_lo=4, side_hi=20)
    rng = np.random.default_rng(77)
    gas = [0.5 * W.gaussian_random_field_gas(rng, 32)]
    for g in w.grids[1:]:
        gas.append(W.inject_gas(gas[g.parent], w.grids[g.parent], g))
    return dataclasses.replace(w, gas=gas)


def periodic_edges():
    """Periodic root 16^3 + a centred 8^3 level with gas on both; particles within a
    cell of the box faces (clouds and stencils across the edges), anywhere in the box,
    on the subgrid, and a few outside the box."""
    grids = W.centred_nested_grids(16, 8, 1)
    rng = np.random.default_rng(81)
    d = 1.0 / 16
    near = np.where(rng.uniform(0, 1, (800, 3)) < 0.5, rng.uniform(0, d, (800, 3)),
                    rng.uniform(1 - d, 1, (800, 3)))
    p = np.concatenate([near, rng.uniform(0, 1, (800, 3)), rng.uniform(0.45, 0.55, (400, 3)),
                        np.array([[-0.01, 0.5, 0.5], [0.5, 1.0, 0.5]])])
    m = rng.uniform(0.5, 1.5, p.shape[0]) / p.shape[0]
    g0 = 0.3 + rng.uniform(0.0, 1.0, (16, 16, 16))
    gas = [g0, W.inject_gas(g0, grids[0], grids[1])]
    return W.Workload("periodic_edges", 16, grids, p[:, 0].copy(), p[:, 1].copy(),
                      p[:, 2].copy(), m, gas, boundary="periodic")


def periodic_sine():
    w = W.workload_sine_wave(period=0.2, root_n=32, ntracer=3000)
    w.m = np.random.default_rng(82).lognormal(0.0, 1.0, w.npart) * 1e-4
    return w


def slab_chain(axis):
    """Root 64^3 and a chain of thin slab grids reaching level 4, FFT lengths 256, 512
    and 1024 along `axis` (the transposed row passes for axis 0, the y column passes
    for 1, the z pass for 2), 32 across."""
    grids = [W.GridSpec(0, -1, (0, 0, 0), (64,) * 3)]
    for lev, (lo, n) in enumerate([(4, 120), (12, 232), (28, 456), (60, 904)], start=1):
        c = 32 * 2 ** lev
        los, ns = [c - 4] * 3, [8] * 3
        los[axis], ns[axis] = lo, n
        grids.append(W.GridSpec(lev, lev - 1, tuple(los), tuple(ns)))
    rng = np.random.default_rng(90 + axis)
    p = [0.5 + rng.normal(0, 0.002, 2500) for _ in range(3)]
    p[axis] = rng.uniform(0.08, 0.92, 2500)
    m = rng.uniform(0.5, 1.5, 2500) / 2500
    return W.Workload(f"slab_chain_axis{axis}", 64, grids, p[0], p[1], p[2], m,
                      [None] * len(grids))


def clustered():
    """5000 particles at one point and 5000 inside one cell of the subgrid, 3000 at
    one point of the root, 500 spread out: the transposed deposit and interpolation
    gather many equal cells into one chunk."""
    grids = W.centred_nested_grids(16, 8, 1)
    rng = np.random.default_rng(83)
    p = np.concatenate([np.tile([0.5 + 0.3 / 32, 0.5 - 0.1 / 32, 0.5 + 0.7 / 32], (5000, 1)),
                        0.5 + rng.uniform(0, 1.0 / 32, (5000, 3)),
                        np.tile([0.2, 0.3, 0.7], (3000, 1)),
                        rng.uniform(0.1, 0.9, (500, 3))])
    m = rng.uniform(0.5, 1.5, p.shape[0]) / p.shape[0]
    return W.Workload("clustered", 16, grids, p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(),
                      m, [None] * 2)


CASES = {
    "clustered_one_cell": clustered,
    "slab_chain_L1024_x": lambda: slab_chain(0),
    "slab_chain_L1024_y": lambda: slab_chain(1),
    "slab_chain_L1024_z": lambda: slab_chain(2),
    "periodic_edges16_gas": periodic_edges,
    "periodic_sine32": periodic_sine,
    "periodic_plummer32": lambda: W.workload_plummer_periodic(root_n=32, sub_n=16, nlevels=2,
                                                              npart=8000),
    "gas_nested32": lambda: W.workload_plummer_gas(root_n=32, sub_n=16, nlevels=2, npart=6000),
    "plummer_nested32_3lev": lambda: W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=3,
                                                                npart=8000),
    "root32_gas_4096": W.workload_root32_uniform_gas,
    "clumps32_24grids_gas": gas_clumps,
}


def gpu_adjoint(w, dtype, abar=None, phibar=None, wbar=0.0, autotune=False):
    plan = P.Plan(w.root_n, w.grids, boundary=w.boundary)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, dtype) for a in (w.x, w.y, w.z, w.m))
    gas = [ctx.pack_gas(l, w.gas, x.dtype) for l in range(plan.nlevels)]
    has_gas = any(g is not None for g in gas)
    if autotune:                       # the transposes then take the tuned launch shapes
        ctx.solve(x, y, z, m, gas if has_gas else None)
        ctx.autotune(x.dtype, reps=2)
    ax, ay, az, pot = ctx.solve(x, y, z, m, gas if has_gas else None)
    ab = None if abar is None else tuple(dev(abar[:, k], dtype) for k in range(3))
    pb = None if phibar is None else dev(phibar, dtype)
    xb, yb, zb, mb, gb = ctx.solve_adjoint(x, y, z, m, gas if has_gas else None, pot, ab, pb, wbar)
    torch.cuda.synchronize()
    got = lambda t: t.cpu().numpy().astype(np.float64)
    gas_out = None
    if gb is not None:
        gas_out = {}
        for l in range(plan.nlevels):
            if gb[l] is None:
                continue
            flat = got(gb[l])
            for g in plan.level_grids(l):
                n = int(np.prod(g["n"]))
                gas_out[g["index"]] = flat[g["gas_offset"]:g["gas_offset"] + n].reshape(
                    g["n"][2], g["n"][1], g["n"][0])
    return dict(x=np.stack([got(xb), got(yb), got(zb)], 1), m=got(mb), gas=gas_out)


def check(name, dtype, got, ref, w):
    tol = 1e-11 if dtype == np.float64 else 1e-5
    ex = rel(got["x"], ref["x"])
    em = rel(got["m"], ref["m"])
    say(f"[adjoint] {name} {dtype.__name__}: x {ex:.2e} m {em:.2e}")
    assert ex <= tol, f"{name}: position gradient rel L2 {ex:.3e}"
    assert em <= tol, f"{name}: mass gradient rel L2 {em:.3e}"
    if got["gas"] is not None:
        for gi, arr in got["gas"].items():
            r = ref["gas"][gi]
            eg = rel(arr, r)
            assert eg <= tol, f"{name}: gas gradient of grid {gi} rel L2 {eg:.3e}"


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_energy_gradient_matches_oracle(case, dtype):
    w = CASES[case]()
    say(f"[adjoint] energy gradient case={case} dtype={dtype.__name__} npart={w.npart}")
    x, y, z, m, gas = rounded(w, dtype)
    ref = A.energy_gradient(O.OraclePlan(w.root_n, w.grids, boundary=w.boundary), x, y, z, m,
                            gas)
    check(case, dtype, gpu_adjoint(w, dtype, wbar=1.0), ref, w)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_general_loss_after_autotune(dtype):
    """The four-component transposes after the autotuner has tuned the forward passes
    (lengths 256 to 1024 along y): each transpose takes a forward pass's tuned launch
    shape only where its own block holds it."""
    w = CASES["slab_chain_L1024_y"]()
    rng = np.random.default_rng(5)
    ab = np.asarray(rng.standard_normal((w.npart, 3)), dtype).astype(np.float64)
    pb = np.asarray(rng.standard_normal(w.npart), dtype).astype(np.float64)
    say(f"[adjoint] general loss after autotune dtype={dtype.__name__}")
    x, y, z, m, gas = rounded(w, dtype)
    ref = A.adjoint(O.OraclePlan(w.root_n, w.grids, boundary=w.boundary), x, y, z, m, gas,
                    abar=ab, phibar=pb, wbar=0.5)
    check("slab_chain_L1024_y tuned", dtype, gpu_adjoint(w, dtype, ab, pb, 0.5, autotune=True),
          ref, w)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", ["gas_nested32", "clumps32_24grids_gas", "periodic_edges16_gas",
                                  "periodic_sine32", "slab_chain_L1024_y", "slab_chain_L1024_z",
                                  "clustered_one_cell"])
def test_general_loss_gradient_matches_oracle(case, dtype):
    w = CASES[case]()
    rng = np.random.default_rng(3)
    ab = np.asarray(rng.standard_normal((w.npart, 3)), dtype).astype(np.float64)
    pb = np.asarray(rng.standard_normal(w.npart), dtype).astype(np.float64)
    say(f"[adjoint] general loss case={case} dtype={dtype.__name__}")
    x, y, z, m, gas = rounded(w, dtype)
    ref = A.adjoint(O.OraclePlan(w.root_n, w.grids, boundary=w.boundary), x, y, z, m, gas,
                    abar=ab, phibar=pb, wbar=0.5)
    check(case, dtype, gpu_adjoint(w, dtype, ab, pb, 0.5), ref, w)


def test_adjoint_needs_matching_solve():
    w = W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=1, npart=1000)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, np.float64) for a in (w.x, w.y, w.z, w.m))
    with pytest.raises(P.APMError):
        ctx.solve_adjoint(x, y, z, m, wbar=1.0, pot=torch.zeros_like(x))
    ax, ay, az, pot = ctx.solve(x, y, z, m)
    x2 = x.clone()
    with pytest.raises(P.APMError):
        ctx.solve_adjoint(x2, y, z, m, wbar=1.0, pot=pot)
    # the autotuner's trial launches overwrite the level fields; a deposit rebinds a
    # level: either leaves no state for the reverse sweep until the next solve
    ctx.autotune(torch.float64, reps=1)
    with pytest.raises(P.APMError):
        ctx.solve_adjoint(x, y, z, m, wbar=1.0, pot=pot)
    ax, ay, az, pot = ctx.solve(x, y, z, m)
    ctx.solve_adjoint(x, y, z, m, wbar=1.0, pot=pot)
    ctx.deposit(0, x, y, z, m)
    with pytest.raises(P.APMError):
        ctx.solve_adjoint(x, y, z, m, wbar=1.0, pot=pot)


def test_adjoint_needs_the_gas_of_the_last_solve():
    """The composed fields the reverse sweep reads depend on the gas: after a second
    solve with other gas, the reverse sweep of the first (its gas pointers) is refused,
    by the library and, through autograd, by the context's solve count."""
    w = W.workload_plummer_gas(root_n=32, sub_n=16, nlevels=1, npart=2000)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, np.float64) for a in (w.x, w.y, w.z, w.m))
    gas_a = [ctx.pack_gas(l, w.gas, x.dtype) for l in range(plan.nlevels)]
    gas_b = [None if g is None else 2.0 * g for g in gas_a]
    _, _, _, pot_a = ctx.solve(x, y, z, m, gas_a)
    ctx.solve(x, y, z, m, gas_b)
    with pytest.raises(P.APMError) as e:
        ctx.solve_adjoint(x, y, z, m, gas_a, pot_a, wbar=1.0)
    assert e.value.status == P._apm.APM_ERR_STATE
    xr, yr, zr, mr = (t.clone().requires_grad_() for t in (x, y, z, m))
    ga = [None if g is None else g.clone().requires_grad_() for g in gas_a]
    gb = [None if g is None else g.clone().requires_grad_() for g in gas_b]
    e1 = AG.potential_energy(ctx, xr, yr, zr, mr, ga)
    e2 = AG.potential_energy(ctx, xr, yr, zr, mr, gb)
    with pytest.raises(RuntimeError):
        torch.autograd.grad(e1, [xr])
    g2 = torch.autograd.grad(e2, [xr])[0]             # the most recent one still works
    assert torch.isfinite(g2).all()


def test_gas_totals_need_a_current_solve():
    w = W.workload_plummer_gas(root_n=32, sub_n=16, nlevels=1, npart=2000)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, np.float64) for a in (w.x, w.y, w.z, w.m))
    gas = [ctx.pack_gas(l, w.gas, x.dtype) for l in range(plan.nlevels)]
    ax, ay, az, pot = ctx.solve(x, y, z, m, gas)
    before = ctx.solve_totals(m, ax, ay, az, pot, gas=gas)
    ctx.autotune(torch.float64, reps=1)
    with pytest.raises(P.APMError):
        ctx.solve_totals(m, ax, ay, az, pot, gas=gas)
    ctx.solve_totals(m, ax, ay, az, pot)             # no gas term: GMF and particles only
    ax, ay, az, pot = ctx.solve(x, y, z, m, gas)
    after = ctx.solve_totals(m, ax, ay, az, pot, gas=gas)
    assert np.allclose(before, after, rtol=1e-12, atol=0)


def test_autograd_energy_finite_difference_fp64():
    """d W / d(x, m, gas) from torch.autograd (the reverse sweep) against central
    differences of the GPU forward energy along random directions (FP64)."""
    w = W.workload_plummer_gas(root_n=32, sub_n=16, nlevels=2, npart=3000)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, np.float64).requires_grad_() for a in (w.x, w.y, w.z, w.m))
    gas = [ctx.pack_gas(l, w.gas, torch.float64) for l in range(plan.nlevels)]
    for g in gas:
        g.requires_grad_()
    e = AG.potential_energy(ctx, x, y, z, m, gas)
    grads = torch.autograd.grad(e, [x, y, z, m] + gas)
    rng = np.random.default_rng(5)
    dirs = [dev(rng.standard_normal(t.shape[0]), np.float64) for t in [x, y, z, m] + gas]

    def energy_at(s, which):
        with torch.no_grad():
            vals = [t.detach().clone() for t in [x, y, z, m] + gas]
            for k in which:
                vals[k] = vals[k] + s * dirs[k] * (vals[k] if k >= 3 else 1.0)
            ax, ay, az, pot = ctx.solve(*vals[:4], vals[4:])
            return ctx.solve_totals(vals[3], ax, ay, az, pot, gas=vals[4:])[plan.nlevels]

    # positions: W is C1 in x (quadratic TSC pieces); masses and gas: W is quadratic
    for which, eps, tol in (([0, 1, 2], 1e-7, 1e-6), ([3], 1e-3, 1e-9), ([4, 5, 6], 1e-3, 1e-9)):
        fd = (energy_at(eps, which) - energy_at(-eps, which)) / (2 * eps)
        an = sum(float(torch.sum(grads[k] * dirs[k] * ((x, y, z, m, *gas)[k].detach()
                                                      if k >= 3 else 1.0))) for k in which)
        scale = sum(float(torch.sum(torch.abs(grads[k] * dirs[k] * ((x, y, z, m, *gas)[k].detach()
                                                                   if k >= 3 else 1.0))))
                    for k in which)
        say(f"[adjoint] autograd FD {which}: fd {fd:.10e} adjoint {an:.10e}")
        assert abs(fd - an) <= tol * scale


def test_autograd_solve_backward_matches_adjoint_fp32():
    w = W.workload_plummer_nested(root_n=32, sub_n=16, nlevels=2, npart=4000)
    plan = P.Plan(w.root_n, w.grids)
    ctx = P.Context(plan, 0)
    x, y, z, m = (dev(a, np.float32).requires_grad_() for a in (w.x, w.y, w.z, w.m))
    ax, ay, az, pot = AG.solve(ctx, x, y, z, m)
    rng = np.random.default_rng(8)
    c = [dev(rng.standard_normal(w.npart), np.float32) for _ in range(4)]
    loss = (ax * c[0]).sum() + (ay * c[1]).sum() + (az * c[2]).sum() + (pot * c[3]).sum()
    g = torch.autograd.grad(loss, [x, y, z, m])
    xr, yr, zr, mr, _ = rounded(w, np.float32)
    ref = A.adjoint(O.OraclePlan(w.root_n, w.grids), xr, yr, zr, mr,
                    abar=np.stack([t.cpu().numpy() for t in c[:3]], 1).astype(np.float64),
                    phibar=c[3].cpu().numpy().astype(np.float64))
    got = np.stack([t.cpu().numpy() for t in g[:3]], 1)
    assert rel(got, ref["x"]) <= 1e-5 and rel(g[3].cpu().numpy(), ref["m"]) <= 1e-5
