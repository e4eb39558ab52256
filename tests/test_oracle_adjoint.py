"""Pins of the oracle's adjoint sweep (oracle/apm_adjoint.py), each against
something other than the adjoint itself:

* transpose identities <A u, v> = <u, A^T v> of every linear stage (deposit of
  masses and gas, per-grid convolution, level composition, interpolation), with
  the forward maps of oracle/apm_oracle.py on random inputs;
* position derivatives of the deposit and interpolation against central finite
  differences of the forward maps;
* the whole gradient of the potential energy W and of a general loss on
  accelerations and potentials against central finite differences of the forward
  solve (W is quadratic in masses and gas, so those differences are exact up to
  rounding);
* the symmetry closed form dW/dm_p = Phi_p on a single root grid (the potential
  operator, interpolation after deposition with the same weights and an even
  kernel, is symmetric for particles whose clouds lie inside the grid).

The transposes and gradients are checked on the isolated and on the periodic root
(particles over the whole box, clouds across its edges, the average density
subtracted from every GMF)."""

import numpy as np
import pytest

import apm_workloads as W
from apm_workloads import GridSpec
from oracle import apm_oracle as O
from oracle import apm_adjoint as A


def nested_case(npart=300, seed=5, gas=True, boundary="isolated"):
    """Root 16^3 + one centred 8^3 level (+ gas on both); particles in the centre, or,
    on a periodic root, a third of them within a cell of the box faces and the rest
    anywhere."""
    rng = np.random.default_rng(seed)
    grids = [GridSpec(0, -1, (0, 0, 0), (16,) * 3), GridSpec(1, 0, (12, 12, 12), (8,) * 3)]
    if boundary == "periodic":
        p = rng.uniform(0.0, 1.0, (npart, 3))
        k = npart // 3
        p[:k] = np.where(rng.uniform(0, 1, (k, 3)) < 0.5, rng.uniform(0, 1 / 16, (k, 3)),
                         rng.uniform(1 - 1 / 16, 1, (k, 3)))
    else:
        p = rng.uniform(0.3, 0.7, (npart, 3))
    m = rng.uniform(0.5, 1.5, npart) / npart
    g = None
    if gas:
        g0 = 0.3 + rng.uniform(0.0, 1.0, (16, 16, 16))
        g = [g0, W.inject_gas(g0, grids[0], grids[1])]
    return (O.OraclePlan(16, grids, boundary=boundary), p[:, 0].copy(), p[:, 1].copy(),
            p[:, 2].copy(), m, g)


BCS = ["isolated", "periodic"]


def dot(a, b):
    return float(sum(np.sum(u * v) for u, v in zip(a, b) if u is not None))


@pytest.mark.parametrize("bc", BCS)
def test_convolution_transpose(bc):
    plan, *_ = nested_case(boundary=bc)
    rng = np.random.default_rng(1)
    for g in plan.grids:
        k = O.greens(plan, g)
        rho = rng.standard_normal(tuple(int(v) for v in g.gmf_n[::-1]))
        sb = rng.standard_normal(tuple(int(v) for v in g.fld_n[::-1]) + (4,))
        lhs = np.sum(O.convolve(plan, g, rho, k) * sb)
        rhs = np.sum(rho * A.convolve_adjoint(plan, g, sb, k))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-300), (lhs, rhs)


def test_composition_transpose():
    plan, *_ = nested_case()
    rng = np.random.default_rng(2)
    s = [rng.standard_normal(tuple(int(v) for v in g.fld_n[::-1]) + (4,)) for g in plan.grids]
    fb = [rng.standard_normal(x.shape) for x in s]
    f = [None] * len(s)
    for lev in range(plan.nlevels):
        for g in plan.level_grids(lev):
            f[g.index] = O.compose(plan, g, s[g.index], f[g.parent] if g.parent >= 0 else None)
    lhs = dot(f, fb)
    rhs = dot(s, A.compose_adjoint(plan, fb))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("bc", BCS)
def test_interpolation_transpose_and_position_derivative(bc):
    plan, x, y, z, m, _ = nested_case(boundary=bc)
    rng = np.random.default_rng(3)
    F = [rng.standard_normal(tuple(int(v) for v in g.fld_n[::-1]) + (4,)) for g in plan.grids]
    own = O.owner_of(plan, x, y, z)
    cot = rng.standard_normal((x.size, 4))
    fbar, xbar = A.interp_adjoint(plan, F, own, x, y, z, cot)
    lhs = np.sum(O.interp(plan, F, own, x, y, z) * cot)
    assert abs(lhs - dot(F, fbar)) <= 1e-12 * abs(lhs)
    eps = 1e-7
    for axis in range(3):
        for i in range(0, x.size, 37):
            pp = [x.copy(), y.copy(), z.copy()]
            pm = [x.copy(), y.copy(), z.copy()]
            pp[axis][i] += eps
            pm[axis][i] -= eps
            lp = np.sum(O.interp(plan, F, own, *pp)[i] * cot[i])
            lm = np.sum(O.interp(plan, F, own, *pm)[i] * cot[i])
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - xbar[i, axis]) <= 1e-5 * (abs(xbar[i, axis]) + 1.0), (axis, i)


@pytest.mark.parametrize("bc", BCS)
def test_deposit_transpose_and_position_derivative(bc):
    plan, x, y, z, m, gas = nested_case(boundary=bc)
    rng = np.random.default_rng(4)
    gb = [rng.standard_normal(tuple(int(v) for v in g.gmf_n[::-1])) for g in plan.grids]
    mbar, xbar, gas_bar = A.deposit_adjoint(plan, x, y, z, m, gb, gas)
    # masses and gas enter the GMF linearly
    rho_p = [O.deposit_particles(plan, g, x, y, z, m) for g in plan.grids]
    assert abs(dot(rho_p, gb) - np.sum(m * mbar)) <= 1e-12 * abs(dot(rho_p, gb))
    zero = [np.zeros_like(r) for r in rho_p]
    rho_g = [O.add_gas(plan, g, zero[g.index], gas) for g in plan.grids]
    assert abs(dot(rho_g, gb) - dot(gas, gas_bar)) <= 1e-12 * abs(dot(rho_g, gb))
    eps = 1e-7
    for axis in range(3):
        for i in range(0, x.size, 41):
            pp = [x.copy(), y.copy(), z.copy()]
            pm = [x.copy(), y.copy(), z.copy()]
            pp[axis][i] += eps
            pm[axis][i] -= eps
            lp = dot([O.deposit_particles(plan, g, *pp, m) for g in plan.grids], gb)
            lm = dot([O.deposit_particles(plan, g, *pm, m) for g in plan.grids], gb)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - xbar[i, axis]) <= 1e-5 * (abs(xbar[i, axis]) + 1.0), (axis, i)


def test_energy_mass_gradient_is_potential_on_single_grid():
    rng = np.random.default_rng(6)
    n = 400
    p = rng.uniform(0.25, 0.75, (n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    plan = O.OraclePlan(16, [GridSpec(0, -1, (0, 0, 0), (16,) * 3)])
    gr = A.energy_gradient(plan, p[:, 0], p[:, 1], p[:, 2], m)
    phi = gr["fwd"]["pot"]
    assert np.max(np.abs(gr["m"] - phi)) <= 1e-12 * np.max(np.abs(phi))


@pytest.fixture(scope="module", params=BCS)
def energy_case(request):
    plan, x, y, z, m, gas = nested_case(npart=200, seed=9, boundary=request.param)
    cache = {}
    gr = A.energy_gradient(plan, x, y, z, m, gas, cache=cache)
    return plan, x, y, z, m, gas, cache, gr


def _energy(plan, x, y, z, m, gas, cache):
    return O.solve(plan, x, y, z, m, gas, cache)["energy"]


def test_energy_gradient_masses_and_gas_fd(energy_case):
    plan, x, y, z, m, gas, cache, gr = energy_case
    rng = np.random.default_rng(10)
    dm = rng.standard_normal(m.size) * m
    e = 1e-3
    fd = (_energy(plan, x, y, z, m + e * dm, gas, cache)
          - _energy(plan, x, y, z, m - e * dm, gas, cache)) / (2 * e)
    assert abs(fd - np.sum(gr["m"] * dm)) <= 1e-9 * abs(fd)
    dg = [rng.standard_normal(a.shape) * a for a in gas]
    gp = [a + e * d for a, d in zip(gas, dg)]
    gm = [a - e * d for a, d in zip(gas, dg)]
    fd = (_energy(plan, x, y, z, m, gp, cache) - _energy(plan, x, y, z, m, gm, cache)) / (2 * e)
    assert abs(fd - dot(gr["gas"], dg)) <= 1e-9 * abs(fd)


def test_energy_gradient_positions_fd(energy_case):
    plan, x, y, z, m, gas, cache, gr = energy_case
    rng = np.random.default_rng(11)
    v = rng.standard_normal((x.size, 3))
    e = 1e-7
    wp = _energy(plan, x + e * v[:, 0], y + e * v[:, 1], z + e * v[:, 2], m, gas, cache)
    wm = _energy(plan, x - e * v[:, 0], y - e * v[:, 1], z - e * v[:, 2], m, gas, cache)
    fd = (wp - wm) / (2 * e)
    an = np.sum(gr["x"] * v)
    assert abs(fd - an) <= 1e-6 * np.sum(np.abs(gr["x"] * v)), (fd, an)


@pytest.mark.parametrize("bc", BCS)
def test_general_loss_gradient_fd(bc):
    plan, x, y, z, m, gas = nested_case(npart=150, seed=12, boundary=bc)
    rng = np.random.default_rng(13)
    ab = rng.standard_normal((x.size, 3))
    pb = rng.standard_normal(x.size)
    cache = {}

    def loss(px, py, pz, mm, gg):
        r = O.solve(plan, px, py, pz, mm, gg, cache)
        return np.sum(r["acc"] * ab) + np.sum(r["pot"] * pb)

    gr = A.adjoint(plan, x, y, z, m, gas, abar=ab, phibar=pb, cache=cache)
    v = rng.standard_normal((x.size, 3))
    e = 1e-7
    fd = (loss(x + e * v[:, 0], y + e * v[:, 1], z + e * v[:, 2], m, gas)
          - loss(x - e * v[:, 0], y - e * v[:, 1], z - e * v[:, 2], m, gas)) / (2 * e)
    assert abs(fd - np.sum(gr["x"] * v)) <= 1e-6 * np.sum(np.abs(gr["x"] * v))
    dm = rng.standard_normal(m.size) * m
    e = 1e-3
    fd = (loss(x, y, z, m + e * dm, gas) - loss(x, y, z, m - e * dm, gas)) / (2 * e)
    assert abs(fd - np.sum(gr["m"] * dm)) <= 1e-9 * abs(fd)
    dg = [rng.standard_normal(a.shape) for a in gas]
    fd = (loss(x, y, z, m, [a + e * d for a, d in zip(gas, dg)])
          - loss(x, y, z, m, [a - e * d for a, d in zip(gas, dg)])) / (2 * e)
    assert abs(fd - dot(gr["gas"], dg)) <= 1e-9 * abs(fd)
