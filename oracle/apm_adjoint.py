"""Plain FP64 CPU reference of the reverse (adjoint) sweep of the APM solve.

TEST INFRASTRUCTURE ONLY, like apm_oracle (whose forward pieces it reuses): the
product path never imports it, and it shares nothing with the HIP code.

The forward solve (Sec. 2 and 2.2) is a chain of linear maps in the masses and gas
(deposit, per-grid convolution with Fourier-space differencing, level composition,
TSC interpolation), with the particle positions entering the deposit and the
interpolation weights.  For a loss

    L = wbar * W + sum_p abar_p . a_p + sum_p phibar_p Phi_p,

W the potential energy of the solve (1/2 sum_p m_p Phi_p plus the owned-gas term),
the gradient with respect to positions, masses and gas is obtained by running each
step's transpose in reverse order:

  interpolation^T   scatter of the cotangents (abar, phibar) with the TSC weights onto
                    the owner grid's field box; the position gradient from the
                    derivative of the weights against the forward field;
  composition^T     the transpose of the trilinear prolongation (a restriction with
                    weights 3/4, 1/4 per axis), applied from the finest level down;
  convolution^T     cyclic convolution with the flipped kernels: Fourier multipliers
                    conj(-i d_i Gf) = +i d_i Gf for the force and Gp for the potential,
                    the four field-box inputs summed into one GMF-box output;
  deposit^T         TSC gather of the GMF cotangent (over 1/dx^3) at the particles for
                    the mass gradient, its weight derivative (times m) for the
                    positions; own gas takes the active cells, the parent's gas the
                    ghost cells it was copied to.

Owner grids are piecewise constant in the positions and are held fixed (the loss
is not differentiable where a particle crosses an ownership boundary).

Periodic plans: the root's transposes wrap like its forward stencils, and the
subtraction of the average density rho_bar from every GMF (apm_oracle R24) adds
rho_bar's cotangent, minus the sum of every GMF cotangent, to the mass of every
in-domain particle and (times dx_0^3) to every root gas cell.
"""

from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import apm_oracle as O


def tsc_weight_derivs(t: np.ndarray):
    """d/dt of the TSC weights on cells i0-1, i0, i0+1 (offset t, as tsc_weights)."""
    return (-(0.5 - t), -2.0 * t, 0.5 + t)


def _stencil(g, x, y, z):
    ix, tx = O.cell_coords(x, g.dx)
    iy, ty = O.cell_coords(y, g.dx)
    iz, tz = O.cell_coords(z, g.dx)
    return ((ix, iy, iz), (O.tsc_weights(tx), O.tsc_weights(ty), O.tsc_weights(tz)),
            (tsc_weight_derivs(tx), tsc_weight_derivs(ty), tsc_weight_derivs(tz)))


def interp_adjoint(plan, fields: List[np.ndarray], own: np.ndarray, x, y, z, cot: np.ndarray):
    """Transpose of interp for cotangents cot (N, 4) = (abar, phibar): returns the field
    cotangents per grid (shape of fields) and the position gradient (N, 3)."""
    fbar = [np.zeros_like(f) for f in fields]
    xbar = np.zeros((x.shape[0], 3))
    for g in plan.grids:
        sel = np.nonzero(own == g.index)[0]
        if sel.size == 0:
            continue
        F = fields[g.index]
        wrap = plan.periodic and g.level == 0
        (ix, iy, iz), (wx, wy, wz), (dwx, dwy, dwz) = _stencil(g, x[sel], y[sel], z[sel])
        c = cot[sel]
        for dz in (-1, 0, 1):
            cz = iz + dz - g.fld_lo[2]
            if wrap:
                cz = cz % g.fld_n[2]
            for dy in (-1, 0, 1):
                cy = iy + dy - g.fld_lo[1]
                if wrap:
                    cy = cy % g.fld_n[1]
                for dxo in (-1, 0, 1):
                    cx = ix + dxo - g.fld_lo[0]
                    if wrap:
                        cx = cx % g.fld_n[0]
                    ins = ((cx >= 0) & (cx < g.fld_n[0]) & (cy >= 0) & (cy < g.fld_n[1])
                           & (cz >= 0) & (cz < g.fld_n[2]))
                    a, b, e = wx[dxo + 1], wy[dy + 1], wz[dz + 1]
                    w = a * b * e
                    np.add.at(fbar[g.index], (cz[ins], cy[ins], cx[ins]), w[ins, None] * c[ins])
                    v = np.zeros((sel.size, 4))
                    v[ins] = F[cz[ins], cy[ins], cx[ins]]
                    s = np.sum(v * c, axis=1)
                    xbar[sel, 0] += dwx[dxo + 1] * b * e * s / g.dx
                    xbar[sel, 1] += a * dwy[dy + 1] * e * s / g.dx
                    xbar[sel, 2] += a * b * dwz[dz + 1] * s / g.dx
    return fbar, xbar


def restrict(child_bar: np.ndarray, par, g) -> np.ndarray:
    """Transpose of O.prolong: the child field-box cotangent summed onto the parent's
    field box with the prolongation weights."""
    out = np.zeros((int(par.fld_n[2]), int(par.fld_n[1]), int(par.fld_n[0])) + child_bar.shape[3:])
    cs = [g.fld_lo[a] + np.arange(g.fld_n[a]) for a in range(3)]
    pq = [O._prolong_axis(c) for c in cs]
    for sz, wz in ((0, 0.75), (1, 0.25)):
        iz = pq[2][sz] - par.fld_lo[2]
        for sy, wy in ((0, 0.75), (1, 0.25)):
            iy = pq[1][sy] - par.fld_lo[1]
            for sx, wx in ((0, 0.75), (1, 0.25)):
                ix = pq[0][sx] - par.fld_lo[0]
                Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
                np.add.at(out, (Z, Y, X), wz * wy * wx * child_bar)
    return out


def compose_adjoint(plan, fbar: List[np.ndarray]) -> List[np.ndarray]:
    """Transpose of the composition: returns the own (short-range) field cotangents.
    The finest levels go first; each grid passes its cotangent to its parent."""
    sbar = [f.copy() for f in fbar]
    for lev in reversed(range(1, plan.nlevels)):
        for g in plan.level_grids(lev):
            sbar[g.parent] += restrict(sbar[g.index], plan.grids[g.parent], g)
    return sbar


def convolve_adjoint(plan, g, sbar: np.ndarray, kernels=None) -> np.ndarray:
    """Transpose of O.convolve: from (fz, fy, fx, 4) field-box cotangents to the GMF-box
    cotangent (gz, gy, gx)."""
    if kernels is None:
        kernels = O.greens(plan, g)
    gf, gp = kernels
    Mx, My, Mz = (int(v) for v in g.M)
    off = g.fld_lo - g.gmf_lo
    iz = (off[2] + np.arange(g.fld_n[2])) % Mz
    iy = (off[1] + np.arange(g.fld_n[1])) % My
    ix = (off[0] + np.arange(g.fld_n[0])) % Mx
    dsym = O._rfft_d(g.M, g.dx, plan.gradient)
    acc = None
    for c in range(4):
        pad = np.zeros((Mz, My, Mx))
        np.add.at(pad, np.ix_(iz, iy, ix), sbar[..., c])
        ck = np.fft.rfftn(pad)
        mult = np.conj(-1j * dsym[c] * gf) if c < 3 else gp
        acc = mult * ck if acc is None else acc + mult * ck
    full = np.fft.irfftn(acc, s=(Mz, My, Mx), axes=(0, 1, 2))
    gz, gy, gx = (int(v) for v in (g.gmf_n[2], g.gmf_n[1], g.gmf_n[0]))
    return full[:gz, :gy, :gx].copy()


def deposit_adjoint(plan, x, y, z, m, gmf_bar: List[np.ndarray], gas):
    """Transpose of the deposit (particles and gas): returns mbar (N,), xbar (N, 3) and
    the gas cotangent per grid (None where the grid has no gas)."""
    n = x.shape[0]
    mbar = np.zeros(n)
    xbar = np.zeros((n, 3))
    gas_bar = [None if a is None else np.zeros_like(a) for a in gas]
    ok = np.nonzero(O.valid_particles(x, y, z))[0]
    for g in plan.grids:
        gb = gmf_bar[g.index] / g.dx ** 3
        gx, gy, gz = (int(v) for v in g.gmf_n)
        wrap = plan.periodic and g.level == 0
        (ix, iy, iz), (wx, wy, wz), (dwx, dwy, dwz) = _stencil(g, x[ok], y[ok], z[ok])
        for dz in (-1, 0, 1):
            cz = iz + dz - g.gmf_lo[2]
            if wrap:
                cz = cz % gz
            for dy in (-1, 0, 1):
                cy = iy + dy - g.gmf_lo[1]
                if wrap:
                    cy = cy % gy
                for dxo in (-1, 0, 1):
                    cx = ix + dxo - g.gmf_lo[0]
                    if wrap:
                        cx = cx % gx
                    ins = (cx >= 0) & (cx < gx) & (cy >= 0) & (cy < gy) & (cz >= 0) & (cz < gz)
                    v = np.zeros(ok.size)
                    v[ins] = gb[cz[ins], cy[ins], cx[ins]]
                    a, b, e = wx[dxo + 1], wy[dy + 1], wz[dz + 1]
                    mbar[ok] += a * b * e * v
                    xbar[ok, 0] += m[ok] * dwx[dxo + 1] * b * e * v / g.dx
                    xbar[ok, 1] += m[ok] * a * dwy[dy + 1] * e * v / g.dx
                    xbar[ok, 2] += m[ok] * a * b * dwz[dz + 1] * v / g.dx
        # gas: own gas on the active cells, the parent's on the ghost cells
        a0 = g.lo - g.gmf_lo
        if gas_bar[g.index] is not None:
            gas_bar[g.index] += gmf_bar[g.index][a0[2]:a0[2] + g.n[2], a0[1]:a0[1] + g.n[1],
                                                 a0[0]:a0[0] + g.n[0]]
        if g.parent >= 0 and gas_bar[g.parent] is not None:
            par = plan.grids[g.parent]
            cs = [g.gmf_lo[a] + np.arange(g.gmf_n[a]) for a in range(3)]
            Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
            active = ((X >= g.lo[0]) & (X < g.lo[0] + g.n[0]) & (Y >= g.lo[1])
                      & (Y < g.lo[1] + g.n[1]) & (Z >= g.lo[2]) & (Z < g.lo[2] + g.n[2]))
            gh = ~active
            np.add.at(gas_bar[g.parent],
                      (Z[gh] // 2 - par.lo[2], Y[gh] // 2 - par.lo[1], X[gh] // 2 - par.lo[0]),
                      gmf_bar[g.index][gh])
    return mbar, xbar, gas_bar


def owned_gas_mask(plan, g) -> np.ndarray:
    """Active cells of g whose centre g owns (the cells counted in the gas energy)."""
    cs = [(g.lo[a] + np.arange(g.n[a]) + 0.5) * g.dx for a in range(3)]
    zz, yy, xx = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
    return O.owner_of(plan, xx.ravel(), yy.ravel(), zz.ravel()).reshape(xx.shape) == g.index


def adjoint(plan, x, y, z, m, gas=None, abar=None, phibar=None, wbar: float = 0.0,
            cache: Optional[dict] = None, fwd: Optional[dict] = None) -> dict:
    """Gradient of L = wbar W + sum abar.a + sum phibar Phi with respect to x, y, z
    (as an (N, 3) array), m and the gas of every grid.  Also returns the
    intermediate cotangents: fbar (composed fields), sbar (own fields), gmf_bar."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64); m = np.asarray(m, np.float64)
    n = x.shape[0]
    if gas is None:
        gas = [None] * len(plan.grids)
    gas = [None if a is None else np.asarray(a, np.float64) for a in gas]
    if cache is None:
        cache = {}
    if fwd is None:
        fwd = O.solve(plan, x, y, z, m, gas, cache)
    own = fwd["owner"]
    owned = own >= 0
    cot = np.zeros((n, 4))
    if abar is not None:
        cot[:, :3] = np.asarray(abar, np.float64)
    if phibar is not None:
        cot[:, 3] = np.asarray(phibar, np.float64)
    cot[:, 3] += wbar * 0.5 * m * owned
    cot[~owned] = 0.0
    fbar, xbar = interp_adjoint(plan, fwd["field"], own, x, y, z, cot)
    gas_direct = [None if a is None else np.zeros_like(a) for a in gas]
    if wbar != 0.0:
        for g in plan.grids:
            if gas[g.index] is None:
                continue
            mask = owned_gas_mask(plan, g)
            a0 = g.lo - g.fld_lo
            sl = (slice(a0[2], a0[2] + g.n[2]), slice(a0[1], a0[1] + g.n[1]),
                  slice(a0[0], a0[0] + g.n[0]))
            fbar[g.index][sl + (3,)] += np.where(mask, wbar * 0.5 * gas[g.index] * g.dx ** 3, 0.0)
            gas_direct[g.index] += np.where(mask, wbar * 0.5 * fwd["field"][g.index][sl + (3,)]
                                            * g.dx ** 3, 0.0)
    sbar = compose_adjoint(plan, fbar)
    for g in plan.grids:
        if g.index not in cache:
            cache[g.index] = O.greens(plan, g)
    gmf_bar = [convolve_adjoint(plan, g, sbar[g.index], cache[g.index]) for g in plan.grids]
    mbar, xbar2, gas_bar = deposit_adjoint(plan, x, y, z, m, gmf_bar, gas)
    if plan.periodic:
        # every GMF was convolved minus rho_bar = sum of in-domain masses + root gas dx^3
        rho_bar_bar = -sum(float(np.sum(b)) for b in gmf_bar)
        mbar = mbar + rho_bar_bar * O.valid_particles(x, y, z)
        if gas_bar[0] is not None:
            gas_bar[0] = gas_bar[0] + rho_bar_bar * plan.grids[0].dx ** 3
    mbar = mbar + wbar * 0.5 * fwd["pot"] * owned
    gas_bar = [None if a is None else a + d for a, d in zip(gas_bar, gas_direct)]
    return dict(x=xbar + xbar2, m=mbar, gas=gas_bar, fbar=fbar, sbar=sbar, gmf_bar=gmf_bar,
                fwd=fwd)


def energy_gradient(plan, x, y, z, m, gas=None, cache=None, fwd=None) -> dict:
    """dW/d(x, m, gas): the adjoint with wbar = 1 and no other cotangents."""
    return adjoint(plan, x, y, z, m, gas, wbar=1.0, cache=cache, fwd=fwd)
