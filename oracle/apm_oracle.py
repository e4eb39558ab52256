"""Plain FP64 CPU oracle of the adaptive particle-mesh (APM) gravity solve on
static nested grids (Passy & Bryan, "An adaptive particle-mesh gravity solver for
ENZO", Sec. 2 and 2.2).

TEST INFRASTRUCTURE ONLY.  This module is imported by the tests, by the package's
smoke check and by the benchmark's CPU-baseline leg; the product path never calls
it.  It shares no code with the HIP path: every step below is written out here
from the paper, in numpy float64, with the library FFT (numpy.fft) as the only
borrowed primitive.  It is slow on purpose (whole-array numpy, no blocking or
fusion) so that each function can be read against the paper.

What it computes, per solve (the paper's order):
  1. TSC deposit of particles into each grid's GravitatingMassField (GMF), plus
     gas (own gas on active cells, the parent's gas copied onto the ghost zone)
     -- Sec. 2, mass assignment and the modified subgrid deposition.
  2. Per grid, the potential of its GMF by a zero-padded cyclic FFT convolution
     (Eq. 2), differenced in Fourier space into the three force components:
       * subgrids: the optimal influence function Eq. 5 with the TSC assignment
         Eq. 7-8, the short-range reference force Eq. 9 (S_l^2 - S_{l-1}^2),
         Brillouin zones n in [-1,1]^3 (Eq. 6), zero padding of 0.65 R a/dx cells
         (Sec. 2.2, last paragraph);
       * root (level 0, isolated boundary, Sec. 2.1): the level-0 optimal
         influence function (reference S_0^2, Eq. 9) made isolated on the
         doubled mesh (James 1977).
  3. The parent's acceleration (and potential) interpolated onto the grid and
     added to the grid's own short-range field (Sec. 2.2).
  4. TSC interpolation of the accelerations to the particles, on the finest grid
     holding each particle.
  5. FP64 totals: deposited mass, potential energy, net force.

Readings of the paper used here (each one also listed in the design notes):
  R1  Eq. 5 is in the repulsive unit-charge convention with no G; the gravity
      kernel is -4 pi G times it, G = 1.
  R2  Eq. 7 prints prod sinc^6 for U; that is U^2 for TSC (U = prod sinc^3).  The
      closed form Eq. 8 is the alias sum of sinc^6 (pinned in the tests).
  R3  The level-0 reference force uses S_0^2 (Eq. 9 with S_{-1} = 0).
  R4  sinc x = sin(x)/x.
  R5  Numerator of Eq. 5 over n in [-1,1]^3; denominator uses the exact sum Eq. 8.
  R6  Gradient: the direct Fourier-space operator D = -i k (Sec. 2.2 names it and
      the finite-difference one as the two choices); the two-point central
      difference D = -i sin(k dx)/dx is kept as an option.  The potential is
      differenced in Fourier space (Sec. 2.2), so both are exact multiplications;
      the derivative symbol is 0 at the Nyquist index.
  R7  Conjugate D* in Eq. 5; where |D|^2 = 0 the force kernel is 0 (the force
      multiplier D vanishes there too).
  R21 Potential: Sec. 2.2 takes the potential from Eq. 2 with Eq. 5's G, and the
      force from the potential differenced in Fourier space.  With the spectral
      gradient (the default) that is done literally: one kernel, Eq. 5's G, whose
      removable singularity at k = 0 is filled by its limit (only the n = 0 alias
      term survives there: -4 pi G (a_{l-1}^2 - a_l^2)/30 on a subgrid; on the
      isolated root the limit of the short-range difference, -pi G dx^2, is added
      to the James part).  With the two-point gradient Eq. 5's G grows without
      bound next to the Nyquist corners where |D| -> 0, so there the potential
      uses HE's potential-optimal influence function (Eq. 5 with D -> 1 and the
      reference potential) instead.
  R22 Root kernel: optimal influence function of level 0 made isolated as the
      James doubled-mesh reference potential plus the (short-ranged) difference
      optimal - reference on the doubled mesh.
  R8  Small-argument series for S(eta) and for (S_l^2 - S_{l-1}^2)/k^2.
  R9  Root Green's function: the S2-S2 reference potential at a_0 sampled on the
      (2N)^3 mirrored mesh and transformed (real, even).
  R10 Subgrid zero padding p = ceil(0.65 * R * 3.4) = 5 cells in total per axis;
      FFT length M = smallest supported length >= n + 2b + p.
  R11 GMF ghost width b = 3 on subgrids; the root GMF is its active box.
  R12 A subgrid GMF receives every particle whose TSC cloud overlaps it (clipped
      at its edge); the root clips clouds at the domain edge.
  R13 Parent gas is copied piecewise-constant onto the ghost cells.
  R14 Parent acceleration and potential are interpolated trilinearly between
      cell centres (weights 3/4, 1/4 per axis).
  R15 Particles take TSC-interpolated accelerations from their owner grid: the
      finest grid whose active box holds them, lowest index among equals.
  R16 Particles with a coordinate outside [0, 1) (or NaN) are not deposited and
      get zero acceleration.
  R18 The potential is composed like the acceleration: Phi = P(Phi_parent) + phi.
  R20 Energy W = 1/2 sum_p m_p Phi_p + 1/2 sum over owned gas cells rho Phi dx^3.

Periodic boundary (Sec. 2.1 for the periodic root Green's function, and the sine
wave test of Sec. 3): with boundary="periodic"
  R23 the root's kernels are the level-0 optimal influence functions of Eq. 5
      (reference S_0^2, R3) on the root's own N^3 mesh, no doubling, with the
      k = 0 value of both set to 0;
  R24 the average density of the system, rho_bar = (sum of the in-domain particle
      masses + root gas mass) / box volume, is subtracted from the GMF of every
      grid, on every GMF cell, before its convolution (the solve needs zero net
      mass); the GMF itself (and the deposited mass it reports) is the density;
  R25 the root's TSC clouds and interpolation stencils wrap around the box edges
      (cell indices modulo N); subgrids are unchanged (their GMF boxes lie inside
      the root's active box);
  R26 the leapfrog drift maps positions back into [0, 1).

Subcycling (Sec. 2: levels advance with their own steps, dt_{l+1} <= dt_l / 2,
Eq. 10; Sec. 3.1 and 3.5 evolve with dt_{l+1} = dt_l / 2):
  R27 the levels advance recursively (root step, then two steps of the next level,
      and so on): a step of size h on level l, starting at the level's clock t_l,
      (i) hands every particle of level l or finer to level max(l, level of its
      owner grid) (those particles all sit at time t_l), (ii) deposits every
      particle at its position predicted to the mid-step time t_l + h/2 from its
      own level's clock, x + v (t_l + h/2 - t_own) (the time-centred density of
      Sec. 2), solves the level's grids and adds the parent's latest composed
      field (Sec. 2.2), then (iii) moves the particles of level l only, about the
      predicted position: v += h a(x_mid), x = x_mid + v h/2, a interpolated from
      the finest grid of level <= l holding x_mid.  The parent field a level adds
      (Sec. 2.2) is the parent's composed field taken linearly in time through the
      parent's two latest solves (at their mid-step times) to the level's own
      mid-step time (the paper leaves the parent's time open; held fixed instead,
      the coarse part of a particle's own field, centred at another time, pulls
      it).  The different levels' contributions still come from different times,
      the time-integration error Sec. 3.1 and 3.5 attribute to subcycling; with
      one step size on every level each step reduces to a single consistent solve
      at the mid-step positions.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

# --------------------------------------------------------------------------
# numeric contract constants (Sec. 2.2: a = 3.4 dx_l, padding 0.65 R a/dx, R = 2)
# --------------------------------------------------------------------------
A_CELLS = 3.4
PAD_FACTOR = 0.65
REFINE = 2
GHOST = 3


def fft_length(n: int, policy: str = "pow2") -> int:
    """Smallest supported FFT length >= n (R10)."""
    if policy == "pow2":
        m = 1
        while m < n:
            m *= 2
        return m
    if policy == "smooth":          # 2^a 3^b 5^c with a >= 3
        m = n
        while True:
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1 and m % 8 == 0:
                return m
            m += 1
    raise ValueError(policy)


@dataclass
class OGrid:
    index: int
    level: int
    parent: int
    lo: np.ndarray          # (x, y, z) first active cell, level-l global index
    n: np.ndarray           # active cells per axis
    dx: float
    gmf_lo: np.ndarray
    gmf_n: np.ndarray
    fld_lo: np.ndarray
    fld_n: np.ndarray
    M: np.ndarray           # FFT length per axis (x, y, z)


class OraclePlan:
    """Derived geometry of a static hierarchy (the oracle's own rules)."""

    def __init__(self, root_n: int, grids: Sequence, G: float = 1.0,
                 a_cells: float = A_CELLS, pad_factor: float = PAD_FACTOR,
                 ghost: int = GHOST, fft_policy: str = "pow2", gradient: str = "spectral",
                 boundary: str = "isolated"):
        self.root_n = int(root_n)
        if boundary not in ("isolated", "periodic"):
            raise ValueError(boundary)
        self.boundary = boundary
        self.periodic = boundary == "periodic"
        self.G = float(G)
        self.a_cells = float(a_cells)
        self.ghost = int(ghost)
        self.pad = int(math.ceil(pad_factor * REFINE * a_cells - 1e-12))
        self.fft_policy = fft_policy
        if gradient not in ("spectral", "fd2"):
            raise ValueError(gradient)
        self.gradient = gradient
        self.grids: List[OGrid] = []
        for i, g in enumerate(grids):
            lo = np.array(g.lo, dtype=np.int64)
            n = np.array(g.n, dtype=np.int64)
            dx = 1.0 / (self.root_n * 2 ** g.level)
            if g.level == 0:
                gmf_lo, gmf_n = lo.copy(), n.copy()
                fld_lo, fld_n = lo.copy(), n.copy()
                M = np.array([self.root_n if self.periodic else 2 * self.root_n] * 3,
                             dtype=np.int64)
            else:
                b = self.ghost
                gmf_lo, gmf_n = lo - b, n + 2 * b
                fld_lo, fld_n = lo - 1, n + 2
                M = np.array([fft_length(int(gn) + self.pad, fft_policy) for gn in gmf_n],
                             dtype=np.int64)
            self.grids.append(OGrid(i, int(g.level), int(g.parent), lo, n, dx,
                                    gmf_lo, gmf_n, fld_lo, fld_n, M))
        self.nlevels = 1 + max(g.level for g in self.grids)

    def a_soft(self, level: int) -> float:
        return self.a_cells / (self.root_n * 2 ** level)

    def level_grids(self, level: int) -> List[OGrid]:
        return [g for g in self.grids if g.level == level]


# --------------------------------------------------------------------------
# 1. TSC assignment (Sec. 2: triangular-shaped cloud over 3^3 cells)
# --------------------------------------------------------------------------

def cell_coords(x: np.ndarray, dx: float):
    """Cell index i0 = floor(x/dx) and offset t = x/dx - i0 - 1/2 in [-1/2, 1/2)."""
    s = x / dx
    i0 = np.floor(s)
    return i0.astype(np.int64), s - i0 - 0.5


def tsc_weights(t: np.ndarray):
    """TSC weights on cells i0-1, i0, i0+1 for offset t from the centre of cell i0."""
    return (0.5 * (0.5 - t) ** 2, 0.75 - t * t, 0.5 * (0.5 + t) ** 2)


def valid_particles(x, y, z):
    """R16: in-domain, finite positions."""
    ok = np.ones(x.shape, dtype=bool)
    for c in (x, y, z):
        ok &= np.isfinite(c) & (c >= 0.0) & (c < 1.0)
    return ok


def deposit_particles(plan: OraclePlan, g: OGrid, x, y, z, m) -> np.ndarray:
    """TSC mass density of all in-domain particles on g's GMF box (R12).

    rho(c) = sum_p m_p W(c - x_p) / dx^3, clouds clipped at the GMF box; on a
    periodic root the clouds wrap around the box edges instead (R25)."""
    wrap = plan.periodic and g.level == 0
    ok = valid_particles(x, y, z)
    x, y, z, m = x[ok], y[ok], z[ok], m[ok]
    gx, gy, gz = (int(v) for v in g.gmf_n)
    out = np.zeros(gx * gy * gz)
    ix, tx = cell_coords(x, g.dx)
    iy, ty = cell_coords(y, g.dx)
    iz, tz = cell_coords(z, g.dx)
    wx, wy, wz = tsc_weights(tx), tsc_weights(ty), tsc_weights(tz)
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
                inside = (cx >= 0) & (cx < gx) & (cy >= 0) & (cy < gy) & (cz >= 0) & (cz < gz)
                w = m * wx[dxo + 1] * wy[dy + 1] * wz[dz + 1]
                flat = (cz * gy + cy) * gx + cx
                out += np.bincount(flat[inside], weights=w[inside], minlength=out.size)
    return out.reshape(gz, gy, gx) / g.dx ** 3


def add_gas(plan: OraclePlan, g: OGrid, rho: np.ndarray, gas: Sequence[Optional[np.ndarray]]):
    """Own gas on active cells; the parent's gas copied onto ghost cells (R13)."""
    rho = rho.copy()
    own = gas[g.index]
    a0 = g.lo - g.gmf_lo
    if own is not None:
        rho[a0[2]:a0[2] + g.n[2], a0[1]:a0[1] + g.n[1], a0[0]:a0[0] + g.n[0]] += own
    if g.parent >= 0 and gas[g.parent] is not None:
        par = plan.grids[g.parent]
        cs = [g.gmf_lo[a] + np.arange(g.gmf_n[a]) for a in range(3)]
        Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
        active = ((X >= g.lo[0]) & (X < g.lo[0] + g.n[0]) & (Y >= g.lo[1]) & (Y < g.lo[1] + g.n[1])
                  & (Z >= g.lo[2]) & (Z < g.lo[2] + g.n[2]))
        pv = gas[g.parent][Z // 2 - par.lo[2], Y // 2 - par.lo[1], X // 2 - par.lo[0]]
        rho += np.where(active, 0.0, pv)
    return rho


def deposit_grid(plan, g, x, y, z, m, gas):
    return add_gas(plan, g, deposit_particles(plan, g, x, y, z, m), gas)


# --------------------------------------------------------------------------
# 2a. S2 softening (Eq. 3, 4)
# --------------------------------------------------------------------------

_SERIES_TERMS = 14


def _s2_series_coeffs():
    # S(eta) = 12 * sum_{j>=0} (-1)^j (2j+2)/(2j+4)! eta^(2j)
    return [12.0 * (-1) ** j * (2 * j + 2) / math.factorial(2 * j + 4) for j in range(_SERIES_TERMS)]


_S2C = _s2_series_coeffs()


def s2_hat(eta: np.ndarray) -> np.ndarray:
    """Fourier transform of the S2 sphere (Eq. 4), eta = k a / 2; series for eta < 1 (R8)."""
    eta = np.asarray(eta, dtype=np.float64)
    out = np.empty_like(eta)
    small = eta < 1.0
    e = eta[~small]
    out[~small] = 12.0 / e ** 4 * (2.0 - 2.0 * np.cos(e) - e * np.sin(e))
    e2 = eta[small] ** 2
    acc = np.zeros_like(e2)
    for c in reversed(_S2C):
        acc = acc * e2 + c
    out[small] = acc
    return out


def s2_density(r: np.ndarray, a: float) -> np.ndarray:
    """Eq. 3: S(r) = 48/(pi a^4) (a/2 - r) for r <= a/2, else 0."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r <= a / 2, 48.0 / (math.pi * a ** 4) * (a / 2 - r), 0.0)


def ref_force_factor(k: np.ndarray, a_l: float, a_lm1: Optional[float]) -> np.ndarray:
    """f_l(k) = (S_l^2 - S_{l-1}^2)/k^2 (Eq. 9 without the -i k), S_{-1} = 0 at the root.

    Small-k path (R8): S(eta_l) - S(eta_{l-1}) as a series in k^2 with the constant
    term cancelled exactly, so no digits are lost; f(0) = (a_{l-1}^2 - a_l^2)/30."""
    k = np.asarray(k, dtype=np.float64)
    sl = s2_hat(k * a_l / 2)
    if a_lm1 is None:
        with np.errstate(divide="ignore", invalid="ignore"):
            return sl * sl / (k * k)
    sm = s2_hat(k * a_lm1 / 2)
    out = np.empty_like(k)
    small = (k * a_lm1 / 2) < 1.0
    with np.errstate(divide="ignore", invalid="ignore"):
        kb = k[~small]
        out[~small] = (sl[~small] - sm[~small]) * (sl[~small] + sm[~small]) / (kb * kb)
    k2 = k[small] ** 2
    # (S_l - S_{l-1})/k^2 = sum_{j>=1} c_j (a_l^(2j) - a_{l-1}^(2j)) / 4^j k^(2j-2)
    acc = np.zeros_like(k2)
    for j in reversed(range(1, _SERIES_TERMS)):
        cj = _S2C[j] * (a_l ** (2 * j) - a_lm1 ** (2 * j)) / 4.0 ** j
        acc = acc * k2 + cj
    out[small] = acc * (sl[small] + sm[small])
    return out


# --------------------------------------------------------------------------
# 2b. Root Green's function: S2-S2 reference potential, isolated (R9)
# --------------------------------------------------------------------------

def s2s2_potential_shape(u: np.ndarray) -> np.ndarray:
    """P(u), u = 2r/a: the potential of two unit S2 clouds at separation r is
    P(2r/a) * 2/a in units where a point pair gives 1/r.  Obtained by integrating
    the S2 self-convolution against 1/r; P(u) = 1/u for u >= 2 (no overlap)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    a = u <= 1.0
    b = (u > 1.0) & (u < 2.0)
    c = u >= 2.0
    ua = u[a]
    out[a] = (52.0 / 35.0 - 4.0 * ua ** 2 / 5.0 + 2.0 * ua ** 4 / 5.0 - ua ** 5 / 10.0
              - 2.0 * ua ** 6 / 35.0 + 3.0 * ua ** 7 / 140.0)
    ub = u[b]
    out[b] = (32.0 / 35.0 + 3.0 / (35.0 * ub) + 8.0 * ub / 5.0 - 16.0 * ub ** 2 / 5.0
              + 2.0 * ub ** 3 - 2.0 * ub ** 4 / 5.0 - ub ** 5 / 10.0 + 2.0 * ub ** 6 / 35.0
              - ub ** 7 / 140.0)
    out[c] = 1.0 / u[c]
    return out


def s2s2_potential_shape_deriv(u: np.ndarray) -> np.ndarray:
    """dP/du (term by term from P above)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    a = u <= 1.0
    b = (u > 1.0) & (u < 2.0)
    c = u >= 2.0
    ua = u[a]
    out[a] = (-8.0 * ua / 5.0 + 8.0 * ua ** 3 / 5.0 - ua ** 4 / 2.0 - 12.0 * ua ** 5 / 35.0
              + 3.0 * ua ** 6 / 20.0)
    ub = u[b]
    out[b] = (-3.0 / (35.0 * ub ** 2) + 8.0 / 5.0 - 32.0 * ub / 5.0 + 6.0 * ub ** 2
              - 8.0 * ub ** 3 / 5.0 - ub ** 4 / 2.0 + 12.0 * ub ** 5 / 35.0 - 7.0 * ub ** 6 / 140.0)
    out[c] = -1.0 / u[c] ** 2
    return out


def root_kernel(r: np.ndarray, a0: float, G: float) -> np.ndarray:
    """g_0(r) = -G (2/a_0) P(2r/a_0): potential at r of a unit S2 cloud seen by an S2 cloud."""
    return -G * (2.0 / a0) * s2s2_potential_shape(2.0 * np.asarray(r) / a0)


def greens_root_james(plan: OraclePlan) -> np.ndarray:
    """DFT of the S2-S2 reference potential sampled on the (2N)^3 doubled mesh at
    mirrored separations r = dx sqrt(sum_i min(j_i, 2N-j_i)^2), times dx_0^3, on the
    rfft grid.  With this kernel the cyclic convolution on (2N)^3 equals the
    isolated direct sum over the root (James 1977, Sec. 2.1)."""
    N = plan.root_n
    M = 2 * N
    dx = 1.0 / N
    j = np.arange(M)
    jm = np.minimum(j, M - j).astype(np.float64)
    r = dx * np.sqrt(jm[:, None, None] ** 2 + jm[None, :, None] ** 2 + jm[None, None, :] ** 2)
    g = root_kernel(r, plan.a_soft(0), plan.G)
    return np.fft.rfftn(g).real * dx ** 3


# --------------------------------------------------------------------------
# 2c. Optimal influence functions (Eq. 5-9)
# --------------------------------------------------------------------------

def _k_axis(M: int, dx: float, half: bool) -> np.ndarray:
    """Wavenumbers 2 pi m / (M dx), m in (-M/2, M/2] (rfft half axis if ``half``)."""
    if half:
        m = np.arange(M // 2 + 1)
    else:
        m = np.arange(M)
        m = np.where(m > M // 2, m - M, m)
    return 2.0 * math.pi * m / (M * dx)


def grad_symbol(m: np.ndarray, M: int, dx: float, mode: str) -> np.ndarray:
    """d(k) for mesh index m (signed, k = 2 pi m/(M dx)); the gradient operator is
    D = -i d (the force is D applied to the potential).  "spectral": d = k (Sec. 2.2,
    the direct Fourier-space gradient); "fd2": d = sin(k dx)/dx, the two-point
    central difference (R6).  At the Nyquist index m = M/2 the sign of k is
    ambiguous and d is 0 (the two-point difference is 0 there too)."""
    m = np.asarray(m)
    k = 2.0 * math.pi * m / (M * dx)
    if mode == "fd2":
        d = np.sin(k * dx) / dx
    else:
        d = k.astype(np.float64)
    if M % 2 == 0:
        d = np.where(np.abs(m) * 2 == M, 0.0, d)
    return d


def _alias_factor(k: np.ndarray, dx: float) -> np.ndarray:
    """Eq. 8 per axis: sum over Brillouin zones of sinc^6 = 1 - sin^2 + 2/15 sin^4."""
    s = np.sin(k * dx / 2) ** 2
    return 1.0 - s + 2.0 / 15.0 * s * s


def _sinc6(k: np.ndarray, dx: float) -> np.ndarray:
    """TSC U^2 per axis (R2, R4): sinc^6(k dx / 2), sinc x = sin x / x."""
    h = k * dx / 2
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.where(h == 0.0, 1.0, np.sin(h) / np.where(h == 0.0, 1.0, h))
    return v ** 6


def influence(kx, ky, kz, dx: float, a_l: float, a_lm1: Optional[float], G: float,
              dsym, bz: int = 1, ref=None):
    """The two optimal influence functions at wavenumbers (kx, ky, kz) (broadcastable
    1-D axes), both times -4 pi G (R1):

    force:      Eq. 5, D*(k) . sum_n U^2(k_n) R(k_n) / (|D(k)|^2 [sum_n U^2(k_n)]^2)
                with the gradient D = -i d, d = dsym per axis (grad_symbol),
                reference force R(q) = -i q f_l(|q|) (Eq. 9), Brillouin zones
                n in [-bz, bz]^3 (Eq. 6), U^2 the TSC sinc^6 product (Eq. 7, R2) and
                the denominator sum in closed form (Eq. 8, R5).  Zero where
                |d|^2 = 0 (there the force multiplier -i d vanishes anyway, R7).
    potential:  the same construction with the gradient replaced by the identity and
                the reference force by the reference potential f_l, i.e.
                sum_n U^2(k_n) f_l(|k_n|) / [sum_n U^2(k_n)]^2.  (With the
                two-point gradient the force kernel grows without bound next to
                the Nyquist corners where |d| -> 0, so it cannot give the potential.)
    The mesh force is IDFT(-i d_i force rho_hat); which kernel gives the potential
    is decided by the caller (R21).  With a_lm1 None (the root, S_{-1} = 0) the
    k = 0 values are infinite and are replaced by the caller.  ``ref``, if given,
    replaces f_l(|q|) (a function of the alias wavenumber magnitude q alone)."""
    kx, ky, kz = (np.asarray(v, dtype=np.float64) for v in (kx, ky, kz))
    sx, sy, sz = (np.asarray(v, dtype=np.float64) for v in dsym)
    s2 = sx * sx + sy * sy + sz * sz
    c2 = (_alias_factor(kx, dx) * _alias_factor(ky, dx) * _alias_factor(kz, dx)) ** 2
    shape = np.broadcast_shapes(kx.shape, ky.shape, kz.shape)
    num_f = np.zeros(shape)
    num_p = np.zeros(shape)
    kg = 2.0 * math.pi / dx
    for nz in range(-bz, bz + 1):
        qz = kz + nz * kg
        uz = _sinc6(qz, dx)
        for ny in range(-bz, bz + 1):
            qy = ky + ny * kg
            uy = _sinc6(qy, dx)
            for nx in range(-bz, bz + 1):
                qx = kx + nx * kg
                ux = _sinc6(qx, dx)
                q = np.sqrt(qx * qx + qy * qy + qz * qz)
                with np.errstate(divide="ignore", invalid="ignore"):
                    if ref is not None:
                        f = ref(q)
                    else:
                        f = ref_force_factor(q, a_l, a_lm1)
                        if a_lm1 is not None:
                            f = np.where(q == 0.0, (a_lm1 ** 2 - a_l ** 2) / 30.0, f)
                u2f = ux * uy * uz * f
                num_p += u2f
                num_f += np.where(np.isfinite(u2f), u2f, 0.0) * (sx * qx + sy * qy + sz * qz)
    den_f = s2 * c2
    with np.errstate(invalid="ignore", divide="ignore"):
        force = np.where(den_f > 0.0, num_f / np.where(den_f > 0.0, den_f, 1.0), 0.0)
        pot = num_p / c2
    return -4.0 * math.pi * G * force, -4.0 * math.pi * G * pot


def _rfft_k(M, dx):
    Mx, My, Mz = (int(v) for v in M)
    return (_k_axis(Mx, dx, True)[None, None, :], _k_axis(My, dx, False)[None, :, None],
            _k_axis(Mz, dx, False)[:, None, None])


def _rfft_d(M, dx, mode):
    """Gradient symbols per axis on the rfft grid, broadcastable like _rfft_k."""
    Mx, My, Mz = (int(v) for v in M)
    mx = np.arange(Mx // 2 + 1)
    my = np.arange(My); my = np.where(my > My // 2, my - My, my)
    mz = np.arange(Mz); mz = np.where(mz > Mz // 2, mz - Mz, mz)
    return (grad_symbol(mx, Mx, dx, mode)[None, None, :],
            grad_symbol(my, My, dx, mode)[None, :, None],
            grad_symbol(mz, Mz, dx, mode)[:, None, None])


def _planes(k3, d3, planes):
    """The rfft-grid axes restricted to the kz planes [p0, p1) (all planes if None)."""
    if planes is None:
        return k3, d3
    p0, p1 = planes
    return (k3[0], k3[1], k3[2][p0:p1]), (d3[0], d3[1], d3[2][p0:p1])


def greens_sub(plan: OraclePlan, g: OGrid, planes=None):
    """(force kernel, potential kernel) of subgrid g on its padded rfft grid
    (Mz, My, Mx//2+1), or on its kz planes [p0, p1) only; short-range reference
    S_l^2 - S_{l-1}^2 (Eq. 9).

    Spectral gradient (R21): both are Eq. 5's G, with the value at k = 0 set to its
    limit -4 pi G (a_{l-1}^2 - a_l^2)/30 (the force multiplier -i d is 0 there, so
    the forces do not see it).  Two-point gradient: the potential-optimal kernel."""
    (kx, ky, kz), dsym = _planes(_rfft_k(g.M, g.dx), _rfft_d(g.M, g.dx, plan.gradient), planes)
    al, alm1 = plan.a_soft(g.level), plan.a_soft(g.level - 1)
    gf, gpo = influence(kx, ky, kz, g.dx, al, alm1, plan.G, dsym)
    if plan.gradient == "fd2":
        return gf, gpo
    gf = gf.copy()
    if planes is None or planes[0] == 0:
        gf[0, 0, 0] = -4.0 * math.pi * plan.G * (alm1 ** 2 - al ** 2) / 30.0
    return gf, gf


def greens_root(plan: OraclePlan, planes=None, james=None):
    """(force kernel, potential kernel) of the isolated root on the (2N)^3 rfft grid
    (or on its kz planes [p0, p1) only; ``james``, if given, is greens_root_james on
    those planes).

    The optimal influence functions of level 0 (reference S_0^2, R3) are periodic.
    They are made isolated by splitting them into the reference potential, whose
    isolated form comes from the doubled-mesh James construction, plus the
    difference optimal - reference, which only corrects the TSC smoothing and the
    finite difference at short range and is added on the doubled mesh as is.
    k = 0 of the short-range difference: its limit -pi G dx^2 (the n = 0 alias term
    gives f (U^2/C^2 - 1) -> dx^2/4 in unit-charge units; the other terms vanish like
    k^5).  The limit is the same for the force kernel with the spectral gradient
    (there d . k_0 / |d|^2 = 1), whose k = 0 value the forces never see (d = 0).
    Spectral gradient: the potential kernel is the force kernel (R21); two-point
    gradient: the potential-optimal kernel."""
    g = plan.grids[0]
    (kx, ky, kz), dsym = _planes(_rfft_k(g.M, g.dx), _rfft_d(g.M, g.dx, plan.gradient), planes)
    a0 = plan.a_soft(0)
    if james is not None:
        gj = james
    else:
        gj = greens_root_james(plan)
        if planes is not None:
            gj = gj[planes[0]:planes[1]]
    KX, KY, KZ = np.broadcast_arrays(kx, ky, kz)
    k = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    with np.errstate(divide="ignore", invalid="ignore"):
        gref = -4.0 * math.pi * plan.G * s2_hat(k * a0 / 2) ** 2 / (k * k)
        fo, po = influence(kx, ky, kz, g.dx, a0, None, plan.G, dsym)
        dF = fo - gref
        dP = po - gref
    if planes is None or planes[0] == 0:
        dF[0, 0, 0] = -math.pi * plan.G * g.dx ** 2 if plan.gradient == "spectral" else 0.0
        dP[0, 0, 0] = -math.pi * plan.G * g.dx ** 2
    gf = gj + dF
    return (gf, gf) if plan.gradient == "spectral" else (gf, gj + dP)


def greens_root_periodic(plan: OraclePlan):
    """(force kernel, potential kernel) of the periodic root on its N^3 rfft grid
    (R23): the level-0 optimal influence functions of Eq. 5 taken directly in
    Fourier space, zero at k = 0 (there the force multiplier vanishes and the
    mean density carries no potential).  Spectral gradient: the potential kernel
    is the force kernel (R21); two-point gradient: the potential-optimal one."""
    g = plan.grids[0]
    kx, ky, kz = _rfft_k(g.M, g.dx)
    with np.errstate(divide="ignore", invalid="ignore"):
        fo, po = influence(kx, ky, kz, g.dx, plan.a_soft(0), None, plan.G,
                           _rfft_d(g.M, g.dx, plan.gradient))
    fo[0, 0, 0] = 0.0
    po[0, 0, 0] = 0.0
    return (fo, fo) if plan.gradient == "spectral" else (fo, po)


def greens(plan: OraclePlan, g: OGrid, planes=None):
    """(force, potential) kernels of grid g on its rfft grid, or on its kz planes
    [p0, p1) only (the same values: each plane depends on its own wavenumbers)."""
    if g.level > 0:
        return greens_sub(plan, g, planes)
    if plan.periodic:
        fo, fp = greens_root_periodic(plan)
        return (fo, fp) if planes is None else (fo[planes[0]:planes[1]], fp[planes[0]:planes[1]])
    return greens_root(plan, planes)


# --------------------------------------------------------------------------
# 2d. Convolution (Eq. 2) and differencing in Fourier space
# --------------------------------------------------------------------------

def convolve(plan: OraclePlan, g: OGrid, rho: np.ndarray, kernels=None) -> np.ndarray:
    """Short-range field of g's GMF on its field box, shape (fz, fy, fx, 4):
    a_i = IDFT(-i d_i Gf rho_hat), phi = IDFT(Gp rho_hat), cyclic on the zero-padded
    mesh M (the potential is differenced in Fourier space, Sec. 2.2)."""
    if kernels is None:
        kernels = greens(plan, g)
    gf, gp = kernels
    Mx, My, Mz = (int(v) for v in g.M)
    pad = np.zeros((Mz, My, Mx))
    gz, gy, gx = rho.shape
    pad[:gz, :gy, :gx] = rho
    rk = np.fft.rfftn(pad)
    dsym = _rfft_d(g.M, g.dx, plan.gradient)
    off = g.fld_lo - g.gmf_lo
    iz = (off[2] + np.arange(g.fld_n[2])) % Mz
    iy = (off[1] + np.arange(g.fld_n[1])) % My
    ix = (off[0] + np.arange(g.fld_n[0])) % Mx
    out = np.empty((int(g.fld_n[2]), int(g.fld_n[1]), int(g.fld_n[0]), 4))
    for c, dc in enumerate(dsym):
        full = np.fft.irfftn(-1j * dc * gf * rk, s=(Mz, My, Mx), axes=(0, 1, 2))
        out[..., c] = full[np.ix_(iz, iy, ix)]
    full = np.fft.irfftn(gp * rk, s=(Mz, My, Mx), axes=(0, 1, 2))
    out[..., 3] = full[np.ix_(iz, iy, ix)]
    return out


def convolve_scalar(g: OGrid, rho: np.ndarray, ghat: np.ndarray) -> np.ndarray:
    """IDFT(ghat * DFT(zero-padded rho)) on g's field box (one scalar kernel)."""
    Mx, My, Mz = (int(v) for v in g.M)
    pad = np.zeros((Mz, My, Mx))
    gz, gy, gx = rho.shape
    pad[:gz, :gy, :gx] = rho
    full = np.fft.irfftn(np.fft.rfftn(pad) * ghat, s=(Mz, My, Mx), axes=(0, 1, 2))
    off = g.fld_lo - g.gmf_lo
    iz = (off[2] + np.arange(g.fld_n[2])) % Mz
    iy = (off[1] + np.arange(g.fld_n[1])) % My
    ix = (off[0] + np.arange(g.fld_n[0])) % Mx
    return full[np.ix_(iz, iy, ix)]


# --------------------------------------------------------------------------
# 3. Level composition (Sec. 2.2)
# --------------------------------------------------------------------------

def _prolong_axis(c: np.ndarray):
    """Parent cells and weights for child cells c (R14)."""
    p = c // 2
    q = np.where(c % 2 == 0, p - 1, p + 1)
    return p, q


def prolong(parent_field: np.ndarray, par: OGrid, g: OGrid) -> np.ndarray:
    """Trilinear interpolation of a parent field (on the parent's field box) to the
    centres of g's field-box cells."""
    cs = [g.fld_lo[a] + np.arange(g.fld_n[a]) for a in range(3)]
    pq = [_prolong_axis(c) for c in cs]
    out = np.zeros((int(g.fld_n[2]), int(g.fld_n[1]), int(g.fld_n[0])) + parent_field.shape[3:])
    for sz, wz in ((0, 0.75), (1, 0.25)):
        iz = pq[2][sz] - par.fld_lo[2]
        for sy, wy in ((0, 0.75), (1, 0.25)):
            iy = pq[1][sy] - par.fld_lo[1]
            for sx, wx in ((0, 0.75), (1, 0.25)):
                ix = pq[0][sx] - par.fld_lo[0]
                for idx, nmax in ((ix, par.fld_n[0]), (iy, par.fld_n[1]), (iz, par.fld_n[2])):
                    if idx.min() < 0 or idx.max() >= nmax:
                        raise ValueError("child field box not covered by the parent's field box")
                out += wz * wy * wx * parent_field[np.ix_(iz, iy, ix)]
    return out


def compose(plan: OraclePlan, g: OGrid, short: np.ndarray,
            parent_field: Optional[np.ndarray]) -> np.ndarray:
    """Total field of g: its short-range field plus the parent's field interpolated
    onto its cells (R14, R18); the root's field is its own."""
    if g.parent >= 0 and parent_field is not None:
        return short + prolong(parent_field, plan.grids[g.parent], g)
    return short.copy()


# --------------------------------------------------------------------------
# 4. Owner grid and TSC interpolation to particles
# --------------------------------------------------------------------------

def owner_of(plan: OraclePlan, x, y, z) -> np.ndarray:
    """Finest grid whose active box holds the point, lowest index among equals (R15)."""
    own = np.full(x.shape, -1, dtype=np.int64)
    ok = valid_particles(x, y, z)
    for lev in range(plan.nlevels):
        for g in reversed(plan.level_grids(lev)):
            inside = ok.copy()
            for a, c in enumerate((x, y, z)):
                i = np.floor(np.where(ok, c, 0.0) / g.dx)
                inside &= (i >= g.lo[a]) & (i < g.lo[a] + g.n[a])
            own[inside] = g.index
    return own


def interp(plan: OraclePlan, fields: List[np.ndarray], own: np.ndarray, x, y, z):
    """TSC interpolation of (ax, ay, az, Phi) from each particle's owner grid (R15);
    the stencil wraps around the box edges on a periodic root (R25)."""
    out = np.zeros((x.shape[0], 4))
    for g in plan.grids:
        sel = np.nonzero(own == g.index)[0]
        if sel.size == 0:
            continue
        wrap = plan.periodic and g.level == 0
        F = fields[g.index]
        ix, tx = cell_coords(x[sel], g.dx)
        iy, ty = cell_coords(y[sel], g.dx)
        iz, tz = cell_coords(z[sel], g.dx)
        wx, wy, wz = tsc_weights(tx), tsc_weights(ty), tsc_weights(tz)
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
                    inside = ((cx >= 0) & (cx < g.fld_n[0]) & (cy >= 0) & (cy < g.fld_n[1])
                              & (cz >= 0) & (cz < g.fld_n[2]))
                    w = wx[dxo + 1] * wy[dy + 1] * wz[dz + 1]
                    v = np.zeros((sel.size, 4))
                    v[inside] = F[cz[inside], cy[inside], cx[inside]]
                    out[sel] += w[:, None] * v
    return out


# --------------------------------------------------------------------------
# 5. Whole forward solve and FP64 totals
# --------------------------------------------------------------------------

def gas_energy(plan: OraclePlan, fields, gas) -> float:
    """1/2 sum over gas cells owned by their grid (not covered by a finer grid) of rho Phi dx^3."""
    tot = 0.0
    for g in plan.grids:
        if gas[g.index] is None:
            continue
        cs = [(g.lo[a] + np.arange(g.n[a]) + 0.5) * g.dx for a in range(3)]
        zz, yy, xx = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
        own = owner_of(plan, xx.ravel(), yy.ravel(), zz.ravel()).reshape(xx.shape)
        a0 = g.lo - g.fld_lo
        phi = fields[g.index][a0[2]:a0[2] + g.n[2], a0[1]:a0[1] + g.n[1], a0[0]:a0[0] + g.n[0], 3]
        tot += 0.5 * float(np.sum(np.where(own == g.index, gas[g.index] * phi, 0.0))) * g.dx ** 3
    return tot


def solve(plan: OraclePlan, x, y, z, m, gas=None, cache: Optional[dict] = None):
    """The full forward APM solve in the paper's order: deposit every grid, solve
    every grid, compose level by level from the root down, interpolate to the
    particles.  ``cache`` keeps Green's functions between calls (the paper caches
    frequently used Green's functions, Sec. 2.2).  Returns per-grid gmf, short
    (own short-range field), field (composed), per-particle acc (N,3), pot (N,),
    owner, and FP64 totals: mass per grid, energy, net force on particles.  With a
    periodic root the average density rho_bar (returned too) is subtracted from
    every GMF before its convolution (R24)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64); m = np.asarray(m, np.float64)
    if gas is None:
        gas = [None] * len(plan.grids)
    gas = [None if a is None else np.asarray(a, np.float64) for a in gas]
    if cache is None:
        cache = {}
    for g in plan.grids:
        if g.index not in cache:
            cache[g.index] = greens(plan, g)
    gmf = [deposit_grid(plan, g, x, y, z, m, gas) for g in plan.grids]
    rho_bar = mean_density(plan, x, y, z, m, gas) if plan.periodic else 0.0
    short = [convolve(plan, g, gmf[g.index] - rho_bar, cache[g.index]) for g in plan.grids]
    fld = [None] * len(plan.grids)
    for lev in range(plan.nlevels):
        for g in plan.level_grids(lev):
            fld[g.index] = compose(plan, g, short[g.index],
                                   fld[g.parent] if g.parent >= 0 else None)
    own = owner_of(plan, x, y, z)
    pa = interp(plan, fld, own, x, y, z)
    mass = [float(gmf[g.index].sum() * g.dx ** 3) for g in plan.grids]
    w = 0.5 * float(np.sum(m[own >= 0] * pa[own >= 0, 3])) + gas_energy(plan, fld, gas)
    fnet = (m[:, None] * pa[:, :3]).sum(axis=0)
    return dict(gmf=gmf, short=short, field=fld, owner=own, acc=pa[:, :3], pot=pa[:, 3],
                mass=mass, energy=w, net_force=fnet, rho_bar=rho_bar)


def mean_density(plan: OraclePlan, x, y, z, m, gas) -> float:
    """Average density of the system (R24): the in-domain particle mass plus the
    root's gas mass over the unit box."""
    ok = valid_particles(x, y, z)
    tot = float(np.sum(m[ok]))
    if gas[0] is not None:
        tot += float(np.sum(gas[0])) * plan.grids[0].dx ** 3
    return tot


# --------------------------------------------------------------------------
# Independent references used by the pins (not part of the solve)
# --------------------------------------------------------------------------

def direct_root_potential(plan: OraclePlan, rho: np.ndarray) -> np.ndarray:
    """Reference potential on the root's active cells by direct summation
    sum_j rho_j dx^3 g_0(|x_i - x_j|) (isolated, no mesh)."""
    g = plan.grids[0]
    N = plan.root_n
    dx = 1.0 / N
    a0 = plan.a_soft(0)
    src = np.argwhere(rho != 0.0)                 # (k, 3) as (z, y, x)
    w = rho[rho != 0.0] * dx ** 3
    out = np.zeros((int(g.n[2]), int(g.n[1]), int(g.n[0])))
    for kz in range(out.shape[0]):
        for ky in range(out.shape[1]):
            for kx in range(out.shape[2]):
                c = np.array([kz, ky, kx]) + g.lo[::-1]
                r = dx * np.sqrt(((src - c) ** 2).sum(axis=1))
                out[kz, ky, kx] = np.sum(w * root_kernel(r, a0, plan.G))
    return out


def pp_reference_accel(x, y, z, m, a: float, G: float = 1.0):
    """Direct particle-particle accelerations with the S2-S2 reference force at
    softening a (the force the mesh hierarchy approximates on the finest level)."""
    p = np.stack([x, y, z], axis=1)
    acc = np.zeros_like(p)
    for i in range(p.shape[0]):
        d = p - p[i]
        r = np.sqrt((d * d).sum(axis=1))
        nz = r > 0
        # potential of j at i: -G m_j (2/a) P(2r/a); accel = -grad_i = dPhi/dr * d/r
        dphi = -G * m[nz] * (2.0 / a) * s2s2_potential_shape_deriv(2.0 * r[nz] / a) * (2.0 / a)
        acc[i] = ((dphi / r[nz])[:, None] * d[nz]).sum(axis=0)
    return acc


def owner_up_to(plan: OraclePlan, x, y, z, lmax: int) -> np.ndarray:
    """owner_of restricted to the grids of levels 0..lmax (R15, R27)."""
    own = np.full(x.shape, -1, dtype=np.int64)
    ok = valid_particles(x, y, z)
    for lev in range(min(lmax, plan.nlevels - 1) + 1):
        for g in reversed(plan.level_grids(lev)):
            inside = ok.copy()
            for a, c in enumerate((x, y, z)):
                i = np.floor(np.where(ok, c, 0.0) / g.dx)
                inside &= (i >= g.lo[a]) & (i < g.lo[a] + g.n[a])
            own[inside] = g.index
    return own


def evolve_subcycled(plan: OraclePlan, x, y, z, vx, vy, vz, m, dt0: float, nroot: int,
                     gas=None, ratio: int = 2, energy: bool = False):
    """``nroot`` root steps of ``dt0`` with level l stepping dt0 / ratio^l (R27);
    ratio = 2 is Eq. 10 with equality, ratio = 1 steps every level together.
    Returns the final state and, per root step (and at the start), the positions,
    velocities and, with ``energy``, K + W from a solve at the synchronised
    positions."""
    if plan.periodic:
        raise ValueError("subcycling is read for the isolated root only")
    x, y, z = (np.array(c, np.float64) for c in (x, y, z))
    v = [np.array(c, np.float64) for c in (vx, vy, vz)]
    m = np.asarray(m, np.float64)
    if gas is None:
        gas = [None] * len(plan.grids)
    gas = [None if a is None else np.asarray(a, np.float64) for a in gas]
    nl = plan.nlevels
    cache = {g.index: greens(plan, g) for g in plan.grids}
    level_of = np.array([g.level for g in plan.grids])
    own0 = owner_of(plan, x, y, z)
    lev = np.where(own0 >= 0, level_of[np.maximum(own0, 0)], 0)
    clock = np.zeros(nl)
    fld = [None] * len(plan.grids)          # latest composed field of each grid
    prev = [None] * len(plan.grids)         # the one before
    t_cur = np.full(nl, np.nan)             # mid-step times of those two solves
    t_prev = np.full(nl, np.nan)

    def parent_field(g, tm):
        """The parent's composed field at time tm: linear in time through its two
        latest solves (R27), or its latest alone when it has solved once."""
        p, lp = g.parent, g.level - 1
        if prev[p] is None or t_cur[lp] == t_prev[lp]:
            return fld[p]
        al = (tm - t_prev[lp]) / (t_cur[lp] - t_prev[lp])
        return (1.0 - al) * prev[p] + al * fld[p]

    def level_step(l, h):
        nonlocal x, y, z
        mine = lev >= l                                        # (i) at time clock[l]
        if np.any(mine):
            o = owner_of(plan, x[mine], y[mine], z[mine])
            lev[mine] = np.maximum(l, np.where(o >= 0, level_of[np.maximum(o, 0)], 0))
        tm = clock[l] + 0.5 * h
        dt_p = tm - clock[lev]                                 # (ii) predicted positions
        xp, yp, zp = x + v[0] * dt_p, y + v[1] * dt_p, z + v[2] * dt_p
        for g in plan.level_grids(l):
            rho = deposit_grid(plan, g, xp, yp, zp, m, gas)
            short = convolve(plan, g, rho, cache[g.index])
            prev[g.index] = fld[g.index]
            fld[g.index] = compose(plan, g, short,
                                   parent_field(g, tm) if g.parent >= 0 else None)
        t_prev[l], t_cur[l] = t_cur[l], tm
        sel = np.nonzero(lev == l)[0]                          # (iii) level l moves
        if sel.size:
            o = owner_up_to(plan, xp[sel], yp[sel], zp[sel], l)
            a = interp(plan, fld, o, xp[sel], yp[sel], zp[sel])
            for c in range(3):
                v[c][sel] += h * a[:, c]
            x[sel] = xp[sel] + 0.5 * h * v[0][sel]
            y[sel] = yp[sel] + 0.5 * h * v[1][sel]
            z[sel] = zp[sel] + 0.5 * h * v[2][sel]
        clock[l] += h
        if l + 1 < nl:
            for _ in range(ratio):
                level_step(l + 1, h / ratio)

    def total_energy():
        r = solve(plan, x, y, z, m, gas, cache)
        return r["energy"] + 0.5 * float(np.sum(m * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)))

    pos, vel, en = [np.stack([x, y, z], 1)], [np.stack(v, 1)], []
    if energy:
        en.append(total_energy())
    for _ in range(nroot):
        level_step(0, dt0)
        pos.append(np.stack([x, y, z], 1))
        vel.append(np.stack(v, 1))
        if energy:
            en.append(total_energy())
    return dict(x=x, y=y, z=z, vx=v[0], vy=v[1], vz=v[2], level=lev, pos=np.array(pos),
                vel=np.array(vel), energy=np.array(en))


def wrap_unit(a: np.ndarray) -> np.ndarray:
    """a modulo 1 in [0, 1): a - floor(a), with the value that rounds up to 1 (a tiny
    negative a) mapped to 0, the same point of the periodic box."""
    r = a - np.floor(a)
    return np.where(r >= 1.0, 0.0, r)


def leapfrog(plan: OraclePlan, x, y, z, vx, vy, vz, m, dt: float, nsteps: int,
             gas=None, every: int = 1):
    """Kick-drift-kick leapfrog with every level on the same step (no subcycling,
    Sec. 3.1 and 3.5); the half-step drift between kicks is the time-centring of
    the density described in Sec. 2.  Returns positions recorded every ``every``
    steps (including step 0) and the final state."""
    x, y, z = (np.array(c, np.float64) for c in (x, y, z))
    vx, vy, vz = (np.array(c, np.float64) for c in (vx, vy, vz))
    m = np.asarray(m, np.float64)
    cache = {}

    def accel(px, py, pz):
        r = solve(plan, px, py, pz, m, gas, cache)
        return r["acc"], r["energy"]

    a, w = accel(x, y, z)
    track = [np.stack([x, y, z], axis=1)]
    energy = [w + 0.5 * float(np.sum(m * (vx * vx + vy * vy + vz * vz)))]
    for s in range(nsteps):
        vx += 0.5 * dt * a[:, 0]; vy += 0.5 * dt * a[:, 1]; vz += 0.5 * dt * a[:, 2]
        x += dt * vx; y += dt * vy; z += dt * vz
        if plan.periodic:                                  # R26
            x, y, z = wrap_unit(x), wrap_unit(y), wrap_unit(z)
        a, w = accel(x, y, z)
        vx += 0.5 * dt * a[:, 0]; vy += 0.5 * dt * a[:, 1]; vz += 0.5 * dt * a[:, 2]
        if (s + 1) % every == 0:
            track.append(np.stack([x, y, z], axis=1))
            energy.append(w + 0.5 * float(np.sum(m * (vx * vx + vy * vy + vz * vz))))
    return dict(track=np.array(track), energy=np.array(energy), x=x, y=y, z=z,
                vx=vx, vy=vy, vz=vz)
