"""Seeded synthetic inputs for the APM gravity solve.

This module holds only input generation: grid hierarchies (static nested boxes),
particle positions / masses / velocities and gas density fields.  It contains none
of the solver's arithmetic (no deposit, no Green's function, no FFT, no
differencing), so both the FP64 oracle and the GPU path may import it.

Conventions shared by every generator
-------------------------------------
* The computational domain is the unit box [0, 1)^3 (Passy & Bryan, Sec. 3: the
  coarse grid covers [0;1]^3 in code units), G = 1.
* Level l has cell size 1 / (root_n * 2**l) (refinement factor 2, Sec. 2.2 and
  Sec. 3).  A grid is given by its level, its parent grid index and its active box
  ``lo``/``n`` in level-l global cell indices, as (x, y, z) triples.  Grid 0 is
  always the root grid, covering [0, root_n)^3.
* Gas density fields are numpy arrays shaped (n_z, n_y, n_x) over the active
  cells of a grid (x fastest in memory).
* Positions are float64 arrays; callers that run in FP32 cast them once and feed
  the same cast values to both sides.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "GridSpec",
    "Workload",
    "plummer_positions",
    "plummer_velocities",
    "centred_nested_grids",
    "root_uniform_gas",
    "workload_root32_uniform_gas",
    "workload_plummer_nested",
    "workload_clumps",
    "workload_plummer_gas",
    "workload_large_nested",
    "workload_orbit",
    "workload_point_source",
    "workload_self_force",
    "workload_uniform_sphere",
    "inject_gas",
    "grid_centre_gas",
    "workload_sine_wave",
    "workload_plummer_periodic",
    "BENCH_WORKLOADS",
]

SEED_BASE = 14100010


@dataclasses.dataclass
class GridSpec:
    level: int
    parent: int
    lo: Tuple[int, int, int]
    n: Tuple[int, int, int]


@dataclasses.dataclass
class Workload:
    name: str
    root_n: int
    grids: List[GridSpec]
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    gas: List[Optional[np.ndarray]]            # per grid, active-shaped, or None
    vx: Optional[np.ndarray] = None
    vy: Optional[np.ndarray] = None
    vz: Optional[np.ndarray] = None
    G: float = 1.0
    note: str = ""
    boundary: str = "isolated"                 # root boundary: "isolated" or "periodic"

    @property
    def npart(self) -> int:
        return int(self.x.shape[0])

    def nlevels(self) -> int:
        return 1 + max(g.level for g in self.grids)

    def active_cells(self) -> int:
        return int(sum(int(np.prod(g.n)) for g in self.grids))

    def has_gas(self) -> bool:
        return any(g is not None for g in self.gas)

    def astype(self, dtype) -> "Workload":
        """Cast positions, masses, velocities and gas once (e.g. to float32)."""
        cast = lambda a: None if a is None else np.ascontiguousarray(a.astype(dtype))
        return dataclasses.replace(
            self,
            x=cast(self.x), y=cast(self.y), z=cast(self.z), m=cast(self.m),
            vx=cast(self.vx), vy=cast(self.vy), vz=cast(self.vz),
            gas=[cast(g) for g in self.gas],
        )


# ----------------------------------------------------------------------------
# particle samplers
# ----------------------------------------------------------------------------

def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(1.0 - cz * cz)
    return sz * np.cos(ph), sz * np.sin(ph), cz


def plummer_positions(rng, n, b, centre=(0.5, 0.5, 0.5), lo=0.0, hi=1.0):
    """Plummer sphere of scale radius b: r = b (u^(-2/3) - 1)^(-1/2), isotropic.

    Samples outside [lo, hi)^3 are rejected and redrawn, so exactly n are returned.
    """
    out = np.empty((0, 3))
    while out.shape[0] < n:
        k = int((n - out.shape[0]) * 1.05) + 16
        u = rng.uniform(0.0, 1.0, k)
        u = np.clip(u, 1e-300, 1.0 - 1e-16)
        r = b / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        dx, dy, dz = _isotropic(rng, k)
        p = np.stack([centre[0] + r * dx, centre[1] + r * dy, centre[2] + r * dz], axis=1)
        ok = np.all((p >= lo) & (p < hi), axis=1)
        out = np.concatenate([out, p[ok]], axis=0)
    out = out[:n]
    return out[:, 0].copy(), out[:, 1].copy(), out[:, 2].copy()


def plummer_velocities(rng, x, y, z, b, mass=1.0, G=1.0, centre=(0.5, 0.5, 0.5)):
    """Equilibrium Plummer velocities (Aarseth, Henon & Wielen 1974 rejection method)."""
    n = x.shape[0]
    r = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x4 = rng.uniform(0.0, 1.0, todo.size)
        x5 = rng.uniform(0.0, 1.0, todo.size)
        acc = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        q[todo[acc]] = x4[acc]
        todo = todo[~acc]
    vesc = np.sqrt(2.0 * G * mass / b) * (1.0 + (r / b) ** 2) ** (-0.25)
    v = q * vesc
    dx, dy, dz = _isotropic(rng, n)
    return v * dx, v * dy, v * dz


# ----------------------------------------------------------------------------
# hierarchies
# ----------------------------------------------------------------------------

def centred_nested_grids(root_n, sub_n, nlevels):
    """Root plus ``nlevels`` centred cubic grids of ``sub_n`` active cells each."""
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3)]
    for lev in range(1, nlevels + 1):
        cells = root_n * 2 ** lev
        lo = cells // 2 - sub_n // 2
        grids.append(GridSpec(lev, lev - 1, (lo,) * 3, (sub_n,) * 3))
    return grids


def _box_grid(root_n, level, parent, xlo, xhi):
    cells = root_n * 2 ** level
    lo = int(round(xlo * cells))
    hi = int(round(xhi * cells))
    return GridSpec(level, parent, (lo,) * 3, (hi - lo,) * 3)


# ----------------------------------------------------------------------------
# gas fields
# ----------------------------------------------------------------------------

def root_uniform_gas(root_n, fn):
    """Sample fn(x, y, z) at root cell centres; returns (N, N, N) array [z][y][x]."""
    c = (np.arange(root_n) + 0.5) / root_n
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    return fn(xx, yy, zz)


def grid_centre_gas(root_n, spec, fn):
    """Sample fn(x, y, z) at the cell centres of a grid's active box; (nz, ny, nx)."""
    d = 1.0 / (root_n * 2 ** spec.level)
    cs = [(spec.lo[a] + np.arange(spec.n[a]) + 0.5) * d for a in range(3)]
    zz, yy, xx = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
    return fn(xx, yy, zz)


def inject_gas(parent_gas, parent_spec, child_spec):
    """Piecewise-constant copy of a parent's gas onto a child's active cells."""
    nz, ny, nx = child_spec.n[2], child_spec.n[1], child_spec.n[0]
    iz = (child_spec.lo[2] + np.arange(nz)) // 2 - parent_spec.lo[2]
    iy = (child_spec.lo[1] + np.arange(ny)) // 2 - parent_spec.lo[1]
    ix = (child_spec.lo[0] + np.arange(nx)) // 2 - parent_spec.lo[0]
    return np.ascontiguousarray(parent_gas[np.ix_(iz, iy, ix)])


def gaussian_random_field_gas(rng, n, total_mass=1.0):
    """White noise filtered by k^-1 (P(k) ~ k^-2), k=0 removed, unit variance, lognormal."""
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    kz = np.fft.fftfreq(n)[:, None, None]
    ky = np.fft.fftfreq(n)[None, :, None]
    kx = np.fft.rfftfreq(n)[None, None, :]
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    k[0, 0, 0] = 1.0
    wk = wk / k
    wk[0, 0, 0] = 0.0
    g = np.fft.irfftn(wk, s=(n, n, n))
    g = g / g.std()
    rho = np.exp(g - 0.5)
    dv = (1.0 / n) ** 3
    return rho * (total_mass / (rho.sum() * dv))


# ----------------------------------------------------------------------------
# workloads (each names its sizes; seeds are fixed per workload)
# ----------------------------------------------------------------------------

def workload_root32_uniform_gas(seed=SEED_BASE + 1, root_n=32, npart=4096):
    """Single isolated root 32^3; 4096 particles uniform in [0.25,0.75)^3, m = 1/4096;
    gas: Gaussian blob sigma 0.1 at the box centre, normalised to total gas mass 1."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.25, 0.75, (npart, 3))
    m = np.full(npart, 1.0 / npart)
    gas = root_uniform_gas(root_n, lambda x, y, z: np.exp(
        -((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / (2 * 0.1 ** 2)))
    gas = gas / (gas.sum() * (1.0 / root_n) ** 3)
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3)]
    return Workload(f"root{root_n}_uniform{npart}_gasblob", root_n, grids,
                    p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(), m, [gas])


def workload_plummer_nested(seed=SEED_BASE + 2, root_n=128, sub_n=64, nlevels=2,
                            npart=2 ** 20, b=0.05):
    """Root + centred nested levels, equal-mass Plummer sphere, total mass 1, no gas.
    Particles are kept inside [2 dx_0, 1 - 2 dx_0)^3."""
    rng = np.random.default_rng(seed)
    d0 = 1.0 / root_n
    x, y, z = plummer_positions(rng, npart, b, lo=2 * d0, hi=1 - 2 * d0)
    m = np.full(npart, 1.0 / npart)
    grids = centred_nested_grids(root_n, sub_n, nlevels)
    return Workload(f"plummer{npart}_root{root_n}_{nlevels}x{sub_n}", root_n, grids,
                    x, y, z, m, [None] * len(grids))


def workload_clumps(seed=SEED_BASE + 3, root_n=64, ngrids=256, per_clump=8192,
                    b=0.01, side_lo=8, side_hi=48):
    """Root 64^3 and ``ngrids`` level-1 grids of non-cubic even sides in
    [side_lo, side_hi], each centred on a Plummer clump of ``per_clump`` particles;
    clump centres uniform in [0.15, 0.85]^3, lognormal masses (sigma 1) normalised
    to total 1.  Grids are clamped to stay 2 root cells inside the domain; they may
    overlap (non-overlapping placement of that many boxes cannot fit)."""
    rng = np.random.default_rng(seed)
    d0 = 1.0 / root_n
    l1 = 2 * root_n
    centres = rng.uniform(0.15, 0.85, (ngrids, 3))
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3)]
    xs, ys, zs = [], [], []
    for c in range(ngrids):
        n = tuple(int(2 * rng.integers(side_lo // 2, side_hi // 2 + 1)) for _ in range(3))
        lo = []
        for ax in range(3):
            l = int(round((centres[c, ax] * l1 - n[ax] / 2) / 2)) * 2
            l = max(4, min(l, l1 - 4 - n[ax]))
            lo.append(l)
        grids.append(GridSpec(1, 0, tuple(lo), n))
        x, y, z = plummer_positions(rng, per_clump, b, centre=tuple(centres[c]),
                                    lo=2 * d0, hi=1 - 2 * d0)
        xs.append(x); ys.append(y); zs.append(z)
    m = np.exp(rng.standard_normal(ngrids * per_clump))
    m = m / m.sum()
    return Workload(f"clumps{ngrids}x{per_clump}_root{root_n}", root_n, grids,
                    np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), m,
                    [None] * len(grids))


def workload_plummer_gas(seed=SEED_BASE + 4, root_n=256, sub_n=128, nlevels=2,
                         npart=2 ** 22, b=0.05):
    """Root + centred nested levels, Plummer particles (mass 1) plus a lognormal
    Gaussian-random-field gas (P(k) ~ k^-2, mass 1) on the root; subgrid gas is the
    piecewise-constant injection of the parent's gas."""
    w = workload_plummer_nested(seed, root_n, sub_n, nlevels, npart, b)
    rng = np.random.default_rng(seed + 1000)
    gas = [gaussian_random_field_gas(rng, root_n)]
    for g in w.grids[1:]:
        gas.append(inject_gas(gas[g.parent], w.grids[g.parent], g))
    return dataclasses.replace(w, name=w.name + "_grfgas", gas=gas)


def workload_large_nested(seed=SEED_BASE + 5, root_n=512, sub_n=256, nlevels=3,
                          npart=2 ** 24, b=0.02, with_velocities=True):
    """Root 512^3 + 3 centred 256^3 levels; Plummer (b=0.02, mass 1, equilibrium
    velocities) plus two point masses m=0.1 at centre +-(0.036,0,0) on a circular
    orbit that crosses the finest level's boundary."""
    rng = np.random.default_rng(seed)
    d0 = 1.0 / root_n
    x, y, z = plummer_positions(rng, npart, b, lo=2 * d0, hi=1 - 2 * d0)
    m = np.full(npart, 1.0 / npart)
    vx = vy = vz = None
    if with_velocities:
        vx, vy, vz = plummer_velocities(rng, x, y, z, b)
    r = 0.036
    mp = 0.1
    menc = r ** 3 / (r * r + b * b) ** 1.5
    v = np.sqrt(r * (mp / (2 * r) ** 2 + menc / r ** 2))
    x = np.concatenate([x, [0.5 + r, 0.5 - r]])
    y = np.concatenate([y, [0.5, 0.5]])
    z = np.concatenate([z, [0.5, 0.5]])
    m = np.concatenate([m, [mp, mp]])
    if with_velocities:
        vx = np.concatenate([vx, [0.0, 0.0]])
        vy = np.concatenate([vy, [v, -v]])
        vz = np.concatenate([vz, [0.0, 0.0]])
    grids = centred_nested_grids(root_n, sub_n, nlevels)
    return Workload(f"plummer{npart}+2pm_root{root_n}_{nlevels}x{sub_n}", root_n, grids,
                    x, y, z, m, [None] * len(grids), vx, vy, vz,
                    note=f"point-mass circular speed {v:.6f}")


def workload_orbit(case=2):
    """Two-body orbit (Sec. 3.5): M1 = 1 at the centre, M2 = 0.1 at (0.2, 0.5, 0.5),
    root 16^3.  Case 2: one refined level around the central body.  Case 4: two
    refined levels covering both bodies.  Centre-of-mass-frame circular velocities."""
    root_n = 16
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3)]
    if case == 2:
        grids.append(_box_grid(root_n, 1, 0, 0.375, 0.625))
    elif case == 4:
        grids.append(_box_grid(root_n, 1, 0, 0.125, 0.875))
        grids.append(_box_grid(root_n, 2, 1, 0.1875, 0.8125))
    else:
        raise ValueError("case must be 2 or 4")
    m1, m2, sep = 1.0, 0.1, 0.3
    vrel = np.sqrt((m1 + m2) / sep)
    x = np.array([0.5, 0.2]); y = np.array([0.5, 0.5]); z = np.array([0.5, 0.5])
    m = np.array([m1, m2])
    vy = np.array([vrel * m2 / (m1 + m2), -vrel * m1 / (m1 + m2)])
    zeros = np.zeros(2)
    return Workload(f"orbit_case{case}", root_n, grids, x, y, z, m,
                    [None] * len(grids), zeros.copy(), vy, zeros.copy())


def workload_point_source(corner=False, seed=SEED_BASE + 30, ntest=5000, m_test=1e-10):
    """Point-source test (Sec. 3.2): root 32^3 + one refined grid, central particle of
    density 1 on the finest grid holding it, ``ntest`` test particles of mass 1e-10
    distributed uniformly in log r."""
    root_n = 32
    rng = np.random.default_rng(seed)
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3)]
    if corner:
        grids.append(GridSpec(1, 0, (32, 32, 32), (4, 4, 4)))       # [0.5, 0.5625)^3
    else:
        grids.append(GridSpec(1, 0, (28, 28, 28), (8, 8, 8)))       # [0.4375, 0.5625)^3
    d1 = 1.0 / 64
    mc = 1.0 * d1 ** 3
    lr = rng.uniform(np.log(0.5 * d1), np.log(0.4), ntest)
    r = np.exp(lr)
    dx, dy, dz = _isotropic(rng, ntest)
    x = np.concatenate([[0.5], 0.5 + r * dx])
    y = np.concatenate([[0.5], 0.5 + r * dy])
    z = np.concatenate([[0.5], 0.5 + r * dz])
    m = np.concatenate([[mc], np.full(ntest, m_test)])
    return Workload("point_source_" + ("corner" if corner else "centre"), root_n, grids,
                    x, y, z, m, [None] * len(grids))


def workload_self_force(pos=(0.15, 0.15, 0.15)):
    """Self-force geometry (Sec. 3.1): root 16^3 and three static levels
    [0.1875,0.8125]^3, [0.3125,0.6875]^3, [0.40625,0.59375]^3, one particle of mass 1."""
    root_n = 16
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3),
             _box_grid(root_n, 1, 0, 0.1875, 0.8125),
             _box_grid(root_n, 2, 1, 0.3125, 0.6875),
             _box_grid(root_n, 3, 2, 0.40625, 0.59375)]
    x = np.array([pos[0]]); y = np.array([pos[1]]); z = np.array([pos[2]])
    return Workload("self_force", root_n, grids, x, y, z, np.array([1.0]),
                    [None] * len(grids), np.ones(1), np.ones(1), np.ones(1))


def workload_uniform_sphere(root_n=32, radius=0.3, rho0=1.0, rho_out=1e-10, sub=4):
    """Uniform-density gas sphere (Sec. 3.3, i = 1) of radius 0.3 at the centre on a
    root 32^3 and two static refined levels; cell values are volume averages
    (sub^3 samples per cell).  No particles."""
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3),
             _box_grid(root_n, 1, 0, 0.1875, 0.8125),
             _box_grid(root_n, 2, 1, 0.3125, 0.6875)]
    gas = []
    for g in grids:
        d = 1.0 / (root_n * 2 ** g.level)
        offs = (np.arange(sub) + 0.5) / sub
        ax = [(g.lo[a] + np.arange(g.n[a])[:, None] + offs[None, :]).ravel() * d for a in range(3)]
        zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        inside = ((xx - 0.5) ** 2 + (yy - 0.5) ** 2 + (zz - 0.5) ** 2) <= radius ** 2
        f = inside.reshape(g.n[2], sub, g.n[1], sub, g.n[0], sub).mean(axis=(1, 3, 5))
        gas.append(rho_out + (rho0 - rho_out) * f)
    e = np.zeros(0)
    return Workload("uniform_sphere", root_n, grids, e, e.copy(), e.copy(), e.copy(), gas)


def workload_sine_wave(period=1.0, root_n=64, ntracer=4096, seed=SEED_BASE + 6):
    """The sine wave test (Sec. 3, periodic boundary): gas density
    2 + sin(2 pi x / period) sampled at the cell centres of every grid, a periodic
    root of root_n^3 and two static levels covering [0.34375, 0.65625)^3 (level 1)
    and [0.421875, 0.578125)^3 (level 2).  ``ntracer`` massless particles uniform in
    the box sample the field (their deposit adds nothing)."""
    rng = np.random.default_rng(seed)
    grids = [GridSpec(0, -1, (0, 0, 0), (root_n,) * 3),
             _box_grid(root_n, 1, 0, 0.34375, 0.65625),
             _box_grid(root_n, 2, 1, 0.421875, 0.578125)]
    fn = lambda x, y, z: 2.0 + np.sin(2.0 * np.pi * x / period)
    gas = [grid_centre_gas(root_n, g, fn) for g in grids]
    p = rng.uniform(0.0, 1.0, (ntracer, 3))
    return Workload(f"sine_wave_P{period:g}_root{root_n}", root_n, grids,
                    p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(), np.zeros(ntracer), gas,
                    boundary="periodic")


def workload_plummer_periodic(seed=SEED_BASE + 7, root_n=128, sub_n=64, nlevels=2,
                              npart=2 ** 20, b=0.05):
    """The nested Plummer geometry of workload_plummer_nested with a periodic root:
    equal masses, total mass 1, no gas; positions anywhere in [0, 1)^3 (the tail
    reaches the box edges, where the root's clouds wrap)."""
    rng = np.random.default_rng(seed)
    x, y, z = plummer_positions(rng, npart, b)
    m = np.full(npart, 1.0 / npart)
    grids = centred_nested_grids(root_n, sub_n, nlevels)
    return Workload(f"plummer{npart}_root{root_n}_{nlevels}x{sub_n}_periodic", root_n, grids,
                    x, y, z, m, [None] * len(grids), boundary="periodic")


BENCH_WORKLOADS = {
    "root32_uniform_gas": workload_root32_uniform_gas,
    "plummer_nested": workload_plummer_nested,
    "clumps": workload_clumps,
    "plummer_gas": workload_plummer_gas,
    "large_nested": workload_large_nested,
    "sine_wave": workload_sine_wave,
    "plummer_periodic": workload_plummer_periodic,
}
