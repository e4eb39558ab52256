"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(not against the oracle's own formulas).  CPU only.

Each test names the part of the oracle it pins and the fact used: closed forms,
brute force on tiny inputs, invariants, exact special cases, or the accuracy the
paper reports for its own tests (Sec. 3).
"""

import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import apm_workloads as W
from apm_workloads import GridSpec
from oracle import apm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _root_plan(N, **kw):
    return O.OraclePlan(N, [GridSpec(0, -1, (0, 0, 0), (N, N, N))], **kw)


# ---------------------------------------------------------------------------
# P1: TSC assignment
# ---------------------------------------------------------------------------

def test_tsc_weight_moments():
    """Sum 1, centroid t, second central moment 1/4 cell^2 for every offset t."""
    t = np.linspace(-0.5, 0.5, 1001, endpoint=False)
    w = np.array(O.tsc_weights(t))
    j = np.array([-1.0, 0.0, 1.0])[:, None]
    assert np.allclose(w.sum(0), 1.0, atol=1e-15)
    assert np.allclose((w * j).sum(0), t, atol=1e-15)
    assert np.allclose((w * (j - t) ** 2).sum(0), 0.25, atol=1e-15)
    assert (w >= 0).all()


def test_tsc_equals_cic_at_cell_corner():
    """At a cell corner TSC and CIC give the same weights (Sec. 2)."""
    w = O.tsc_weights(np.array([-0.5]))
    assert np.allclose([v[0] for v in w], [0.5, 0.5, 0.0], atol=0)


def _tsc_kernel_1d(s):
    """Textbook TSC shape as a function of distance s (in cells) from the particle."""
    s = np.abs(s)
    return np.where(s <= 0.5, 0.75 - s * s, np.where(s <= 1.5, 0.5 * (1.5 - s) ** 2, 0.0))


def test_deposit_matches_distance_kernel_brute_force():
    """GMF of a subgrid (clipped at its edges) equals sum_p m W(x_c - x_p)/dx^3 written
    with the distance form of the TSC kernel, cell by cell."""
    N = 16
    grids = [GridSpec(0, -1, (0, 0, 0), (N,) * 3), GridSpec(1, 0, (10, 12, 8), (6, 4, 8))]
    plan = O.OraclePlan(N, grids)
    g = plan.grids[1]
    rng = np.random.default_rng(3)
    lo = (g.gmf_lo - 1) * g.dx
    hi = (g.gmf_lo + g.gmf_n + 1) * g.dx
    p = rng.uniform(lo, hi, (40, 3))
    m = rng.uniform(0.5, 2.0, 40)
    rho = O.deposit_particles(plan, g, p[:, 0], p[:, 1], p[:, 2], m)
    ref = np.zeros_like(rho)
    for kz in range(rho.shape[0]):
        for ky in range(rho.shape[1]):
            for kx in range(rho.shape[2]):
                c = (g.gmf_lo + np.array([kx, ky, kz]) + 0.5) * g.dx
                wgt = np.prod(_tsc_kernel_1d((p - c) / g.dx), axis=1)
                ref[kz, ky, kx] = np.sum(m * wgt) / g.dx ** 3
    assert np.allclose(rho, ref, rtol=1e-13, atol=1e-13 * ref.max())


def test_deposit_conserves_mass():
    N = 32
    plan = _root_plan(N)
    rng = np.random.default_rng(5)
    p = rng.uniform(2.0 / N, 1 - 2.0 / N, (5000, 3))
    m = rng.lognormal(0, 1, 5000)
    rho = O.deposit_particles(plan, plan.grids[0], p[:, 0], p[:, 1], p[:, 2], m)
    assert abs(rho.sum() * plan.grids[0].dx ** 3 - m.sum()) <= 1e-13 * m.sum()


def test_out_of_domain_particles_dropped():
    plan = _root_plan(8)
    x = np.array([0.5, -0.1, np.nan, 1.0])
    y = np.array([0.5, 0.5, 0.5, 0.5])
    rho = O.deposit_particles(plan, plan.grids[0], x, y, y, np.ones(4))
    assert abs(rho.sum() / 8 ** 3 - 1.0) < 1e-14
    own = O.owner_of(plan, x, y, y)
    assert list(own) == [0, -1, -1, -1]


def test_ghost_gas_is_parent_copy():
    """Uniform parent gas fills the ghost zone uniformly; a step in the parent gas
    shows up on exactly the child ghost cells inside the parent's stepped cells."""
    N = 16
    grids = [GridSpec(0, -1, (0, 0, 0), (N,) * 3), GridSpec(1, 0, (12, 12, 12), (8, 8, 8))]
    plan = O.OraclePlan(N, grids)
    g = plan.grids[1]
    pg = np.full((N, N, N), 3.0)
    pg[:, :, :7] = 5.0                         # parent x-cells 0..6 -> child x < 14
    rho = O.add_gas(plan, g, np.zeros((14, 14, 14)), [pg, None])
    xs = g.gmf_lo[0] + np.arange(14)
    act = np.zeros((14, 14, 14), bool)
    act[3:11, 3:11, 3:11] = True
    expect = np.where(xs < 14, 5.0, 3.0)[None, None, :] * np.ones((14, 14, 14))
    assert np.array_equal(rho[~act], expect[~act])
    assert np.all(rho[act] == 0.0)


# ---------------------------------------------------------------------------
# P2: S2 sphere (Eq. 3, 4)
# ---------------------------------------------------------------------------

def test_s2_unit_mass():
    a = 0.37
    v, _ = integrate.quad(lambda r: 4 * math.pi * r * r * O.s2_density(r, a), 0, a / 2,
                          epsabs=1e-14, epsrel=1e-13)
    assert abs(v - 1.0) < 1e-12


def test_s2_hat_is_transform_of_s2():
    """Eq. 4 equals the 3-D Fourier transform of Eq. 3 (radial sine transform)."""
    a = 1.0
    for k in (0.3, 1.7, 5.0, 11.0, 23.0):
        v, _ = integrate.quad(lambda r: 4 * math.pi * r * r * O.s2_density(r, a)
                              * math.sin(k * r) / (k * r), 0, a / 2, epsabs=1e-15, epsrel=1e-13)
        assert abs(O.s2_hat(np.array([k * a / 2]))[0] - v) < 1e-11


def test_s2_hat_small_eta_series():
    """The small-argument branch agrees with the closed form evaluated at 40 digits."""
    mp.mp.dps = 40
    for eta in (1e-6, 1e-3, 0.05, 0.3, 0.999, 1.001, 2.0):
        e = mp.mpf(eta)
        ref = 12 / e ** 4 * (2 - 2 * mp.cos(e) - e * mp.sin(e))
        got = O.s2_hat(np.array([eta]))[0]
        assert abs(got - float(ref)) <= 4e-16 * abs(float(ref))


def test_short_range_factor_small_k():
    """f_l(k) = (S_l^2 - S_{l-1}^2)/k^2 at 90 digits, including k -> 0 where the
    difference cancels; f_l(0) = (a_{l-1}^2 - a_l^2)/30."""
    mp.mp.dps = 90
    al, alm1 = 0.0265625, 0.053125

    def S(k, a):
        e = mp.mpf(k) * a / 2
        return 12 / e ** 4 * (2 - 2 * mp.cos(e) - e * mp.sin(e))

    for k in (1e-4, 0.1, 3.0, 30.0, 37.0, 38.0, 200.0):
        ref = (S(k, mp.mpf(al)) ** 2 - S(k, mp.mpf(alm1)) ** 2) / mp.mpf(k) ** 2
        got = O.ref_force_factor(np.array([k]), al, alm1)[0]
        assert abs(got - float(ref)) <= 1e-14 * abs(float(ref)), k
    lim = (alm1 ** 2 - al ** 2) / 30
    got = O.ref_force_factor(np.array([1e-9]), al, alm1)[0]
    assert abs(got - lim) < 1e-12 * lim


# ---------------------------------------------------------------------------
# P3: Eq. 8 is the alias sum of sinc^6 (pins the reading U^2 = sinc^6, R2)
# ---------------------------------------------------------------------------

def test_eq8_is_alias_sum_of_sinc6():
    dx = 1.0
    k = np.linspace(-math.pi, math.pi, 41)
    n = np.arange(-400, 401)
    h = (k[:, None] + 2 * math.pi * n[None, :] / dx) * dx / 2
    sinc = np.where(h == 0, 1.0, np.sin(h) / np.where(h == 0, 1.0, h))
    brute6 = (sinc ** 6).sum(1)
    brute12 = (sinc ** 12).sum(1)
    closed = O._alias_factor(k, dx)
    assert np.allclose(closed, brute6, rtol=0, atol=1e-12)
    assert np.max(np.abs(closed - brute12)) > 0.1        # the printed sinc^6 as U would not match


def _tail_sum(h, power, nmax=4000):
    """sum over |n| >= 2 of sinc^power(h + pi n) (power 6) or (h + pi n)^-5 (power -5),
    by brute force; h is an array of half-angles k dx / 2."""
    n = np.concatenate([np.arange(-nmax, -1), np.arange(2, nmax + 1)]).astype(np.float64)
    a = h[:, None] + math.pi * n[None, :]
    if power == 6:
        return ((np.sin(a) / a) ** 6).sum(1)
    return (a ** -5).sum(1)


@pytest.mark.parametrize("gradient", ["spectral", "fd2"])
def test_eq6_brillouin_zone_sum(gradient):
    """Pins the alias loop of Eq. 5 over the zones n in [-1, 1]^3 (Eq. 6).  With the
    reference factor replaced by 1, the numerators are sums over a product set of
    products of per-axis terms, so they factor:
      potential  sum_n U^2(k_n)       = prod_i S_i,
      force      sum_n U^2(k_n) d.k_n = sum_i d_i T_i prod_{j != i} S_j,
    S_i = sum_{|n| <= 1} sinc^6(h_i + pi n) and T_i = sum_{|n| <= 1} sinc^6(h_i + pi n)
    (k_i + 2 pi n / dx), h_i = k_i dx / 2.  Each axis sum is the infinite one minus its
    |n| >= 2 tail (brute force): for S_i the infinite sum is Eq. 8's closed form, and
    for T_i it is (2/dx) sin^6 h sum_n (h + pi n)^-5 = (2/dx) sin^6 h D4(h) / 24 with
    D4 the fourth derivative of cot, 8 c (1 + c^2)(2 + 3 c^2), c = cot h
    (differentiating sum_n 1/(x + pi n) = cot x four times).  The kernels'
    denominators are taken off with Eq. 8 written out here."""
    dx = 1.0 / 64
    rng = np.random.default_rng(61)
    # random wavenumbers in the first zone plus the Nyquist corner and edges
    m = rng.uniform(-32, 32, (200, 3))
    m[:4] = [[32, 32, 32], [32, 0.5, -7.25], [0.25, 32, 1.5], [-31.9, 3.1, 32]]
    k = 2 * math.pi * m / (64 * dx)
    if gradient == "spectral":
        d = k.copy()
    else:
        d = np.sin(k * dx) / dx
    G = -1.0 / (4 * math.pi)                            # -4 pi G = 1
    one = lambda q: np.ones_like(q)
    kern_f, kern_p = O.influence(k[:, 0], k[:, 1], k[:, 2], dx, 3.4 * dx, 6.8 * dx, G,
                                 (d[:, 0], d[:, 1], d[:, 2]), ref=one)
    h = k * dx / 2
    eq8 = 1.0 - np.sin(h) ** 2 + (2.0 / 15.0) * np.sin(h) ** 4           # per axis
    S = np.stack([eq8[:, i] - _tail_sum(h[:, i], 6) for i in range(3)], 1)
    cot = np.cos(h) / np.sin(h)
    d4cot = 8 * cot * (1 + cot ** 2) * (2 + 3 * cot ** 2)
    T = np.stack([(2 / dx) * np.sin(h[:, i]) ** 6 * (d4cot[:, i] / 24 - _tail_sum(h[:, i], -5))
                  for i in range(3)], 1)
    den = np.prod(eq8, 1) ** 2
    num_p = kern_p * den
    assert np.allclose(num_p, np.prod(S, 1), rtol=1e-11, atol=0)
    num_f_ref = (d[:, 0] * T[:, 0] * S[:, 1] * S[:, 2] + d[:, 1] * T[:, 1] * S[:, 0] * S[:, 2]
                 + d[:, 2] * T[:, 2] * S[:, 0] * S[:, 1])
    s2 = (d * d).sum(1)
    num_f = kern_f * s2 * den
    scale = np.abs(d).sum(1) * np.abs(T).max(1) + 1e-300
    assert np.all(np.abs(num_f - num_f_ref) <= 1e-10 * scale)
    # the zones matter: one zone (n = 0 only) misses by O(1) at the Nyquist corner
    f0, p0 = O.influence(k[:1, 0], k[:1, 1], k[:1, 2], dx, 3.4 * dx, 6.8 * dx, G,
                         (d[:1, 0], d[:1, 1], d[:1, 2]), bz=0, ref=one)
    assert abs(p0[0] * den[0] / np.prod(S[0]) - 1) > 0.5


# ---------------------------------------------------------------------------
# P4: S2-S2 reference potential
# ---------------------------------------------------------------------------

def test_reference_potential_is_hankel_transform():
    """P(2r/a)/(2 pi a) = 1/(2 pi^2 r) int S^2(k) sin(kr)/k dk: the potential whose
    source is the S2 self-convolution (unit-charge units)."""
    mp.mp.dps = 25
    a = mp.mpf("0.7")

    def Shat(k):
        e = k * a / 2
        return 12 / e ** 4 * (2 - 2 * mp.cos(e) - e * mp.sin(e))

    for r in ("0.07", "0.33", "0.62", "0.9", "1.4"):
        r = mp.mpf(r)
        num = mp.quadosc(lambda k: Shat(k) ** 2 * mp.sin(k * r) / k, [0, mp.inf], omega=r)
        num = num / (2 * mp.pi ** 2 * r)
        got = O.s2s2_potential_shape(np.array([float(2 * r / a)]))[0] / (2 * math.pi * float(a))
        assert abs(got - float(num)) < 1e-13 * abs(float(num)), r


def test_reference_potential_shape_properties():
    u = np.array([1.0 - 1e-12, 1.0 + 1e-12, 2.0 - 1e-12, 2.0 + 1e-12])
    P = O.s2s2_potential_shape(u)
    dP = O.s2s2_potential_shape_deriv(u)
    assert abs(P[0] - P[1]) < 1e-10 and abs(P[2] - P[3]) < 1e-10
    assert abs(dP[0] - dP[1]) < 1e-10 and abs(dP[2] - dP[3]) < 1e-10
    a = 0.3
    assert abs(O.root_kernel(np.array([0.0]), a, 1.0)[0] + 104.0 / (35.0 * a)) < 1e-13
    r = np.linspace(a, 3 * a, 7)
    assert np.allclose(O.root_kernel(r, a, 1.0), -1.0 / r, rtol=1e-15)
    # derivative by central differences
    uu = np.array([0.3, 0.8, 1.2, 1.7, 2.5])
    h = 1e-6
    fd = (O.s2s2_potential_shape(uu + h) - O.s2s2_potential_shape(uu - h)) / (2 * h)
    assert np.allclose(O.s2s2_potential_shape_deriv(uu), fd, atol=1e-9)


# ---------------------------------------------------------------------------
# P5, P6, P7: convolution machinery
# ---------------------------------------------------------------------------

def test_james_doubled_mesh_equals_direct_sum():
    """The cyclic convolution on (2N)^3 with the mirrored kernel equals the isolated
    direct real-space sum on the root (James 1977)."""
    N = 8
    plan = _root_plan(N)
    rng = np.random.default_rng(11)
    rho = np.zeros((N, N, N))
    idx = rng.integers(0, N, (12, 3))
    rho[idx[:, 2], idx[:, 1], idx[:, 0]] = rng.uniform(0.5, 2, 12)
    got = O.convolve_scalar(plan.grids[0], rho, O.greens_root_james(plan))
    ref = O.direct_root_potential(plan, rho)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_cyclic_convolution_odd_noncubic_brute_force():
    """irfft(K_hat * rfft(pad)) restricted to the output box is the cyclic sum
    sum_j rho(j) k((i - j) mod M), for odd and non-cubic M and a ghost offset."""
    M = np.array([9, 10, 7])
    rng = np.random.default_rng(2)
    k = rng.standard_normal((M[2], M[1], M[0]))
    for ax in range(3):                                   # make k even in each axis
        k = 0.5 * (k + np.flip(np.roll(k, -1, axis=ax), axis=ax))
        k = np.roll(k, 1, axis=ax) if False else k
    kz, ky, kx = np.meshgrid(*(np.arange(m) for m in M[::-1]), indexing="ij")
    kern = np.cos(0.3 * np.minimum(kx, M[0] - kx)) + 0.2 * np.minimum(ky, M[1] - ky) ** 2 \
        - 0.1 * np.minimum(kz, M[2] - kz)
    khat = np.fft.rfftn(kern)
    g = O.OGrid(1, 1, 0, np.array([3, 3, 3]), np.array([2, 3, 1]), 0.1,
                np.array([0, 0, 0]), np.array([5, 6, 4]), np.array([2, 2, 2]),
                np.array([4, 5, 3]), M)
    rho = rng.standard_normal((4, 6, 5))
    got = O.convolve_scalar(g, rho, khat)
    ref = np.zeros_like(got)
    for oz in range(got.shape[0]):
        for oy in range(got.shape[1]):
            for ox in range(got.shape[2]):
                i = np.array([ox, oy, oz]) + g.fld_lo - g.gmf_lo
                s = 0.0
                for jz in range(4):
                    for jy in range(6):
                        for jx in range(5):
                            d = (i - np.array([jx, jy, jz])) % M
                            s += rho[jz, jy, jx] * kern[d[2], d[1], d[0]]
                ref[oz, oy, ox] = s
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_kspace_difference_is_two_point_stencil():
    """With the two-point option, the Fourier-space gradient -i sin(k dx)/dx equals
    the real-space difference -(phi(c+1) - phi(c-1))/(2 dx) of the same kernel's
    potential (R6): sign, factor and axis order."""
    N = 16
    plan = _root_plan(N, gradient="fd2")
    g = plan.grids[0]
    rng = np.random.default_rng(4)
    p = rng.uniform(0.3, 0.7, (30, 3))
    rho = O.deposit_particles(plan, g, p[:, 0], p[:, 1], p[:, 2], np.ones(30))
    gf, gp = O.greens(plan, g)
    F = O.convolve(plan, g, rho, (gf, gp))
    phiF = O.convolve_scalar(g, rho, gf)
    s = slice(1, N - 1)
    ax = -(phiF[s, s, 2:] - phiF[s, s, :-2]) / (2 * g.dx)
    ay = -(phiF[s, 2:, s] - phiF[s, :-2, s]) / (2 * g.dx)
    az = -(phiF[2:, s, s] - phiF[:-2, s, s]) / (2 * g.dx)
    scale = np.abs(F[..., :3]).max()
    assert np.abs(F[s, s, s, 0] - ax).max() < 1e-9 * scale
    assert np.abs(F[s, s, s, 1] - ay).max() < 1e-9 * scale
    assert np.abs(F[s, s, s, 2] - az).max() < 1e-9 * scale


def test_fourier_gradient_exact_on_band_limited_field():
    """On a periodic mesh the spectral gradient of a band-limited field is its exact
    derivative (a = -d rho/dx here, kernels = 1), the two-point one is
    sin(k dx)/dx times it, and the Nyquist mode has zero derivative."""
    M = np.array([16, 12, 10])
    g = O.OGrid(0, 1, 0, np.zeros(3, int), M, 1.0 / 16, np.zeros(3, int), M.copy(),
                np.zeros(3, int), M.copy(), M.copy())
    ix, iy, iz = (np.arange(v) for v in M)
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    kx, ky, kz = 2 * math.pi * 3 / (16 * g.dx), 2 * math.pi * 2 / (12 * g.dx), 2 * math.pi / (10 * g.dx)
    px, py, pz = kx * X * g.dx, ky * Y * g.dx, kz * Z * g.dx
    rho = np.sin(px) * np.cos(py) * np.sin(pz) + 0.7 * np.cos(math.pi * X)   # + x-Nyquist mode
    ones = np.ones((10, 12, 9))
    for mode, fac in (("spectral", lambda k: k), ("fd2", lambda k: math.sin(k * g.dx) / g.dx)):
        plan = _root_plan(8, gradient=mode)
        F = O.convolve(plan, g, rho, (ones, ones))
        assert np.allclose(F[..., 3], rho, atol=1e-13)
        assert np.allclose(F[..., 0], -fac(kx) * np.cos(px) * np.cos(py) * np.sin(pz), atol=1e-11)
        assert np.allclose(F[..., 1], fac(ky) * np.sin(px) * np.sin(py) * np.sin(pz), atol=1e-11)
        assert np.allclose(F[..., 2], -fac(kz) * np.sin(px) * np.cos(py) * np.cos(pz), atol=1e-11)


def test_green_functions_real_even_and_cube_symmetric():
    """The mirrored James kernel has a real DFT; the influence functions on a cubic
    mesh are invariant under the 48 symmetries of the cube (axis swaps and
    reflections k -> -k)."""
    N = 8
    plan = O.OraclePlan(N, [GridSpec(0, -1, (0, 0, 0), (N,) * 3),
                            GridSpec(1, 0, (4, 4, 4), (8, 8, 8))])
    j = np.arange(2 * N)
    jm = np.minimum(j, 2 * N - j)
    r = np.sqrt(jm[:, None, None] ** 2 + jm[None, :, None] ** 2 + jm[None, None, :] ** 2) / N
    full = np.fft.fftn(O.root_kernel(r, plan.a_soft(0), 1.0))
    assert np.abs(full.imag).max() < 1e-12 * np.abs(full.real).max()
    for g in plan.grids:
        for K in O.greens(plan, g):
            M = int(g.M[0])
            # expand the rfft half to the full cube using evenness in x
            fullk = np.concatenate([K, K[:, :, 1:M // 2][:, :, ::-1]], axis=2)
            assert fullk.shape == (M, M, M)
            tol = 1e-13 * np.abs(fullk).max()
            for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)]:
                assert np.abs(np.transpose(fullk, perm) - fullk).max() < tol
            refl = np.roll(np.flip(fullk, axis=1), 1, axis=1)
            assert np.abs(refl - fullk).max() < tol


# ---------------------------------------------------------------------------
# P8 - P12: physics of the whole solve
# ---------------------------------------------------------------------------

def test_point_mass_far_field():
    """Single particle on an isolated root: Phi -> -GM/r and a -> -GM r_hat/r^2 away
    from the softening scale.

    Bound on the potential, from the kernel's construction: the root kernel is the
    James reference potential (exactly -G/r beyond a_0, P4-P5) plus the short-range
    difference optimal - reference (its real-space form cK on the doubled mesh).  At
    a mesh point x whose distance to every cloud cell exceeds a_0,
        Phi(x) = -G sum_c w_c / |x - x_c| + sum_c w_c cK(x - x_c),
    so |Phi d + 1| <= |d sum_c w_c / |x - x_c| - 1| + d max_c |cK(x - x_c)|: the
    cloud's multipole error (brute force with the textbook TSC kernel) plus the size
    of the optimal - reference correction.  Checked point by point beyond 2.5 a_0."""
    N = 32
    plan = _root_plan(N)
    x, y, z = np.array([0.5 + 0.27 / N]), np.array([0.5 - 0.11 / N]), np.array([0.5 + 0.4 / N])
    r = O.solve(plan, x, y, z, np.array([1.0]))
    F = r["field"][0]
    g = plan.grids[0]
    dx, M = g.dx, 2 * N
    c = (np.arange(N) + 0.5) / N
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    d = np.sqrt((X - x[0]) ** 2 + (Y - y[0]) ** 2 + (Z - z[0]) ** 2)
    far = d > 2.5 * plan.a_soft(0)
    # correction kernel: potential of a unit point mass at a mesh offset
    cK = np.fft.irfftn(O.greens(plan, g)[1] - O.greens_root_james(plan), s=(M, M, M),
                       axes=(0, 1, 2)) / dx ** 3
    p = np.array([x[0], y[0], z[0]]) / dx
    i0 = np.floor(p).astype(int)
    cloud = [(i0 + np.array(o), float(np.prod(_tsc_kernel_1d(i0 + np.array(o) + 0.5 - p))))
             for o in np.ndindex(3, 3, 3) for o in [np.array(o) - 1]]
    assert abs(sum(w for _, w in cloud) - 1.0) < 1e-14
    idx = np.argwhere(far)
    xm = idx[:, ::-1]                                   # (x, y, z) cell indices
    multipole = np.zeros(len(idx))
    corr = np.zeros(len(idx))
    for cc, w in cloud:
        multipole += w / (np.linalg.norm(xm - cc, axis=1) * dx)
        off = (xm - cc) % M
        corr = np.maximum(corr, np.abs(cK[off[:, 2], off[:, 1], off[:, 0]]))
    dd = d[far]
    bound = np.abs(dd * multipole - 1.0) + dd * corr
    err = np.abs(F[..., 3][far] * dd + 1.0)
    assert np.all(err <= bound * (1 + 1e-9) + 1e-12)
    assert bound.max() < 2e-3                           # the far field is -GM/r to 0.2%
    # pair force on TSC-interpolated test particles (what the optimal kernel targets)
    src = np.array([x[0], y[0], z[0]])
    rr, lev, erad, etan, pr = _radial_errors(plan, r["field"], src, 2.5 * plan.a_soft(0),
                                             0.45, 2000, 21)
    assert abs(np.mean(erad)) < 2e-3 and np.abs(erad).max() < 5e-2
    assert np.mean(etan) < 1e-2
    assert np.abs(pr + 1).max() < 2e-4


def test_no_self_force_single_level():
    """One particle on one level feels no force (even W, odd D, same W for assignment
    and interpolation); Sec. 3.1 reports ~1e-14 for the APM solver."""
    N = 16
    plan = _root_plan(N)
    rng = np.random.default_rng(8)
    for _ in range(5):
        p = rng.uniform(0.3, 0.7, 3)
        r = O.solve(plan, p[:1], p[1:2], p[2:], np.array([1.0]))
        scale = 1.0 / plan.grids[0].dx ** 2
        assert np.abs(r["acc"]).max() < 1e-13 * scale


def test_self_force_nested_is_small():
    """Self-force geometry of Sec. 3.1 (root 16^3 + three levels): a particle on the
    deepest level feels an acceleration at rounding level relative to the force a
    neighbouring cell's mass would exert."""
    w = W.workload_self_force((0.5 + 0.13 / 128, 0.5 - 0.21 / 128, 0.5 + 0.05 / 128))
    plan = O.OraclePlan(w.root_n, w.grids)
    r = O.solve(plan, w.x, w.y, w.z, w.m)
    assert r["owner"][0] == 3
    scale = 1.0 / plan.grids[3].dx ** 2
    assert np.abs(r["acc"]).max() < 1e-12 * scale


def test_newton_third_law_single_level():
    N = 16
    plan = _root_plan(N)
    rng = np.random.default_rng(9)
    p = rng.uniform(0.2, 0.8, (200, 3))
    m = rng.lognormal(0, 1, 200)
    r = O.solve(plan, p[:, 0], p[:, 1], p[:, 2], m)
    tot = np.abs(m[:, None] * r["acc"]).sum()
    assert np.abs(r["net_force"]).max() < 1e-13 * tot


def test_uniform_sphere_potential_percent_level():
    """Sec. 3.3, i = 1: uniform sphere R = 0.3 on a 32^3 root and two levels; the
    potential and radial acceleration match Gauss's law at the percent level."""
    w = W.workload_uniform_sphere()
    plan = O.OraclePlan(w.root_n, w.grids)
    r = O.solve(plan, w.x, w.y, w.z, w.m, w.gas)
    R = 0.3
    M = 4.0 / 3.0 * math.pi * R ** 3 * (1 - 1e-10)
    for g in plan.grids:
        F = r["field"][g.index]
        o = g.lo - g.fld_lo
        F = F[o[2]:o[2] + g.n[2], o[1]:o[1] + g.n[1], o[0]:o[0] + g.n[0]]
        cs = [(g.lo[a] + np.arange(g.n[a]) + 0.5) * g.dx for a in range(3)]
        Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
        rr = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
        ana = np.where(rr <= R, -M / (2 * R) * (3 - rr ** 2 / R ** 2), -M / rr)
        assert np.abs(F[..., 3] / ana - 1).max() < 0.01
        sel = rr > 4 * g.dx
        arad = -(F[..., 0] * (X - 0.5) + F[..., 1] * (Y - 0.5) + F[..., 2] * (Z - 0.5)) / rr
        aana = np.where(rr <= R, M * rr / R ** 3, M / rr ** 2)
        assert np.mean(np.abs(arad[sel] / aana[sel] - 1)) < 0.01


def _radial_errors(plan, field, src, rr_lo, rr_hi, n, seed):
    rng = np.random.default_rng(seed)
    rr = np.exp(rng.uniform(np.log(rr_lo), np.log(rr_hi), n))
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    t = src[None, :] + rr[:, None] * u
    own = O.owner_of(plan, t[:, 0], t[:, 1], t[:, 2])
    pa = O.interp(plan, field, own, t[:, 0], t[:, 1], t[:, 2])
    arad = -(pa[:, :3] * u).sum(1)
    atan = np.linalg.norm(pa[:, :3] + arad[:, None] * u, axis=1)
    lev = np.array([plan.grids[o].level for o in own])
    return rr, lev, arad * rr ** 2 - 1.0, atan * rr ** 2, pa[:, 3] * rr


def test_force_decomposition_telescopes_to_newton():
    """Fig. 1 geometry (32^3 root, three levels): the composed force on each level
    follows GM/r^2 beyond that level's softening a_l (the reference forces of Eq. 9
    telescope to S_L^2, which needs the square at l = 0, R3)."""
    gold = json.load(open(GOLDEN))["finest_cell_fig1"]
    geo = gold["geometry"]
    grids = [GridSpec(0, -1, (0, 0, 0), (32,) * 3)]
    for lev, (a, b) in enumerate(geo["levels"], start=1):
        cells = 32 * 2 ** lev
        lo, hi = int(round(a * cells)), int(round(b * cells))
        grids.append(GridSpec(lev, lev - 1, (lo,) * 3, (hi - lo,) * 3))
    plan = O.OraclePlan(32, grids)
    assert abs(plan.grids[3].dx - gold["value"]) < 5e-7
    src = np.array([0.5 + 0.13 / 256, 0.5 - 0.21 / 256, 0.5 + 0.05 / 256])
    r = O.solve(plan, src[:1], src[1:2], src[2:], np.array([1.0]))
    rr, lev, erad, etan, pr = _radial_errors(plan, r["field"], src, 0.003, 0.45, 3000, 1)
    for L in range(4):
        sel = (lev == L) & (rr > 1.2 * plan.a_soft(L))
        assert sel.sum() > 50
        assert abs(np.mean(erad[sel])) < 0.015, L
        assert np.mean(np.abs(erad[sel])) < 0.08, L
        assert np.mean(etan[sel]) < 0.03, L
        assert np.abs(pr[sel] + 1).max() < 0.03, L


def test_point_source_test_sec32():
    """Sec. 3.2: central particle of density 1 on a refined grid, 5000 light test
    particles.  Mean radial / tangential errors are a few percent and the central
    particle feels no self-force (paper: ~1e-11 centre, ~1e-10 corner).  The test
    masses are made negligible here (the paper's 1e-10 adds a few percent of the
    central mass) so that GM/r^2 is the exact target."""
    for corner in (False, True):
        w = W.workload_point_source(corner=corner, ntest=2000, m_test=1e-20)
        plan = O.OraclePlan(w.root_n, w.grids)
        r = O.solve(plan, w.x, w.y, w.z, w.m)
        src = np.array([w.x[0], w.y[0], w.z[0]])
        d = np.stack([w.x[1:], w.y[1:], w.z[1:]], 1) - src
        rr = np.linalg.norm(d, axis=1)
        u = d / rr[:, None]
        a = r["acc"][1:]
        M = w.m[0]
        arad = -(a * u).sum(1) * rr ** 2 / M
        atan = np.linalg.norm(a + (arad * M / rr ** 2)[:, None] * u, axis=1) * rr ** 2 / M
        sel = rr > 2 * plan.a_soft(1)
        assert abs(np.mean(arad[sel] - 1)) < 0.01
        assert np.mean(atan[sel]) < 0.02
        # central particle: its own force scale is G m / dx_1^2 ~ 1.5e-2
        assert np.abs(r["acc"][0]).max() < 1e-14


# ---------------------------------------------------------------------------
# P13, P16 - P18
# ---------------------------------------------------------------------------

def test_potential_kernel_continuous_at_k0():
    """Subgrid potential kernel tends to -4 pi G (a_{l-1}^2 - a_l^2)/30 as k -> 0, and
    the force kernel's mesh force -i s G_f tends to 0 there."""
    dx, al, alm1 = 1 / 64, 3.4 / 64, 6.8 / 64
    k = np.array([1e-7, 1e-5])
    z = np.zeros(1)
    for d in (k, np.sin(k * dx) / dx):
        f, p = O.influence(k, z, z, dx, al, alm1, 1.0, (d, z, z))
        lim = -4 * math.pi * (alm1 ** 2 - al ** 2) / 30
        assert np.allclose(p, lim, rtol=1e-8)
        assert np.all(np.abs(d * f) < 1e-3 * abs(lim))


def test_linearity_and_G_scaling():
    w = W.workload_plummer_nested(root_n=16, sub_n=8, nlevels=1, npart=300)
    plan = O.OraclePlan(w.root_n, w.grids)
    plan2 = O.OraclePlan(w.root_n, w.grids, G=2.5)
    r1 = O.solve(plan, w.x, w.y, w.z, w.m)
    r2 = O.solve(plan, w.x, w.y, w.z, 3.0 * w.m)
    r3 = O.solve(plan2, w.x, w.y, w.z, w.m)
    for a, b, s in ((r1, r2, 3.0), (r1, r3, 2.5)):
        for f1, f2 in zip(a["field"], b["field"]):
            assert np.allclose(s * f1, f2, rtol=1e-12, atol=1e-12 * np.abs(f2).max())
        assert np.allclose(s * a["acc"], b["acc"], rtol=1e-12, atol=1e-12 * np.abs(b["acc"]).max())


def test_integer_cell_translation():
    N = 16
    plan = _root_plan(N)
    rng = np.random.default_rng(12)
    p = rng.uniform(0.35, 0.6, (20, 3))
    sh = np.array([2, 1, 3]) / N
    r1 = O.solve(plan, p[:, 0], p[:, 1], p[:, 2], np.ones(20))
    r2 = O.solve(plan, p[:, 0] + sh[0], p[:, 1] + sh[1], p[:, 2] + sh[2], np.ones(20))
    F1, F2 = r1["field"][0], r2["field"][0]
    assert np.allclose(F1[:N - 3, :N - 1, :N - 2], F2[3:, 1:, 2:], rtol=1e-11,
                       atol=1e-11 * np.abs(F1).max())
    assert np.allclose(r1["acc"], r2["acc"], rtol=1e-10, atol=1e-10 * np.abs(r1["acc"]).max())


def test_axis_permutation_permutes_solution():
    """Swapping x and y of the input (grids and particles) swaps the output fields and
    accelerations; catches axis and stride bugs."""
    grids = [GridSpec(0, -1, (0, 0, 0), (16,) * 3), GridSpec(1, 0, (10, 12, 12), (12, 8, 6))]
    gridsT = [GridSpec(0, -1, (0, 0, 0), (16,) * 3), GridSpec(1, 0, (12, 10, 12), (8, 12, 6))]
    rng = np.random.default_rng(13)
    p = rng.uniform(0.35, 0.65, (50, 3))
    m = rng.uniform(0.5, 1.5, 50)
    r1 = O.solve(O.OraclePlan(16, grids), p[:, 0], p[:, 1], p[:, 2], m)
    r2 = O.solve(O.OraclePlan(16, gridsT), p[:, 1], p[:, 0], p[:, 2], m)
    for F1, F2 in zip(r1["field"], r2["field"]):
        F1T = np.swapaxes(F1, 1, 2)[..., [1, 0, 2, 3]]
        assert np.allclose(F1T, F2, rtol=1e-11, atol=1e-11 * np.abs(F1).max())
    assert np.allclose(r1["acc"][:, [1, 0, 2]], r2["acc"], rtol=1e-10,
                       atol=1e-10 * np.abs(r1["acc"]).max())


# ---------------------------------------------------------------------------
# P14: orbit across a nested-grid boundary (Sec. 3.5, case 2, no subcycling)
# ---------------------------------------------------------------------------

def test_two_body_orbit_across_levels():
    """Central body on level 1, light body on the root; one orbit with a single
    timestep for all levels.  Separation and centre of mass stay put to the orders
    the paper reports for its no-subcycling cases (Sec. 3.5.2)."""
    gold = json.load(open(GOLDEN))["orbit_case4"]
    w = W.workload_orbit(case=2)
    plan = O.OraclePlan(w.root_n, w.grids)
    own = O.owner_of(plan, w.x, w.y, w.z)
    assert list(own) == [1, 0]
    T = 2 * math.pi * math.sqrt(0.3 ** 3 / 1.1)
    dt = 3e-3
    n = int(round(T / dt))
    res = O.leapfrog(plan, w.x, w.y, w.z, w.vx, w.vy, w.vz, w.m, dt, n, every=10)
    tr = res["track"]
    sep = np.linalg.norm(tr[:, 1] - tr[:, 0], axis=1)
    com = (w.m[None, :, None] * tr).sum(1) / w.m.sum()
    assert np.abs(sep / 0.3 - 1).max() < 2 * gold["separation_change"]
    assert np.abs(com - com[0]).max() < 10 * gold["com_drift"]


# ---------------------------------------------------------------------------
# direct pins of composition, interpolation, energy and the PP reference
# ---------------------------------------------------------------------------

def test_prolong_and_interp_reproduce_linear_fields():
    """Trilinear cell-centre interpolation and TSC interpolation are exact for
    fields linear in position (weights sum to 1, first moments exact)."""
    grids = [GridSpec(0, -1, (0, 0, 0), (16,) * 3), GridSpec(1, 0, (10, 8, 12), (8, 12, 6))]
    plan = O.OraclePlan(16, grids)
    par, g = plan.grids
    coef = np.array([0.3, -1.7, 2.2, 0.9])

    def lin(X, Y, Z):
        return coef[0] + coef[1] * X + coef[2] * Y + coef[3] * Z

    def field_on(gr):
        cs = [(gr.fld_lo[a] + np.arange(gr.fld_n[a]) + 0.5) * gr.dx for a in range(3)]
        Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
        return np.stack([lin(X, Y, Z)] * 4, axis=-1), (X, Y, Z)

    Fp, _ = field_on(par)
    Fc, (X, Y, Z) = field_on(g)
    assert np.allclose(O.prolong(Fp, par, g), Fc, atol=1e-13)
    rng = np.random.default_rng(17)
    lo = (g.lo + 0.0) * g.dx
    hi = (g.lo + g.n) * g.dx
    p = rng.uniform(lo, hi, (200, 3))
    own = np.full(200, 1)
    pa = O.interp(plan, [None, Fc], own, p[:, 0], p[:, 1], p[:, 2])
    assert np.allclose(pa[:, 3], lin(p[:, 0], p[:, 1], p[:, 2]), atol=1e-13)


def test_energy_pair_reciprocity():
    """On one level the interaction energy is symmetric: m1 Phi_2(x1) = m2 Phi_1(x2),
    and W(m1, m2) - W(m1, 0) - W(0, m2) is that pair term, close to -G m1 m2 / r."""
    plan = _root_plan(32)
    x = np.array([0.31, 0.66]); y = np.array([0.42, 0.57]); z = np.array([0.5, 0.38])
    m = np.array([1.3, 0.7])
    r12 = O.solve(plan, x, y, z, m)["energy"]
    r1 = O.solve(plan, x, y, z, np.array([m[0], 0.0]))
    r2 = O.solve(plan, x, y, z, np.array([0.0, m[1]]))
    pair = r12 - r1["energy"] - r2["energy"]
    assert abs(m[0] * r2["pot"][0] - m[1] * r1["pot"][1]) < 1e-12 * abs(pair)
    assert abs(pair - m[0] * r2["pot"][0]) < 1e-12 * abs(pair)
    d = math.sqrt((x[0] - x[1]) ** 2 + (y[0] - y[1]) ** 2 + (z[0] - z[1]) ** 2)
    assert abs(pair / (-m[0] * m[1] / d) - 1) < 1e-3


def test_mesh_forces_match_direct_pp_sum():
    """A small cluster on the finest of two levels: mesh accelerations match the
    direct O(N^2) sum with the S2-S2 reference force at the finest softening."""
    grids = W.centred_nested_grids(16, 16, 2)
    plan = O.OraclePlan(16, grids)
    rng = np.random.default_rng(19)
    p = 0.5 + rng.uniform(-0.09, 0.09, (40, 3))
    m = rng.uniform(0.5, 1.5, 40)
    r = O.solve(plan, p[:, 0], p[:, 1], p[:, 2], m)
    assert (r["owner"] == 2).all()
    ref = O.pp_reference_accel(p[:, 0], p[:, 1], p[:, 2], m, plan.a_soft(2))
    err = np.linalg.norm(r["acc"] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.median(err) < 0.02 and err.max() < 0.08


def test_greens_on_plane_ranges_equal_whole_grid():
    """The kernels of a range of kz planes are those planes of the whole grid's kernels
    (subgrid and isolated root; both gradients)."""
    grids = [GridSpec(0, -1, (0, 0, 0), (8,) * 3), GridSpec(1, 0, (4, 4, 6), (8, 6, 4))]
    for grad in ("spectral", "fd2"):
        plan = O.OraclePlan(8, grids, gradient=grad)
        for g in plan.grids:
            whole = O.greens(plan, g)
            Mz = int(g.M[2])
            cuts = [0, 3, Mz // 2, Mz // 2 + 1, Mz]
            for p0, p1 in zip(cuts[:-1], cuts[1:]):
                part = O.greens(plan, g, planes=(p0, p1))
                for a, b in zip(part, whole):
                    assert np.array_equal(a, b[p0:p1])
