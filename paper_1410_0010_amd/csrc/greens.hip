// Green's functions of the APM levels, generated in FP64 on the device (Sec. 2.2).
//
// Subgrids (level l >= 1): the optimal influence function Eq. 5 for the force,
//   Gf(k) = -4 pi G  D*(k) . sum_n U^2(k_n) R_l(k_n) / (|D(k)|^2 [sum_n U^2(k_n)]^2)
// with U^2 = prod sinc^6 (TSC, Eq. 7), the closed-form alias sum Eq. 8, Brillouin
// zones n in [-bz, bz]^3 (Eq. 6) and the short-range reference force
// R_l(q) = -i q (S_l^2(q) - S_{l-1}^2(q)) / q^2 (Eq. 9, S2 shape Eq. 3-4 with
// a_l = a_cells dx_l).  The potential uses the same construction with the gradient
// replaced by the identity: Gp = -4 pi G sum_n U^2 f_l(k_n) / [sum U^2]^2.
// Root (level 0, isolated): the level-0 kernels (reference S_0^2) made isolated as
// the doubled-mesh reference potential (James) plus optimal - reference.  Periodic
// root (Sec. 2.1): the level-0 kernels on the root's own mesh, zero at k = 0.
// Which kernel gives the potential: Sec. 2.2 takes it from Eqs. 2 and 5 and
// differences it in Fourier space.  With the spectral gradient D = -i k that holds
// literally, Gp = Gf, with Gf's removable singularity at k = 0 filled by its limit
// (the n = 0 alias term alone: -4 pi G (a_{l-1}^2 - a_l^2)/30 on a subgrid, the
// James value - pi G dx^2 on the isolated root, 0 on the periodic root); the force
// multipliers -i d vanish at k = 0, so the forces do not see it.  With the two-point
// gradient Eq. 5's kernel is unbounded next to the Nyquist corners (|D| -> 0), and
// the potential takes the potential-optimal Gp above.
// Tables hold the octant |m_i| <= M_i/2 (both kernels are even in every axis),
// scaled by 1/(Mx My Mz) for the unnormalised transforms, at ((|mz| Oy) + |my|) Ox
// + |mx| (Ox = Mx/2 + 1, Oy = My/2 + 1).
#include <cmath>

#include "apm_kernels.hpp"

namespace apm {

constexpr double kPi = 3.14159265358979323846;

// S(eta), eta = k a / 2 (Eq. 4).  Below eta = 1 the closed form cancels badly, so a
// series is used: S = 12 sum_j (-1)^j (2j+2)/(2j+4)! eta^(2j).
__device__ static double s2hat(double eta) {
  if (eta >= 1.0) {
    double s, c;
    sincos(eta, &s, &c);
    const double e2 = eta * eta;
    return 12.0 / (e2 * e2) * (2.0 - 2.0 * c - eta * s);
  }
  const double e2 = eta * eta;
  // coefficients c_j = 12 (-1)^j (2j+2)/(2j+4)!, j = 13..0 (Horner)
  double fact = 1.0;
  double cj[14];
  // (2j+4)! built incrementally: j=0 -> 4! = 24
  fact = 24.0;
  for (int j = 0; j < 14; ++j) {
    if (j > 0) fact *= (double)(2 * j + 3) * (double)(2 * j + 4);
    cj[j] = 12.0 * (double)(2 * j + 2) / fact * ((j & 1) ? -1.0 : 1.0);
  }
  double acc = 0.0;
  for (int j = 13; j >= 0; --j) acc = acc * e2 + cj[j];
  return acc;
}

// f_l(q) = (S(q a_l/2)^2 - S(q a_{l-1}/2)^2) / q^2; for the root (alm1 < 0) S_{-1} = 0.
// When q a_{l-1}/2 < 1 the difference S_l - S_{l-1} is summed as a series in q^2
// whose constant terms cancel exactly.
__device__ static double fref(double q, double al, double alm1) {
  const double sl = s2hat(0.5 * q * al);
  if (alm1 < 0.0) return sl * sl / (q * q);
  if (q == 0.0) return (alm1 * alm1 - al * al) / 30.0;
  const double sm = s2hat(0.5 * q * alm1);
  if (0.5 * q * alm1 >= 1.0) return (sl - sm) * (sl + sm) / (q * q);
  const double q2 = q * q;
  double fact = 24.0, acc = 0.0;
  double coef[14];
  for (int j = 0; j < 14; ++j) {
    if (j > 0) fact *= (double)(2 * j + 3) * (double)(2 * j + 4);
    coef[j] = 12.0 * (double)(2 * j + 2) / fact * ((j & 1) ? -1.0 : 1.0);
  }
  // sum_{j>=1} c_j (al^(2j) - alm1^(2j)) / 4^j q^(2j-2)
  for (int j = 13; j >= 1; --j) {
    const double pl = pow(0.5 * al, 2.0 * j), pm = pow(0.5 * alm1, 2.0 * j);
    acc = acc * q2 + coef[j] * (pl - pm);
  }
  return acc * (sl + sm);
}

__device__ static double sinc6(double k, double dx) {
  const double h = 0.5 * k * dx;
  if (h == 0.0) return 1.0;
  const double s = sin(h) / h;
  const double s2 = s * s;
  return s2 * s2 * s2;
}

__device__ static double alias_sum(double k, double dx) {   // Eq. 8, one axis
  const double s = sin(0.5 * k * dx);
  const double s2 = s * s;
  return 1.0 - s2 + (2.0 / 15.0) * s2 * s2;
}

__device__ static double grad_sym(int m, int M, double dx, int mode) {
  if (2 * m == M) return 0.0;
  const double k = 2.0 * kPi * (double)m / ((double)M * dx);
  return mode == APM_GRAD_FD2 ? sin(k * dx) / dx : k;
}

__global__ void k_influence(InfluenceParams p, double2* __restrict__ out) {
  const int Ox = p.Mx / 2 + 1, Oy = p.My / 2 + 1, Oz = p.Mz / 2 + 1;
  const int64_t total = (int64_t)Ox * Oy * Oz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int mx = (int)(i % Ox), my = (int)((i / Ox) % Oy), mz = (int)(i / ((int64_t)Ox * Oy));
  const double dx = p.dx;
  const double kx = 2.0 * kPi * mx / (p.Mx * dx), ky = 2.0 * kPi * my / (p.My * dx),
               kz = 2.0 * kPi * mz / (p.Mz * dx);
  const double sx = grad_sym(mx, p.Mx, dx, p.grad), sy = grad_sym(my, p.My, dx, p.grad),
               sz = grad_sym(mz, p.Mz, dx, p.grad);
  const double s2 = sx * sx + sy * sy + sz * sz;
  const double c = alias_sum(kx, dx) * alias_sum(ky, dx) * alias_sum(kz, dx);
  const double c2 = c * c;
  const double kg = 2.0 * kPi / dx;
  double numf = 0.0, nump = 0.0;
  for (int nz = -p.bz; nz <= p.bz; ++nz) {
    const double qz = kz + nz * kg, uz = sinc6(qz, dx);
    for (int ny = -p.bz; ny <= p.bz; ++ny) {
      const double qy = ky + ny * kg, uy = sinc6(qy, dx);
      for (int nx = -p.bz; nx <= p.bz; ++nx) {
        const double qx = kx + nx * kg, ux = sinc6(qx, dx);
        const double q = sqrt(qx * qx + qy * qy + qz * qz);
        if (q == 0.0 && p.a_lm1 < 0.0) continue;       // root k = 0: replaced below
        const double u2f = ux * uy * uz * fref(q, p.a_l, p.a_lm1);
        nump += u2f;
        numf += u2f * (sx * qx + sy * qy + sz * qz);
      }
    }
  }
  const double g4 = -4.0 * kPi * p.G;
  double gf = s2 > 0.0 ? g4 * numf / (s2 * c2) : 0.0;
  double gp = g4 * nump / c2;
  const double k2 = kx * kx + ky * ky + kz * kz;
  const bool spectral = p.grad != APM_GRAD_FD2;
  if (p.a_lm1 < 0.0 && !p.james) {
    // periodic root: the level-0 kernels themselves; zero at k = 0 (the mean
    // density carries no potential)
    if (k2 == 0.0) gf = gp = 0.0;
  } else if (p.a_lm1 < 0.0) {
    // isolated root: James reference + (optimal - reference); the difference tends
    // to -pi G dx^2 at k = 0 (for Gp, and for Gf with the spectral gradient)
    const double jm = p.james[((int64_t)mz * Oy + my) * Ox + mx];
    if (k2 == 0.0) {
      gp = jm - kPi * p.G * dx * dx;
      gf = spectral ? gp : jm;
    } else {
      const double sl = s2hat(0.5 * sqrt(k2) * p.a_l);
      const double gref = g4 * sl * sl / k2;
      gf = jm + (gf - gref);
      gp = jm + (gp - gref);
    }
  } else if (k2 == 0.0 && spectral) {
    gf = gp;                                         // subgrid: the k -> 0 limit
  }
  if (spectral) gp = gf;                             // Eq. 2 with Eq. 5's kernel
  // stored kx-fastest, ((mz Oy) + my) Ox + mx: in the z passes neighbouring lanes
  // work on neighbouring kx columns
  out[((int64_t)mz * Oy + my) * Ox + mx] = make_double2(gf * p.norm, gp * p.norm);
}

hipError_t launch_influence(const InfluenceParams& p, double2* out, hipStream_t s) {
  const int64_t total = (int64_t)(p.Mx / 2 + 1) * (p.My / 2 + 1) * (p.Mz / 2 + 1);
  const unsigned nb = (unsigned)((total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_influence, dim3(nb), dim3(kBlock), 0, s, p, out);
  return hipGetLastError();
}

// ---- James doubled-mesh reference kernel on the octant ---------------------------

// P(u): potential shape of two unit S2 clouds, u = 2r/a (1/u beyond u = 2).
__device__ static double s2s2_shape(double u) {
  if (u >= 2.0) return 1.0 / u;
  const double u2 = u * u, u4 = u2 * u2;
  if (u <= 1.0)
    return 52.0 / 35.0 - 0.8 * u2 + 0.4 * u4 - 0.1 * u4 * u - (2.0 / 35.0) * u4 * u2 +
           (3.0 / 140.0) * u4 * u2 * u;
  return 32.0 / 35.0 + 3.0 / (35.0 * u) + 1.6 * u - 3.2 * u2 + 2.0 * u2 * u - 0.4 * u4 -
         0.1 * u4 * u + (2.0 / 35.0) * u4 * u2 - (1.0 / 140.0) * u4 * u2 * u;
}

__global__ void k_james_sample(int N, double dx, double a0, double G, double* __restrict__ g) {
  const int O = N + 1;
  const int64_t total = (int64_t)O * O * O;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const double jx = (double)(i % O), jy = (double)((i / O) % O), jz = (double)(i / ((int64_t)O * O));
  const double r = dx * sqrt(jx * jx + jy * jy + jz * jz);
  g[i] = -G * (2.0 / a0) * s2s2_shape(2.0 * r / a0) * dx * dx * dx;
}

// One axis of the real-even transform on the octant: the DFT over 2N points of a
// sequence even about 0 and N, T(k) = sum_{j=0..N} c_j g(j) cos(pi j k / N),
// c_0 = c_N = 1, else 2.  axis 0 = x (fastest).
__global__ void k_dct1_axis(int N, int axis, const double* __restrict__ costab,
                            const double* __restrict__ in, double* __restrict__ out) {
  const int O = N + 1;
  const int64_t total = (int64_t)O * O * O;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int c[3] = {(int)(i % O), (int)((i / O) % O), (int)(i / ((int64_t)O * O))};
  const int k = c[axis];
  int64_t stride = axis == 0 ? 1 : (axis == 1 ? O : (int64_t)O * O);
  c[axis] = 0;
  const double* base = in + ((int64_t)c[2] * O + c[1]) * O + c[0];
  double acc = 0.0;
  const int twoN = 2 * N;
  for (int j = 0; j <= N; ++j) {
    const double w = (j == 0 || j == N) ? 1.0 : 2.0;
    acc += w * base[j * stride] * costab[(int)(((int64_t)j * k) % twoN)];
  }
  out[i] = acc;
}

hipError_t launch_james(int N, double dx, double a0, double G, const double* costab, double* b0,
                        double* b1, double** result, hipStream_t s) {
  const int64_t total = (int64_t)(N + 1) * (N + 1) * (N + 1);
  const unsigned nb = (unsigned)((total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_james_sample, dim3(nb), dim3(kBlock), 0, s, N, dx, a0, G, b0);
  hipLaunchKernelGGL(k_dct1_axis, dim3(nb), dim3(kBlock), 0, s, N, 0, costab, (const double*)b0, b1);
  hipLaunchKernelGGL(k_dct1_axis, dim3(nb), dim3(kBlock), 0, s, N, 1, costab, (const double*)b1, b0);
  hipLaunchKernelGGL(k_dct1_axis, dim3(nb), dim3(kBlock), 0, s, N, 2, costab, (const double*)b0, b1);
  *result = b1;
  return hipGetLastError();
}

}  // namespace apm
