// Time integration and energy terms: kick-drift-kick leapfrog with every level on
// the same step (no subcycling, Sec. 3.1 and 3.5), the kinetic energy, and the gas
// part of the potential energy.
#include "apm_kernels.hpp"

namespace apm {

// Position modulo 1 in [0, 1) (periodic box); a value that rounds up to 1 is 0.
template <typename T> __device__ __forceinline__ T wrap_unit(T v) {
  v -= floor(v);
  return v >= (T)1 ? (T)0 : v;
}

// v += hk a, then x += hd v (hd = 0: a kick alone; hk = 0: a drift alone); wrap: the
// drifted positions are taken modulo 1.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_kick_drift(int64_t n, T* __restrict__ x, T* __restrict__ y, T* __restrict__ z,
             T* __restrict__ vx, T* __restrict__ vy, T* __restrict__ vz, const T* __restrict__ ax,
             const T* __restrict__ ay, const T* __restrict__ az, T hk, T hd, int wrap) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T u = vx[i], v = vy[i], w = vz[i];
  if (ax) {
    u += hk * ax[i];
    v += hk * ay[i];
    w += hk * az[i];
    vx[i] = u; vy[i] = v; vz[i] = w;
  }
  if (x) {
    T px = x[i] + hd * u, py = y[i] + hd * v, pz = z[i] + hd * w;
    if (wrap) {
      px = wrap_unit(px);
      py = wrap_unit(py);
      pz = wrap_unit(pz);
    }
    x[i] = px;
    y[i] = py;
    z[i] = pz;
  }
}

template <typename T>
hipError_t launch_kick_drift(int64_t n, T* x, T* y, T* z, T* vx, T* vy, T* vz, const T* ax,
                             const T* ay, const T* az, double hk, double hd, int wrap,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_kick_drift<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, n, x, y, z, vx, vy, vz, ax, ay, az, (T)hk, (T)hd, wrap);
  return hipGetLastError();
}

__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double sh[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// Kinetic energy 1/2 sum m v^2 (every particle) into per-block partials part[b].
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_kinetic(const T* __restrict__ m, const T* __restrict__ vx, const T* __restrict__ vy,
          const T* __restrict__ vz, int64_t n, double* __restrict__ part) {
  double k = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double u = vx[i], v = vy[i], w = vz[i];
    k += 0.5 * (double)m[i] * (u * u + v * v + w * w);
  }
  const double r = block_sum_d(k);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <typename T>
hipError_t launch_kinetic(const T* m, const T* vx, const T* vy, const T* vz, int64_t n, double* part,
                          double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t nb64 = (n + kBlock - 1) / kBlock;
  const int nb = (int)(nb64 > kMaxParts ? kMaxParts : nb64);
  hipLaunchKernelGGL((k_kinetic<T>), dim3(nb), dim3(kBlock), 0, s, m, vx, vy, vz, n, part);
  return launch_sum_parts(part, nb, 1, 1.0, out, s);
}

// Gas potential energy of one level: 1/2 sum over the active gas cells that their own
// grid owns (no finer grid, and no lower-index grid of the level, contains the cell
// centre) of rho_gas Phi dx^3, Phi from the composed field.  One thread per active
// cell of the level; per-block partials part[b].
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_gas_energy(const GridDesc* __restrict__ grids, const OwnerLevel* __restrict__ om, int32_t nlev,
             int32_t first, int32_t count, const int64_t* __restrict__ begin,
             const T* __restrict__ gas, const V4<T>* __restrict__ field,
             double* __restrict__ part) {
  double e = 0.0;
  const int64_t b = blockIdx.x;
  int gl = 0;                                        // grid of this block within the level
  {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (begin[mid] <= b) lo = mid; else hi = mid - 1;
    }
    gl = lo;
  }
  const GridDesc& g = grids[first + gl];
  const int64_t cells = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int64_t local = (b - begin[gl]) * (int64_t)kBlock + threadIdx.x;
  if (local < cells) {
    int lx, ly, lz;
    box_cell(local, g.n[0], g.n[1], lx, ly, lz);
    // owner of the cell centre: finest grid containing it, lowest index on that level
    const double px = (g.lo[0] + lx + 0.5) * g.dx, py = (g.lo[1] + ly + 0.5) * g.dx,
                 pz = (g.lo[2] + lz + 0.5) * g.dx;   // exact: dx is a power of two
    if (owner_lookup(om, nlev, px, py, pz) == first + gl) {
      const double rho = (double)gas[g.gas_offset + local];
      const int fx = g.lo[0] + lx - g.fld_lo[0], fy = g.lo[1] + ly - g.fld_lo[1],
                fz = g.lo[2] + lz - g.fld_lo[2];
      const double phi =
          (double)field[g.fld_offset + ((int64_t)fz * g.fld_n[1] + fy) * g.fld_n[0] + fx].w;
      e = 0.5 * rho * phi * g.dx * g.dx * g.dx;
    }
  }
  const double r = block_sum_d(e);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <typename T>
hipError_t launch_gas_energy(const GridDesc* grids, const OwnerLevel* om, int32_t nlev,
                             int32_t first, int32_t count, const int64_t* begin, int64_t nblocks,
                             const T* gas, const V4<T>* field, double* part, double* out,
                             hipStream_t s) {
  if (nblocks == 0 || !gas) return hipSuccess;
  hipLaunchKernelGGL((k_gas_energy<T>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, grids, om,
                     nlev, first, count, begin, gas, field, part);
  return launch_sum_parts(part, (int)nblocks, 1, 1.0, out, s);
}

#define APM_INST_D(T)                                                                         \
  template hipError_t launch_kick_drift<T>(int64_t, T*, T*, T*, T*, T*, T*, const T*, const T*, \
                                           const T*, double, double, int, hipStream_t);        \
  template hipError_t launch_kinetic<T>(const T*, const T*, const T*, const T*, int64_t,        \
                                        double*, double*, hipStream_t);                         \
  template hipError_t launch_gas_energy<T>(const GridDesc*, const OwnerLevel*, int32_t, int32_t,  \
                                           int32_t, const int64_t*, int64_t, const T*,         \
                                           const V4<T>*, double*, double*, hipStream_t);
APM_INST_D(float)
APM_INST_D(double)

}  // namespace apm
