// Level composition (Sec. 2.2: the parent's field interpolated onto the refined grid
// and added to its own mesh force), FP64 totals and fill kernels.
#include <algorithm>

#include "apm_kernels.hpp"

namespace apm {

__device__ __forceinline__ int find_grid_f(const int64_t* __restrict__ begin, int ngrids, int64_t b) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// field = own + P(parent): P trilinear between cell centres; a child cell c has
// its centre a quarter parent cell from parent centre floor(c/2), towards parent
// floor(c/2) - 1 (c even) or + 1 (c odd): weights 3/4 and 1/4 per axis.  With
// pprev, the parent field is first taken linearly in time on the parent's cells,
// (1 - alpha) pprev + alpha parent, then interpolated.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_compose(const GridDesc* __restrict__ grids, const int64_t* __restrict__ begin, int32_t ngrids,
          const V4<T>* own, const V4<T>* __restrict__ parent, V4<T>* field,
          const V4<T>* __restrict__ pprev, T alpha) {
  const int gi = find_grid_f(begin, ngrids, blockIdx.x);
  const GridDesc& g = grids[gi];
  const int64_t cells = (int64_t)g.fld_n[0] * g.fld_n[1] * g.fld_n[2];
  const int64_t local = (blockIdx.x - begin[gi]) * (int64_t)kBlock + threadIdx.x;
  if (local >= cells) return;
  V4<T> v = own[g.fld_offset + local];
  if (parent) {
    int lx, ly, lz;
    box_cell(local, g.fld_n[0], g.fld_n[1], lx, ly, lz);
    const int c[3] = {g.fld_lo[0] + lx, g.fld_lo[1] + ly, g.fld_lo[2] + lz};
    int pi[3][2];
    for (int a = 0; a < 3; ++a) {
      const int p = c[a] >> 1;
      pi[a][0] = p - g.parent_fld_lo[a];
      pi[a][1] = ((c[a] & 1) ? p + 1 : p - 1) - g.parent_fld_lo[a];
    }
    const V4<T>* P = parent + g.parent_fld_offset;
    const V4<T>* Q = pprev ? pprev + g.parent_fld_offset : nullptr;
    const T wts[2] = {(T)0.75, (T)0.25};
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d) {
          const T w = wts[a] * wts[b] * wts[d];
          const int64_t k = ((int64_t)pi[2][a] * g.parent_fld_n[1] + pi[1][b]) * g.parent_fld_n[0] + pi[0][d];
          V4<T> f = P[k];
          if (Q) {
            const V4<T> q = Q[k];
            const T be = (T)1 - alpha;
            f.x = be * q.x + alpha * f.x; f.y = be * q.y + alpha * f.y;
            f.z = be * q.z + alpha * f.z; f.w = be * q.w + alpha * f.w;
          }
          s0 += w * f.x; s1 += w * f.y; s2 += w * f.z; s3 += w * f.w;
        }
    v.x += s0; v.y += s1; v.z += s2; v.w += s3;
  }
  field[g.fld_offset + local] = v;
}

template <typename T>
hipError_t launch_compose(const GridDesc* grids, const int64_t* begin, int32_t ngrids,
                          const V4<T>* own, const V4<T>* parent, V4<T>* field, int64_t nblocks,
                          hipStream_t s, const V4<T>* pprev, double alpha) {
  hipLaunchKernelGGL((k_compose<T>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, grids, begin,
                     ngrids, own, parent, field, pprev, (T)alpha);
  return hipGetLastError();
}

// ---- FP64 reductions ----------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
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

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum_scaled(const T* __restrict__ a, int64_t n,
                                                       double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    acc += (double)a[i];
  const double r = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// out[q] += scale * sum_{b < nparts} part[q * kMaxParts + b] for q < nq (fixed order)
__global__ void __launch_bounds__(kBlock) k_sum_parts(const double* __restrict__ part, int nparts,
                                                      int nq, double scale,
                                                      double* __restrict__ out) {
  for (int q = 0; q < nq; ++q) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) acc += part[q * kMaxParts + b];
    const double r = block_sum(acc);
    if (threadIdx.x == 0) out[q] += scale * r;
  }
}

hipError_t launch_sum_parts(const double* part, int nparts, int nq, double scale, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, s, part, nparts, nq, scale, out);
  return hipGetLastError();
}

// Average density of a periodic system (the sine wave test, Sec. 3: the solve needs
// zero net mass): in-domain particle masses (NaN or outside [0, 1) excluded, as in
// the deposit) plus the root gas mass, over the unit box.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mean_parts(const T* __restrict__ x, const T* __restrict__ y,
                                                       const T* __restrict__ z, const T* __restrict__ m,
                                                       int64_t npart, const T* __restrict__ gas,
                                                       int64_t ngas, double vol,
                                                       double* __restrict__ part) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double pm = 0.0, gm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npart; i += stride) {
    const T px = x[i], py = y[i], pz = z[i];
    if (px >= (T)0 && px < (T)1 && py >= (T)0 && py < (T)1 && pz >= (T)0 && pz < (T)1)
      pm += (double)m[i];
  }
  if (gas)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ngas; i += stride)
      gm += (double)gas[i];
  const double r = block_sum(pm + gm * vol);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_mean_finish(const double* __restrict__ part, int nparts,
                                                        double* __restrict__ out) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBlock) acc += part[b];
  const double r = block_sum(acc);
  if (threadIdx.x == 0) out[0] = r;
}

static int nparts_for(int64_t n);

// Particles the deposit leaves out (a coordinate outside [0, 1) or NaN): per-block
// partial count and mass at part[b] and part[kMaxParts + b].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dropped_parts(const T* __restrict__ x, const T* __restrict__ y,
                                                          const T* __restrict__ z,
                                                          const T* __restrict__ m, int64_t npart,
                                                          double* __restrict__ part) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double cnt = 0.0, mass = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npart; i += stride) {
    const T px = x[i], py = y[i], pz = z[i];
    if (!(px >= (T)0 && px < (T)1 && py >= (T)0 && py < (T)1 && pz >= (T)0 && pz < (T)1)) {
      cnt += 1.0;
      mass += (double)m[i];
    }
  }
  const double rc = block_sum(cnt), rm = block_sum(mass);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rc;
    part[kMaxParts + blockIdx.x] = rm;
  }
}

template <typename T>
hipError_t launch_mean_density(const T* x, const T* y, const T* z, const T* m, int64_t npart,
                               const T* gas, int64_t ngas, double vol, double* part, double* out,
                               hipStream_t s) {
  const int nb = nparts_for(std::max<int64_t>(npart, gas ? ngas : 0));
  hipLaunchKernelGGL((k_mean_parts<T>), dim3(nb), dim3(kBlock), 0, s, x, y, z, m, npart, gas, ngas,
                     vol, part);
  hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(kBlock), 0, s, (const double*)part, nb, out);
  return hipGetLastError();
}

static int nparts_for(int64_t n) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  return (int)(nb > kMaxParts ? kMaxParts : (nb < 1 ? 1 : nb));
}

template <typename T>
hipError_t launch_dropped(const T* x, const T* y, const T* z, const T* m, int64_t npart,
                          double* part, double* out, hipStream_t s) {
  const int nb = nparts_for(npart);
  hipLaunchKernelGGL((k_dropped_parts<T>), dim3(nb), dim3(kBlock), 0, s, x, y, z, m, npart, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, s, (const double*)part, nb, 2, 1.0, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sum_scaled(const T* a, int64_t n, double scale, double* part, double* out,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = nparts_for(n);
  hipLaunchKernelGGL((k_sum_scaled<T>), dim3(nb), dim3(kBlock), 0, s, a, n, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, s, (const double*)part, nb, 1, scale, out);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_particle_totals(const T* __restrict__ m, const int32_t* __restrict__ owner, int64_t npart,
                  const T* __restrict__ ax, const T* __restrict__ ay, const T* __restrict__ az,
                  const T* __restrict__ pot, double* __restrict__ part) {
  double w = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npart;
       i += (int64_t)gridDim.x * kBlock) {
    if (owner[i] < 0) continue;
    const double mi = (double)m[i];
    if (pot) w += 0.5 * mi * (double)pot[i];
    fx += mi * (double)ax[i];
    fy += mi * (double)ay[i];
    fz += mi * (double)az[i];
  }
  const double rw = block_sum(w), rx = block_sum(fx), ry = block_sum(fy), rz = block_sum(fz);
  if (threadIdx.x == 0) {
    part[0 * kMaxParts + blockIdx.x] = rw;
    part[1 * kMaxParts + blockIdx.x] = rx;
    part[2 * kMaxParts + blockIdx.x] = ry;
    part[3 * kMaxParts + blockIdx.x] = rz;
  }
}

template <typename T>
hipError_t launch_particle_totals(const T* m, const int32_t* owner, int64_t npart, const T* ax,
                                  const T* ay, const T* az, const T* pot, double* part, double* out,
                                  hipStream_t s) {
  if (npart == 0) return hipSuccess;
  const int nb = nparts_for(npart);
  hipLaunchKernelGGL((k_particle_totals<T>), dim3(nb), dim3(kBlock), 0, s, m, owner, npart, ax, ay,
                     az, pot, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, s, (const double*)part, nb, 4, 1.0, out);
  return hipGetLastError();
}

// Partial sums of a solve's totals, one launch: blockIdx.y < nlev sums level y's GMF
// (nb_mass blocks; blocks past a level's size add 0), blockIdx.y = nlev the particle
// terms W_p, sum m a (nb_part blocks).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_totals_parts(TotalsIO<T> io, int nb_mass, int nb_part) {
  const int l = blockIdx.y;
  if (l < io.nlev) {
    if ((int)blockIdx.x >= nb_mass) return;
    const T* __restrict__ a = io.gmf[l];
    const int64_t n = io.gmf_n[l];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)nb_mass * kBlock)
      acc += (double)a[i];
    const double r = block_sum(acc);
    if (threadIdx.x == 0) io.part[(int64_t)l * kMaxParts + blockIdx.x] = r;
    return;
  }
  if ((int)blockIdx.x >= nb_part) return;
  double w = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < io.npart;
       i += (int64_t)nb_part * kBlock) {
    if (io.owner[i] < 0) continue;
    const double mi = (double)io.m[i];
    if (io.pot) w += 0.5 * mi * (double)io.pot[i];
    fx += mi * (double)io.ax[i];
    fy += mi * (double)io.ay[i];
    fz += mi * (double)io.az[i];
  }
  const double rw = block_sum(w), rx = block_sum(fx), ry = block_sum(fy), rz = block_sum(fz);
  if (threadIdx.x == 0) {
    double* part = io.part + (int64_t)io.nlev * kMaxParts;
    part[0 * kMaxParts + blockIdx.x] = rw;
    part[1 * kMaxParts + blockIdx.x] = rx;
    part[2 * kMaxParts + blockIdx.x] = ry;
    part[3 * kMaxParts + blockIdx.x] = rz;
  }
}

// out[q] for q = blockIdx.x < nlev + 5, each block one quantity (fixed summation order)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_totals_finish(TotalsIO<T> io, int nb_mass, int nb_part) {
  const int nl = io.nlev;
  const int q = blockIdx.x;
  const double wg = io.gas_w ? *io.gas_w : 0.0;
  if (q == nl + 4) {
    if (threadIdx.x == 0) io.out[q] = wg;
    return;
  }
  const int nb = q < nl ? nb_mass : nb_part;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc += io.part[(int64_t)q * kMaxParts + b];
  const double r = block_sum(acc);
  if (threadIdx.x == 0) io.out[q] = q < nl ? io.vol[q] * r : (q == nl ? r + wg : r);
}

template <typename T>
hipError_t launch_totals(const TotalsIO<T>& io, hipStream_t s) {
  int64_t nmax = 1;
  for (int l = 0; l < io.nlev; ++l) nmax = io.gmf_n[l] > nmax ? io.gmf_n[l] : nmax;
  const int nb_mass = nparts_for(nmax);
  const int nb_part = io.npart > 0 ? nparts_for(io.npart) : 0;
  const int nbx = nb_mass > nb_part ? nb_mass : nb_part;
  hipLaunchKernelGGL((k_totals_parts<T>), dim3(nbx, io.nlev + 1), dim3(kBlock), 0, s, io, nb_mass,
                     nb_part);
  hipLaunchKernelGGL((k_totals_finish<T>), dim3(io.nlev + 5), dim3(kBlock), 0, s, io, nb_mass, nb_part);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_i32, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

#define APM_INST_F(T)                                                                          \
  template hipError_t launch_compose<T>(const GridDesc*, const int64_t*, int32_t, const V4<T>*,  \
                                        const V4<T>*, V4<T>*, int64_t, hipStream_t, const V4<T>*, \
                                        double);             \
  template hipError_t launch_mean_density<T>(const T*, const T*, const T*, const T*, int64_t,     \
                                             const T*, int64_t, double, double*, double*,         \
                                             hipStream_t);                                        \
  template hipError_t launch_sum_scaled<T>(const T*, int64_t, double, double*, double*,          \
                                          hipStream_t);                                         \
  template hipError_t launch_totals<T>(const TotalsIO<T>&, hipStream_t);                        \
  template hipError_t launch_dropped<T>(const T*, const T*, const T*, const T*, int64_t, double*,  \
                                        double*, hipStream_t);                                   \
  template hipError_t launch_particle_totals<T>(const T*, const int32_t*, int64_t, const T*,     \
                                                const T*, const T*, const T*, double*, double*,  \
                                                hipStream_t);
APM_INST_F(float)
APM_INST_F(double)

}  // namespace apm
