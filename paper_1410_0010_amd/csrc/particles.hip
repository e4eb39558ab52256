// Particle-side kernels: binning, TSC deposit (Sec. 2), owner grid, TSC
// interpolation.
//
// Deposit design: particles are counted into 8^3-cell tiles of their cell
// i0 = floor(x / dx_l) over the level's binning box (union of the level's GMF boxes
// grown by one cell), with block-aggregated atomics (one global atomic per distinct
// tile in a block of 2048 particles), and scattered tile by tile as 16 B records (s_x, s_y, s_z, m),
// s = x/dx - binning-box origin, plus the original index.  A work item is one tile's chunk of at most kChunk
// particles; its block accumulates the 27 TSC contributions of every particle in
// a 10^3 halo-extended tile in LDS with FP64 atomics, then adds the non-zero cells
// to an FP64 key-box grid with global atomics.  A finalize pass divides by dx^3,
// adds the gas and writes the GMF in the working precision.  Heavy tiles (a
// Plummer core holds ~1e5 particles per tile on the root) are split across many
// blocks, so the load is balanced; FP64 accumulation keeps the result at the
// working precision's rounding of the exact sum.
#include "apm_kernels.hpp"

namespace apm {

template <typename T>
__device__ __forceinline__ bool in_domain(T x, T y, T z) {
  return x >= (T)0 && x < (T)1 && y >= (T)0 && y < (T)1 && z >= (T)0 && z < (T)1;
}

// TSC weight on cell i0 + d for offset t = x/dx - i0 - 1/2 in [-1/2, 1/2).
template <typename T> __device__ __forceinline__ T tsc_w(int d, T t) {
  const T h = (T)0.5;
  if (d < 0) { const T u = h - t; return h * u * u; }
  if (d > 0) { const T u = h + t; return h * u * u; }
  return (T)0.75 - t * t;
}

// Block-aggregated tile counting: each block takes kBinPer particles per thread,
// inserts their tile keys into an LDS hash table (linear probing, CAS), takes local
// ranks from LDS atomics, then reserves one range per distinct tile with a single
// global atomic on the block's replica of that tile's counter.  A tile holding many
// particles (the Plummer core) thus sees one global atomic per block instead of one
// per particle or wavefront.
constexpr int kBinPer = 8;
constexpr int kBinBlockParticles = kBlock * kBinPer;     // 2048
constexpr int kHash = 2 * kBinBlockParticles;            // load factor <= 1/2

template <typename T>
__global__ void __launch_bounds__(kBlock) k_bin_count(BinParams<T> p) {
  __shared__ int32_t hkey[kHash];
  __shared__ int32_t hcnt[kHash];
  for (int h = threadIdx.x; h < kHash; h += kBlock) { hkey[h] = -1; hcnt[h] = 0; }
  __syncthreads();
  const int32_t r = (int32_t)(blockIdx.x & (p.rep - 1));
  const int64_t base = (int64_t)blockIdx.x * kBinBlockParticles + threadIdx.x;
  int32_t key[kBinPer], slot[kBinPer], lrank[kBinPer];
#pragma unroll
  for (int q = 0; q < kBinPer; ++q) {
    const int64_t i = base + (int64_t)q * kBlock;
    key[q] = -1;
    slot[q] = -1;
    lrank[q] = 0;
    if (i < p.npart) {
      const T x = p.x[i], y = p.y[i], z = p.z[i];
      if (in_domain(x, y, z)) {
        const T s = (T)p.inv_dx;
        const int ix = (int)floor(x * s) - p.key_lo[0];
        const int iy = (int)floor(y * s) - p.key_lo[1];
        const int iz = (int)floor(z * s) - p.key_lo[2];
        if (ix >= 0 && ix < p.key_n[0] && iy >= 0 && iy < p.key_n[1] && iz >= 0 && iz < p.key_n[2])
          key[q] = ((iz / kTile) * p.tiles_n[1] + iy / kTile) * p.tiles_n[0] + ix / kTile;
      }
    }
    if (key[q] >= 0) {
      int h = (int)(((uint32_t)key[q] * 2654435761u) >> 19) & (kHash - 1);
      while (true) {                                   // table never full: terminates
        const int32_t old = atomicCAS(&hkey[h], -1, key[q]);
        if (old == -1 || old == key[q]) break;
        h = (h + 1) & (kHash - 1);
      }
      slot[q] = h;
      lrank[q] = atomicAdd(&hcnt[h], 1);
    }
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kHash; h += kBlock) {
    const int32_t n = hcnt[h];
    if (n > 0) hcnt[h] = atomicAdd(&p.count[hkey[h] * p.rep + r], n);   // becomes the base
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kBinPer; ++q) {
    const int64_t i = base + (int64_t)q * kBlock;
    if (i < p.npart) {
      p.key[i] = key[q] < 0 ? -1 : key[q] * p.rep + r;        // counter slot
      p.rank[i] = key[q] < 0 ? 0 : hcnt[slot[q]] + lrank[q];
    }
  }
}

template <typename T>
__global__ void k_bin_scatter(BinParams<T> p, const int32_t* __restrict__ start,
                              V4<T>* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.npart) return;
  const int32_t key = p.key[i];
  if (key < 0) return;
  const int32_t tile = key / p.rep;
  const int tx = tile % p.tiles_n[0], ty = (tile / p.tiles_n[0]) % p.tiles_n[1],
            tz = tile / (p.tiles_n[0] * p.tiles_n[1]);
  (void)tx; (void)ty; (void)tz;
  const T s = (T)p.inv_dx;
  V4<T> r;
  // exact: x/dx is exact (dx a power of two) and the origin an integer below it
  r.x = p.x[i] * s - (T)p.key_lo[0];
  r.y = p.y[i] * s - (T)p.key_lo[1];
  r.z = p.z[i] * s - (T)p.key_lo[2];
  r.w = p.m[i];
  const int32_t slot = start[key] + p.rank[i];
  sorted[slot] = r;
  p.sidx[slot] = (int32_t)i;
}

template <typename T>
hipError_t launch_bin_count(const BinParams<T>& p, hipStream_t s) {
  if (p.npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((p.npart + kBinBlockParticles - 1) / kBinBlockParticles);
  hipLaunchKernelGGL((k_bin_count<T>), dim3(nb), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bin_scatter(const BinParams<T>& p, const int32_t* start, V4<T>* sorted,
                              hipStream_t s) {
  if (p.npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((p.npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_bin_scatter<T>), dim3(nb), dim3(kBlock), 0, s, p, start, sorted);
  return hipGetLastError();
}

__global__ void k_chunk_count(const int32_t* __restrict__ start, int32_t ntiles, int32_t rep,
                              int32_t* __restrict__ items) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  items[t] = t < ntiles
      ? (start[(t + 1) * rep] - start[t * rep] + kChunk - 1) / kChunk : 0;
}

hipError_t launch_chunk_count(const int32_t* start, int32_t ntiles, int32_t rep, int32_t* items,
                              hipStream_t s) {
  const unsigned nb = (unsigned)((ntiles + 1 + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_chunk_count, dim3(nb), dim3(kBlock), 0, s, start, ntiles, rep, items);
  return hipGetLastError();
}

// ---- exclusive scan of int32 (three passes, 1024 elements per block) ------------
constexpr int kScanPer = 4;
constexpr int kScanBlock = kBlock * kScanPer;

__device__ static int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int32_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int32_t incl = sh[t];
  *total = sh[kBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_blocks(int32_t* __restrict__ data, int64_t n, int32_t* __restrict__ sums) {
  __shared__ int32_t sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int32_t v[kScanPer], s = 0;
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = (base + q < n) ? data[base + q] : 0;
    s += v[q];
  }
  int32_t total;
  int32_t ex = block_exclusive_scan(s, sh, &total);
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < n) data[base + q] = ex;
    ex += v[q];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(int32_t* __restrict__ sums, int64_t nsums) {
  __shared__ int32_t sh[kBlock];
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < nsums; c0 += kScanBlock) {
    const int64_t base = c0 + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer], s = 0;
    for (int q = 0; q < kScanPer; ++q) {
      v[q] = (base + q < nsums) ? sums[base + q] : 0;
      s += v[q];
    }
    int32_t total;
    int32_t ex = block_exclusive_scan(s, sh, &total) + carry;
    for (int q = 0; q < kScanPer; ++q) {
      if (base + q < nsums) sums[base + q] = ex;
      ex += v[q];
    }
    carry += total;
  }
}

__global__ void k_scan_add(int32_t* __restrict__ data, int64_t n, const int32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  const int32_t add = sums[blockIdx.x];
  for (int q = 0; q < kScanPer; ++q)
    if (base + q < n) data[base + q] += add;
}

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock) + 1; }

hipError_t launch_exclusive_scan(int32_t* data, int64_t n, int32_t* tmp, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kBlock), 0, s, data, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, data, n,
                     (const int32_t*)tmp);
  return hipGetLastError();
}

// ---- deposit: one thread per GMF cell ------------------------------------------
__device__ __forceinline__ int find_grid(const int64_t* __restrict__ begin, int ngrids, int64_t b) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Work item = chunk of one tile: LDS accumulation over the tile and its one-cell
// halo, then global FP64 atomics into the key-box grid.
constexpr int kTH = kTile + 2;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_deposit_tiles(TileDepositParams<T> p) {
  __shared__ double acc[kTH * kTH * kTH];
  const int32_t total = p.item_start[p.ntiles];
  const int64_t item = blockIdx.x;
  if (item >= total) return;                        // uniform for the block
  int lo = 0, hi = p.ntiles - 1;                    // last tile with item_start <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (p.item_start[mid] <= item) lo = mid; else hi = mid - 1;
  }
  const int tile = lo;
  const int64_t begin = p.start[(int64_t)tile * p.rep] + (item - p.item_start[tile]) * (int64_t)kChunk;
  const int64_t end = min((int64_t)p.start[(int64_t)(tile + 1) * p.rep], begin + kChunk);
  for (int c = threadIdx.x; c < kTH * kTH * kTH; c += kBlock) acc[c] = 0.0;
  __syncthreads();
  const int ox = (tile % p.tiles_n[0]) * kTile, oy = ((tile / p.tiles_n[0]) % p.tiles_n[1]) * kTile,
            oz = (tile / (p.tiles_n[0] * p.tiles_n[1])) * kTile;
  for (int64_t q = begin + threadIdx.x; q < end; q += kBlock) {
    const V4<T> v = p.sorted[q];
    const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
    const int ix = min(max((int)fx - ox, 0), kTile - 1), iy = min(max((int)fy - oy, 0), kTile - 1),
              iz = min(max((int)fz - oz, 0), kTile - 1);
    const double tx = (double)(v.x - fx) - 0.5, ty = (double)(v.y - fy) - 0.5,
                 tz = (double)(v.z - fz) - 0.5;
    const double wx[3] = {0.5 * (0.5 - tx) * (0.5 - tx), 0.75 - tx * tx, 0.5 * (0.5 + tx) * (0.5 + tx)};
    const double wy[3] = {0.5 * (0.5 - ty) * (0.5 - ty), 0.75 - ty * ty, 0.5 * (0.5 + ty) * (0.5 + ty)};
    const double wz[3] = {0.5 * (0.5 - tz) * (0.5 - tz), 0.75 - tz * tz, 0.5 * (0.5 + tz) * (0.5 + tz)};
    const double m = (double)v.w;
    // halo-extended tile index of cell i0 + d is (i0 + d + 1)
    double* base = acc + (iz * kTH + iy) * kTH + ix;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      const double mz = m * wz[dz];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const double mzy = mz * wy[dy];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) atomicAdd(base + (dz * kTH + dy) * kTH + dx, mzy * wx[dx]);
      }
    }
  }
  __syncthreads();
  const int tx0 = ox - 1, ty0 = oy - 1, tz0 = oz - 1;
  for (int c = threadIdx.x; c < kTH * kTH * kTH; c += kBlock) {
    const double v = acc[c];
    if (v == 0.0) continue;
    const int gx = tx0 + c % kTH, gy = ty0 + (c / kTH) % kTH, gz = tz0 + c / (kTH * kTH);
    if (gx < 0 || gx >= p.key_n[0] || gy < 0 || gy >= p.key_n[1] || gz < 0 || gz >= p.key_n[2])
      continue;
    atomicAdd(p.accum + ((int64_t)gz * p.key_n[1] + gy) * p.key_n[0] + gx, v);
  }
}

template <typename T>
hipError_t launch_deposit_tiles(const TileDepositParams<T>& p, int64_t max_items, hipStream_t s) {
  if (max_items <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_deposit_tiles<T>), dim3((unsigned)max_items), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

// Finalize: GMF cell c of every grid of the level = accumulated mass / dx^3 + gas
// (own gas on active cells, the parent's copied onto ghost cells).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_deposit(DepositParams<T> p) {
  const int gi = find_grid(p.block_begin, p.ngrids, blockIdx.x);
  const GridDesc& g = p.grids[gi];
  const int64_t cells = (int64_t)g.gmf_n[0] * g.gmf_n[1] * g.gmf_n[2];
  const int64_t local = (blockIdx.x - p.block_begin[gi]) * (int64_t)kBlock + threadIdx.x;
  if (local >= cells) return;
  const int lx = (int)(local % g.gmf_n[0]);
  const int ly = (int)((local / g.gmf_n[0]) % g.gmf_n[1]);
  const int lz = (int)(local / ((int64_t)g.gmf_n[0] * g.gmf_n[1]));
  const int cx = g.gmf_lo[0] + lx, cy = g.gmf_lo[1] + ly, cz = g.gmf_lo[2] + lz;
  const double mass = p.accum[((int64_t)(cz - p.key_lo[2]) * p.key_n[1] + (cy - p.key_lo[1])) *
                                  p.key_n[0] + (cx - p.key_lo[0])];
  T rho = (T)(mass / (p.dx * p.dx * p.dx));
  const bool active = cx >= g.lo[0] && cx < g.lo[0] + g.n[0] && cy >= g.lo[1] &&
                      cy < g.lo[1] + g.n[1] && cz >= g.lo[2] && cz < g.lo[2] + g.n[2];
  if (active) {
    if (p.gas)
      rho += p.gas[g.gas_offset + ((int64_t)(cz - g.lo[2]) * g.n[1] + (cy - g.lo[1])) * g.n[0] +
                   (cx - g.lo[0])];
  } else if (p.parent_gas && g.parent >= 0) {
    const int px = (cx >> 1) - g.parent_lo[0], py = (cy >> 1) - g.parent_lo[1],
              pz = (cz >> 1) - g.parent_lo[2];
    rho += p.parent_gas[g.parent_gas_offset + ((int64_t)pz * g.parent_n[1] + py) * g.parent_n[0] + px];
  }
  p.gmf[g.gmf_offset + local] = rho;
}

template <typename T>
hipError_t launch_deposit(const DepositParams<T>& p, int64_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_deposit<T>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

// ---- owner grid -------------------------------------------------------------------
template <typename T>
__global__ void k_owner(const GridDesc* __restrict__ grids, int32_t ngrids, double root_n,
                        const T* __restrict__ x, const T* __restrict__ y, const T* __restrict__ z,
                        int64_t npart, int32_t* __restrict__ owner) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npart) return;
  const T px = x[i], py = y[i], pz = z[i];
  int32_t best = -1;
  if (in_domain(px, py, pz)) {
    int bestlev = -1;
    for (int gi = ngrids - 1; gi >= 0; --gi) {
      const GridDesc& g = grids[gi];
      if (g.level < bestlev) break;
      const double inv = root_n * (double)(1 << g.level);
      const int cx = (int)floor((double)px * inv), cy = (int)floor((double)py * inv),
                cz = (int)floor((double)pz * inv);
      if (cx >= g.lo[0] && cx < g.lo[0] + g.n[0] && cy >= g.lo[1] && cy < g.lo[1] + g.n[1] &&
          cz >= g.lo[2] && cz < g.lo[2] + g.n[2]) {
        best = gi;
        bestlev = g.level;
      }
    }
  }
  owner[i] = best;
}

template <typename T>
hipError_t launch_owner(const GridDesc* grids, int32_t ngrids, double root_n, const T* x,
                        const T* y, const T* z, int64_t npart, int32_t* owner, hipStream_t s) {
  if (npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_owner<T>), dim3(nb), dim3(kBlock), 0, s, grids, ngrids, root_n, x, y, z,
                     npart, owner);
  return hipGetLastError();
}

// ---- TSC interpolation of the composed field ---------------------------------------
template <typename T>
__global__ void k_interp(const GridDesc* __restrict__ grids, int32_t level,
                         const V4<T>* __restrict__ field, const T* __restrict__ x,
                         const T* __restrict__ y, const T* __restrict__ z,
                         const int32_t* __restrict__ owner, int64_t npart, T* __restrict__ ax,
                         T* __restrict__ ay, T* __restrict__ az, T* __restrict__ pot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npart) return;
  const int32_t o = owner[i];
  if (o < 0) return;
  const GridDesc& g = grids[o];
  if (g.level != level) return;
  const T s = (T)(1.0 / g.dx);
  const T sx = x[i] * s, sy = y[i] * s, sz = z[i] * s;
  const int ix = (int)floor(sx), iy = (int)floor(sy), iz = (int)floor(sz);
  const T tx = sx - (T)ix - (T)0.5, ty = sy - (T)iy - (T)0.5, tz = sz - (T)iz - (T)0.5;
  T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  const V4<T>* F = field + g.fld_offset;
  for (int dz = -1; dz <= 1; ++dz) {
    const int cz = iz + dz - g.fld_lo[2];
    if (cz < 0 || cz >= g.fld_n[2]) continue;
    const T wz = tsc_w(dz, tz);
    for (int dy = -1; dy <= 1; ++dy) {
      const int cy = iy + dy - g.fld_lo[1];
      if (cy < 0 || cy >= g.fld_n[1]) continue;
      const T wzy = wz * tsc_w(dy, ty);
      for (int dx = -1; dx <= 1; ++dx) {
        const int cx = ix + dx - g.fld_lo[0];
        if (cx < 0 || cx >= g.fld_n[0]) continue;
        const T w = wzy * tsc_w(dx, tx);
        const V4<T> f = F[((int64_t)cz * g.fld_n[1] + cy) * g.fld_n[0] + cx];
        acc0 += w * f.x; acc1 += w * f.y; acc2 += w * f.z; acc3 += w * f.w;
      }
    }
  }
  ax[i] = acc0; ay[i] = acc1; az[i] = acc2;
  if (pot) pot[i] = acc3;
}

template <typename T>
hipError_t launch_interp(const GridDesc* grids, int32_t level, const V4<T>* field, const T* x,
                         const T* y, const T* z, const int32_t* owner, int64_t npart, T* ax, T* ay,
                         T* az, T* pot, hipStream_t s) {
  if (npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_interp<T>), dim3(nb), dim3(kBlock), 0, s, grids, level, field, x, y, z,
                     owner, npart, ax, ay, az, pot);
  return hipGetLastError();
}

template <typename T>
__global__ void k_interp_sorted(const GridDesc* __restrict__ grids, int32_t level,
                                const V4<T>* __restrict__ field, const V4<T>* __restrict__ sorted,
                                const int32_t* __restrict__ sidx, const int32_t* __restrict__ total,
                                int32_t klx, int32_t kly, int32_t klz,
                                const int32_t* __restrict__ owner, T* __restrict__ ax,
                                T* __restrict__ ay, T* __restrict__ az, T* __restrict__ pot) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *total) return;
  const int32_t i = sidx[q];
  const int32_t o = owner[i];
  if (o < 0) return;
  const GridDesc& g = grids[o];
  if (g.level != level) return;
  const V4<T> v = sorted[q];
  const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
  const T tx = v.x - fx - (T)0.5, ty = v.y - fy - (T)0.5, tz = v.z - fz - (T)0.5;
  const int ix = (int)fx + klx - g.fld_lo[0], iy = (int)fy + kly - g.fld_lo[1],
            iz = (int)fz + klz - g.fld_lo[2];
  const V4<T>* F = field + g.fld_offset;
  T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int cz = iz + dz;
    if (cz < 0 || cz >= g.fld_n[2]) continue;
    const T wz = tsc_w(dz, tz);
    for (int dy = -1; dy <= 1; ++dy) {
      const int cy = iy + dy;
      if (cy < 0 || cy >= g.fld_n[1]) continue;
      const T wzy = wz * tsc_w(dy, ty);
      const V4<T>* row = F + ((int64_t)cz * g.fld_n[1] + cy) * g.fld_n[0];
      for (int dx = -1; dx <= 1; ++dx) {
        const int cx = ix + dx;
        if (cx < 0 || cx >= g.fld_n[0]) continue;
        const T w = wzy * tsc_w(dx, tx);
        const V4<T> f = row[cx];
        acc0 += w * f.x; acc1 += w * f.y; acc2 += w * f.z; acc3 += w * f.w;
      }
    }
  }
  ax[i] = acc0; ay[i] = acc1; az[i] = acc2;
  if (pot) pot[i] = acc3;
}

template <typename T>
hipError_t launch_interp_sorted(const GridDesc* grids, int32_t level, const V4<T>* field,
                                const V4<T>* sorted, const int32_t* sidx, const int32_t* total,
                                int64_t max_n, const int32_t key_lo[3], const int32_t* owner,
                                T* ax, T* ay, T* az, T* pot, hipStream_t s) {
  if (max_n == 0) return hipSuccess;
  const unsigned nb = (unsigned)((max_n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_interp_sorted<T>), dim3(nb), dim3(kBlock), 0, s, grids, level, field,
                     sorted, sidx, total, key_lo[0], key_lo[1], key_lo[2], owner, ax, ay, az, pot);
  return hipGetLastError();
}

template <typename T>
__global__ void k_interp_all(const GridDesc* __restrict__ grids, FieldTable<T> fields,
                             const T* __restrict__ x, const T* __restrict__ y,
                             const T* __restrict__ z, const int32_t* __restrict__ owner,
                             int64_t npart, T* __restrict__ ax, T* __restrict__ ay,
                             T* __restrict__ az, T* __restrict__ pot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npart) return;
  const int32_t o = owner[i];
  T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  if (o >= 0) {
    const GridDesc& g = grids[o];
    const T s = (T)(1.0 / g.dx);
    const T sx = x[i] * s, sy = y[i] * s, sz = z[i] * s;
    const int ix = (int)floor(sx), iy = (int)floor(sy), iz = (int)floor(sz);
    const T tx = sx - (T)ix - (T)0.5, ty = sy - (T)iy - (T)0.5, tz = sz - (T)iz - (T)0.5;
    const V4<T>* F = fields.f[g.level] + g.fld_offset;
    for (int dz = -1; dz <= 1; ++dz) {
      const int cz = iz + dz - g.fld_lo[2];
      if (cz < 0 || cz >= g.fld_n[2]) continue;
      const T wz = tsc_w(dz, tz);
      for (int dy = -1; dy <= 1; ++dy) {
        const int cy = iy + dy - g.fld_lo[1];
        if (cy < 0 || cy >= g.fld_n[1]) continue;
        const T wzy = wz * tsc_w(dy, ty);
        for (int dx = -1; dx <= 1; ++dx) {
          const int cx = ix + dx - g.fld_lo[0];
          if (cx < 0 || cx >= g.fld_n[0]) continue;
          const T w = wzy * tsc_w(dx, tx);
          const V4<T> f = F[((int64_t)cz * g.fld_n[1] + cy) * g.fld_n[0] + cx];
          acc0 += w * f.x; acc1 += w * f.y; acc2 += w * f.z; acc3 += w * f.w;
        }
      }
    }
  }
  ax[i] = acc0; ay[i] = acc1; az[i] = acc2;
  if (pot) pot[i] = acc3;
}

template <typename T>
hipError_t launch_interp_all(const GridDesc* grids, const FieldTable<T>& fields, const T* x,
                             const T* y, const T* z, const int32_t* owner, int64_t npart, T* ax,
                             T* ay, T* az, T* pot, hipStream_t s) {
  if (npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_interp_all<T>), dim3(nb), dim3(kBlock), 0, s, grids, fields, x, y, z,
                     owner, npart, ax, ay, az, pot);
  return hipGetLastError();
}

#define APM_INST(T)                                                                          \
  template hipError_t launch_bin_count<T>(const BinParams<T>&, hipStream_t);                   \
  template hipError_t launch_bin_scatter<T>(const BinParams<T>&, const int32_t*, V4<T>*,        \
                                            hipStream_t);                                       \
  template hipError_t launch_deposit<T>(const DepositParams<T>&, int64_t, hipStream_t);        \
  template hipError_t launch_deposit_tiles<T>(const TileDepositParams<T>&, int64_t, hipStream_t); \
  template hipError_t launch_interp_sorted<T>(const GridDesc*, int32_t, const V4<T>*,            \
                                              const V4<T>*, const int32_t*, const int32_t*,      \
                                              int64_t, const int32_t*, const int32_t*, T*, T*,   \
                                              T*, T*, hipStream_t);                              \
  template hipError_t launch_interp_all<T>(const GridDesc*, const FieldTable<T>&, const T*,      \
                                           const T*, const T*, const int32_t*, int64_t, T*, T*,  \
                                           T*, T*, hipStream_t);                                 \
  template hipError_t launch_owner<T>(const GridDesc*, int32_t, double, const T*, const T*,     \
                                      const T*, int64_t, int32_t*, hipStream_t);                \
  template hipError_t launch_interp<T>(const GridDesc*, int32_t, const V4<T>*, const T*,       \
                                       const T*, const T*, const int32_t*, int64_t, T*, T*, T*, \
                                       T*, hipStream_t);
APM_INST(float)
APM_INST(double)

}  // namespace apm
