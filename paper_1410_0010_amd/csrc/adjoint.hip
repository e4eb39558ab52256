// Reverse sweep of the solve, particle and field side (the transposes of Sec. 2
// deposit and interpolation and of the Sec. 2.2 level composition).  For a loss
// L = wbar W + sum_p abar_p . a_p + sum_p phibar_p Phi_p the cotangents flow:
//
//   particles --interp^T--> field boxes (FP64) --composition^T (finest first)-->
//   own-field cotangents --convolution^T (fft_adj.hip)--> GMF cotangents
//   --deposit^T--> level key boxes (FP64) --TSC gather--> particle gradients.
//
// All cotangent accumulation is FP64.  Particles are visited in the order of the
// forward solve's sorted list and tile work items (valid until the next solve), so
// neighbouring lanes touch neighbouring cells.
#include "apm_kernels.hpp"

namespace apm {

template <typename T> __device__ __forceinline__ T tsc_w_a(int d, T t) {
  const T h = (T)0.5;
  if (d < 0) { const T u = h - t; return h * u * u; }
  if (d > 0) { const T u = h + t; return h * u * u; }
  return (T)0.75 - t * t;
}
// d/dt of tsc_w_a
template <typename T> __device__ __forceinline__ T tsc_dw_a(int d, T t) {
  if (d < 0) return t - (T)0.5;
  if (d > 0) return (T)0.5 + t;
  return (T)-2 * t;
}

__device__ __forceinline__ int batch_of(const int64_t* blk0, int nlev, int64_t blk) {
  int b = 0;
  while (b + 1 < nlev && blk0[b + 1] <= blk) ++b;
  return b;
}

// ---- zero a list of FP64 ranges (blockIdx.y = range) ---------------------------------
__global__ void __launch_bounds__(kBlock) k_zero_ranges(ZeroList zl) {
  double* p = zl.p[blockIdx.y];
  const int64_t n = zl.n[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    p[i] = 0.0;
}

hipError_t launch_zero_ranges(const ZeroList& zl, hipStream_t s) {
  if (zl.count == 0) return hipSuccess;
  int64_t mx = 0;
  for (int i = 0; i < zl.count; ++i) mx = zl.n[i] > mx ? zl.n[i] : mx;
  int64_t nb = (mx + 4 * kBlock - 1) / (4 * kBlock);
  nb = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
  hipLaunchKernelGGL(k_zero_ranges, dim3((unsigned)nb, (unsigned)zl.count), dim3(kBlock), 0, s, zl);
  return hipGetLastError();
}

// ---- interpolation transpose ---------------------------------------------------------
// Work item = (level, tile, chunk) of the forward deposit.  Entries owned by a grid of
// the level add w * (abar, phibar + wbar m / 2) to an LDS tile (halo-extended, FP64)
// of their owner grid -- one tile for the chunk's first owner grid with 4 components,
// or up to 4 grids' tiles with the Phi component alone -- and straight to the field
// cotangent in HBM when their grid has no tile; each tile is then added to its
// grid's field box.  The entries' position gradients are k_adj_interp_grad's.
constexpr int kTH3 = kHaloCells;

template <typename T, int NC>
__global__ void __launch_bounds__(kBlock)
k_adj_interp(AdjIO<T> io, const DepLevel* __restrict__ tab, const GridDesc* __restrict__ grids) {
  // NC = 4 components, or 1 when only Phi flows back; then KG = 4 LDS tiles, one per
  // distinct owner grid of the chunk (overlapping grids of a level share tiles)
  constexpr int KG = NC == 1 ? 4 : 1;
  __shared__ double acc[KG * NC * kTH3];
  __shared__ int gsl[KG];
  __shared__ int gnext;
  const int lb = batch_of(io.item_blk0, io.nlev, blockIdx.x);
  const DepLevel L = load_global(tab + lb);   // its fields as values, not re-read after stores
  const int64_t item = blockIdx.x - io.item_blk0[lb];
  const int32_t total = L.items[L.ntiles];
  const int4 wk = L.work[item];                     // in the table's room; read with the count
  if (item >= total) return;                        // uniform for the block
  const int tile = wk.x;
  const int64_t begin = wk.y, end = wk.z;
  if (threadIdx.x < KG) gsl[threadIdx.x] = INT32_MAX;
  int ox, oy, oz;
  tile_origin(L, tile, ox, oy, oz);
  static_assert(kChunk == 8 * kBlock, "a chunk is eight records per thread");
  int2 ref[8];
  V4<T> rec[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {                      // the chunk's loads first
    const int64_t q = begin + threadIdx.x + (int64_t)k * kBlock;
    const int64_t qc = q < end ? q : begin;          // begin < end: a valid entry
    ref[k] = level_ref(L, qc);
    rec[k] = level_rec<T>(L, qc);
    if (q >= end) ref[k].y = -1;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) pin4(rec[k]);
  // the KG smallest distinct owner grids of the chunk, one round each, until a round
  // finds none (the usual chunk has one; on a level of one grid it is that grid, with
  // no round); then only those tiles are cleared
  // (a wavefront's minimum first, then one LDS atomic per wavefront: every thread
  // hitting the one word serialised 2048 atomics per round)
  int prev = -1, ng = 0;
  if (L.ngrids == 1) {                              // the level's one grid owns them all
    if (threadIdx.x == 0) gsl[0] = L.first;
    ng = 1;
  }
  for (int r = 0; r < KG && L.ngrids > 1; ++r) {
    if (threadIdx.x == 0) gnext = INT32_MAX;
    __syncthreads();
    int mn = INT32_MAX;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (ref[k].y > prev) mn = min(mn, ref[k].y);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, 64));
    if ((threadIdx.x & 63) == 0 && mn != INT32_MAX) atomicMin(&gnext, mn);
    __syncthreads();
    prev = gnext;                                    // the same value in every thread
    if (threadIdx.x == 0) gsl[r] = prev;
    __syncthreads();
    if (prev == INT32_MAX) break;
    ++ng;
  }
  for (int c = threadIdx.x; c < ng * NC * kTH3; c += kBlock) acc[c] = 0.0;
  __syncthreads();
  double* fbar = io.fbar[lb];
  const int c0 = 4 - NC;                            // first component carried
  // the owner grid's field box per entry; on a level of one grid, read once
  struct Box { int lo[3], n[3], wrap; int64_t off; };
  const auto box_of = [&](int gi) {
    const GridDesc& d = grids[gi];
    return Box{{d.fld_lo[0], d.fld_lo[1], d.fld_lo[2]}, {d.fld_n[0], d.fld_n[1], d.fld_n[2]},
               d.wrap, d.fld_offset};
  };
  const bool one = L.ngrids == 1;
  const Box box1 = one ? box_of(L.first) : Box{};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (ref[k].y < 0) continue;
    const int64_t i = ref[k].x;
    const V4<T> v = rec[k];
    const double cot[4] = {io.abx ? (double)io.abx[i] : 0.0, io.aby ? (double)io.aby[i] : 0.0,
                           io.abz ? (double)io.abz[i] : 0.0,
                           (io.phib ? (double)io.phib[i] : 0.0) + io.wbar * 0.5 * (double)v.w};
    const Box g = one ? box1 : box_of(ref[k].y);
    const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
    const T tx = v.x - fx - (T)0.5, ty = v.y - fy - (T)0.5, tz = v.z - fz - (T)0.5;
    const int cx = (int)fx - g.lo[0], cy = (int)fy - g.lo[1], cz = (int)fz - g.lo[2];
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    int slot = -1;                                  // LDS tile of this particle's grid
#pragma unroll
    for (int r = 0; r < KG; ++r)
      if (gsl[r] == ref[k].y) slot = r;
    const bool local = slot >= 0;
    // cell relative to the tile origin (always inside the tile; clamped defensively)
    const int ix = min(max((int)fx - L.key_lo[0] - ox, 0), kTile - 1),
              iy = min(max((int)fy - L.key_lo[1] - oy, 0), kTile - 1),
              iz = min(max((int)fz - L.key_lo[2] - oz, 0), kTile - 1);
    // per-axis cells (clamped into the box, weight 0 outside; wrapped on a periodic
    // root) and weights
    int ax_[3], ay_[3], az_[3];
    double wx[3], wy[3], wz[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int xx = cx + d - 1, yy = cy + d - 1, zz = cz + d - 1;
      if (g.wrap) {
        xx = wrap_cell(xx, nx);
        yy = wrap_cell(yy, ny);
        zz = wrap_cell(zz, nz);
      }
      const bool ox_ = (xx >= 0) & (xx < nx), oy_ = (yy >= 0) & (yy < ny), oz_ = (zz >= 0) & (zz < nz);
      ax_[d] = ox_ ? xx : 0; ay_[d] = oy_ ? yy : 0; az_[d] = oz_ ? zz : 0;
      wx[d] = ox_ ? (double)tsc_w_a(d - 1, tx) : 0.0;
      wy[d] = oy_ ? (double)tsc_w_a(d - 1, ty) : 0.0;
      wz[d] = oz_ ? (double)tsc_w_a(d - 1, tz) : 0.0;
    }
    // scatter of the cotangent (skipped components are zero for every particle)
#pragma unroll 1
    for (int dz = 0; dz < 3; ++dz) {
      for (int dy = 0; dy < 3; ++dy) {
        for (int dx = 0; dx < 3; ++dx) {
          const double w = wx[dx] * wy[dy] * wz[dz];
          if (w == 0.0) continue;
          if (local) {
            double* a = acc + NC * ((slot * 10 + iz + dz) * 100 + (iy + dy) * 10 + (ix + dx));
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) atomicAdd(a + cc, w * cot[c0 + cc]);
          } else {
            // 4 components per cell, or the Phi component alone, densely (NC == 1)
            double* a = fbar + (NC == 1 ? 1 : 4) *
                                   (g.off + ((int64_t)az_[dz] * ny + ay_[dy]) * nx + ax_[dx]);
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) atomicAdd(a + (NC == 1 ? 0 : c0 + cc), w * cot[c0 + cc]);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int r = 0; r < KG; ++r) {
    const int gs = gsl[r];
    if (gs == INT32_MAX) break;                     // no more owner grids in the chunk
    const GridDesc& g = grids[gs];
    for (int c = threadIdx.x; c < kTH3; c += kBlock) {
      const double* a = acc + NC * (r * kTH3 + c);
      bool any = false;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) any |= a[cc] != 0.0;
      if (!any) continue;
      const int lx = c % 10, ly = (c / 10) % 10, lz = c / 100;
      int xx = L.key_lo[0] + ox + lx - 1 - g.fld_lo[0];
      int yy = L.key_lo[1] + oy + ly - 1 - g.fld_lo[1];
      int zz = L.key_lo[2] + oz + lz - 1 - g.fld_lo[2];
      if (g.wrap) {                                 // periodic root: cells -1 and N
        xx = wrap_cell(xx, g.fld_n[0]);
        yy = wrap_cell(yy, g.fld_n[1]);
        zz = wrap_cell(zz, g.fld_n[2]);
      }
      if (xx < 0 || xx >= g.fld_n[0] || yy < 0 || yy >= g.fld_n[1] || zz < 0 || zz >= g.fld_n[2])
        continue;                                   // cannot hold weight (owned stencils lie inside)
      double* f = fbar + (NC == 1 ? 1 : 4) *
                             (g.fld_offset + ((int64_t)zz * g.fld_n[1] + yy) * g.fld_n[0] + xx);
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) atomicAdd(f + (NC == 1 ? 0 : c0 + cc), a[cc]);
    }
  }
}

// Position part of the interpolation transpose: one thread per entry of the sorted list
// (neighbouring lanes gather neighbouring cells), owned entries only:
//   pint[q] = (1/dx) sum_f grad w(f) . <F(f), cot_i>
// with F the forward composed field of the owner grid and cot_i the particle's
// cotangent (abar, phibar + wbar m / 2).  One writer per particle.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_interp_grad(AdjIO<T> io, const DepLevel* __restrict__ tab, const GridDesc* __restrict__ grids) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= io.npart) return;
  const int2 r = load_i2(tab[0].sref, q);
  if (r.y < 0) return;
  const GridDesc& g = grids[r.y];
  const V4<T> v = level_rec<T>(tab[g.level], q);
  const int64_t i = r.x;
  const double cot[4] = {io.abx ? (double)io.abx[i] : 0.0, io.aby ? (double)io.aby[i] : 0.0,
                         io.abz ? (double)io.abz[i] : 0.0,
                         (io.phib ? (double)io.phib[i] : 0.0) + io.wbar * 0.5 * (double)v.w};
  const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
  const T tx = v.x - fx - (T)0.5, ty = v.y - fy - (T)0.5, tz = v.z - fz - (T)0.5;
  const int cx = (int)fx - g.fld_lo[0], cy = (int)fy - g.fld_lo[1], cz = (int)fz - g.fld_lo[2];
  const int nx = g.fld_n[0], ny = g.fld_n[1], nz = g.fld_n[2];
  // per-axis cells (clamped into the box, weight 0 outside: the loads issue together;
  // wrapped on a periodic root)
  int ax_[3], ay_[3], az_[3];
  double wx[3], wy[3], wz[3], dwx[3], dwy[3], dwz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int xx = cx + d - 1, yy = cy + d - 1, zz = cz + d - 1;
    if (g.wrap) {
      xx = wrap_cell(xx, nx);
      yy = wrap_cell(yy, ny);
      zz = wrap_cell(zz, nz);
    }
    const bool ox_ = (xx >= 0) & (xx < nx), oy_ = (yy >= 0) & (yy < ny), oz_ = (zz >= 0) & (zz < nz);
    ax_[d] = ox_ ? xx : 0; ay_[d] = oy_ ? yy : 0; az_[d] = oz_ ? zz : 0;
    wx[d] = ox_ ? (double)tsc_w_a(d - 1, tx) : 0.0;
    wy[d] = oy_ ? (double)tsc_w_a(d - 1, ty) : 0.0;
    wz[d] = oz_ ? (double)tsc_w_a(d - 1, tz) : 0.0;
    dwx[d] = ox_ ? (double)tsc_dw_a(d - 1, tx) : 0.0;
    dwy[d] = oy_ ? (double)tsc_dw_a(d - 1, ty) : 0.0;
    dwz[d] = oz_ ? (double)tsc_dw_a(d - 1, tz) : 0.0;
  }
  const V4<T>* F = io.fld[g.level] + g.fld_offset;
  double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) {
    V4<T> f9[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
        f9[3 * dy + dx] = load_v4<T>(F, ((int64_t)az_[dz] * ny + ay_[dy]) * nx + ax_[dx]);
#pragma unroll
    for (int k9 = 0; k9 < 9; ++k9) pin4(f9[k9]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const V4<T>& f = f9[3 * dy + dx];
        const double s = cot[0] * f.x + cot[1] * f.y + cot[2] * f.z + cot[3] * f.w;
        gx += dwx[dx] * wy[dy] * wz[dz] * s;
        gy += wx[dx] * dwy[dy] * wz[dz] * s;
        gz += wx[dx] * wy[dy] * dwz[dz] * s;
      }
    }
  }
  const double inv = 1.0 / g.dx;
  // at the entry's sorted position (coalesced), not at i
  io.pint[q] = V4<T>{(T)(gx * inv), (T)(gy * inv), (T)(gz * inv), (T)0};
}

template <typename T>
hipError_t launch_adj_interp(const AdjIO<T>& io, const DepLevel* tab, const GridDesc* grids,
                             hipStream_t s) {
  const int64_t nb = io.item_blk0[io.nlev];
  if (nb <= 0) return hipSuccess;
  if (io.c0 == 3)
    hipLaunchKernelGGL((k_adj_interp<T, 1>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab, grids);
  else
    hipLaunchKernelGGL((k_adj_interp<T, 4>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab, grids);
  if (io.npart > 0)
    hipLaunchKernelGGL((k_adj_interp_grad<T>), dim3((unsigned)((io.npart + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, io, tab, grids);
  return hipGetLastError();
}

// ---- gas-energy seeds: owned active gas cells of one level ---------------------------
// fbar.w += wbar rho dx^3 / 2 and gas_bar += wbar Phi dx^3 / 2 (the two factors of the
// gas term of W).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_gas_seed(const GridDesc* __restrict__ grids, const OwnerLevel* __restrict__ om, int32_t nlev,
               int32_t first, int32_t count, const int64_t* __restrict__ begin,
               const T* __restrict__ gas, const V4<T>* __restrict__ field, double wbar,
               double* __restrict__ fbar, int fs, double* __restrict__ gas_bar) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const GridDesc& g = grids[first + lo];
  const int64_t cells = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int64_t local = (b - begin[lo]) * (int64_t)kBlock + threadIdx.x;
  if (local >= cells) return;
  int lx, ly, lz;
  box_cell(local, g.n[0], g.n[1], lx, ly, lz);
  const double px = (g.lo[0] + lx + 0.5) * g.dx, py = (g.lo[1] + ly + 0.5) * g.dx,
               pz = (g.lo[2] + lz + 0.5) * g.dx;
  if (owner_lookup(om, nlev, px, py, pz) != first + lo) return;
  const int64_t fc = g.fld_offset + ((int64_t)(g.lo[2] + lz - g.fld_lo[2]) * g.fld_n[1] +
                                     (g.lo[1] + ly - g.fld_lo[1])) * g.fld_n[0] +
                     (g.lo[0] + lx - g.fld_lo[0]);
  const double v = g.dx * g.dx * g.dx * 0.5 * wbar;
  fbar[fs * fc + fs - 1] += v * (double)gas[g.gas_offset + local];   // the Phi component
  gas_bar[g.gas_offset + local] += v * (double)field[fc].w;
}

template <typename T>
hipError_t launch_adj_gas_seed(const GridDesc* grids, const OwnerLevel* om, int32_t nlev,
                               int32_t first, int32_t count, const int64_t* begin, int64_t nblocks,
                               const T* gas, const V4<T>* field, double wbar, double* fbar,
                               int fs, double* gas_bar, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_gas_seed<T>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, grids, om,
                     nlev, first, count, begin, gas, field, wbar, fbar, fs, gas_bar);
  return hipGetLastError();
}

// ---- composition transpose: one child level into its parents -------------------------
// Thread = parent field cell q in the footprint of one child grid; it gathers the child
// cells 2q-1, 2q, 2q+1, 2q+2 per axis (weights 1/4, 3/4, 3/4, 1/4: the trilinear
// prolongation between cell centres, transposed) and adds the sum to the parent (a
// plain read-modify-write when the child level has one grid: one writer per cell).
template <int FS>
__global__ void __launch_bounds__(kBlock)
k_adj_restrict(const GridDesc* __restrict__ grids, int32_t first, int32_t count,
               const int64_t* __restrict__ begin, const double* __restrict__ child_bar,
               double* __restrict__ parent_bar) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const GridDesc& g = grids[first + lo];
  int flo[3], fn[3];
  int64_t cells = 1;
  for (int a = 0; a < 3; ++a) {
    const int l0 = (g.fld_lo[a] >> 1) - 1, h0 = ((g.fld_lo[a] + g.fld_n[a] - 1) >> 1) + 1;
    flo[a] = max(l0, g.parent_fld_lo[a]);
    fn[a] = min(h0, g.parent_fld_lo[a] + g.parent_fld_n[a] - 1) - flo[a] + 1;
    cells *= fn[a] > 0 ? fn[a] : 0;
  }
  const int64_t local = (b - begin[lo]) * (int64_t)kBlock + threadIdx.x;
  if (local >= cells) return;
  // a parent footprint has fewer than 2^31 cells: 32-bit index arithmetic
  const uint32_t loc = (uint32_t)local, rowu = loc / (uint32_t)fn[0];
  const uint32_t zq = rowu / (uint32_t)fn[1];
  const int q[3] = {flo[0] + (int)(loc - rowu * (uint32_t)fn[0]),
                    flo[1] + (int)(rowu - zq * (uint32_t)fn[1]), flo[2] + (int)zq};
  // the 4 child cells per axis, clamped into the box with weight 0 outside, so a
  // row's four loads issue together
  const double wts[4] = {0.25, 0.75, 0.75, 0.25};
  int ci[3][4];
  double cw[3][4];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = 2 * q[a] - 1 + k - g.fld_lo[a];
      const bool ok = c >= 0 && c < g.fld_n[a];
      ci[a][k] = ok ? c : 0;
      cw[a][k] = ok ? wts[k] : 0.0;
    }
  const int64_t pc = g.parent_fld_offset +
                     ((int64_t)(q[2] - g.parent_fld_lo[2]) * g.parent_fld_n[1] +
                      (q[1] - g.parent_fld_lo[1])) * g.parent_fld_n[0] +
                     (q[0] - g.parent_fld_lo[0]);
  if constexpr (FS == 4) {
    const V4<double>* cb = reinterpret_cast<const V4<double>*>(child_bar) + g.fld_offset;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
#pragma unroll
      for (int ky = 0; ky < 4; ++ky) {
        const int64_t row = ((int64_t)ci[2][kz] * g.fld_n[1] + ci[1][ky]) * g.fld_n[0];
        V4<double> v[4];
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) v[kx] = load_v4<double>(cb, row + ci[0][kx]);
        const double wzy = cw[2][kz] * cw[1][ky];
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) {
          const double w = wzy * cw[0][kx];
          s0 += w * v[kx].x; s1 += w * v[kx].y; s2 += w * v[kx].z; s3 += w * v[kx].w;
        }
      }
    }
    if (s0 == 0.0 && s1 == 0.0 && s2 == 0.0 && s3 == 0.0) return;
    double* p = parent_bar + 4 * pc;
    if (count == 1) {                                // the parent cell's only writer here
      p[0] += s0; p[1] += s1; p[2] += s2; p[3] += s3;
    } else {
      atomicAdd(p + 0, s0);
      atomicAdd(p + 1, s1);
      atomicAdd(p + 2, s2);
      atomicAdd(p + 3, s3);
    }
  } else {                                           // the Phi component alone, dense
    const gptr<double> cb = as_global<double>(child_bar + g.fld_offset);
    double s3 = 0.0;
#pragma unroll
    for (int kz = 0; kz < 4; ++kz) {
#pragma unroll
      for (int ky = 0; ky < 4; ++ky) {
        const int64_t row = ((int64_t)ci[2][kz] * g.fld_n[1] + ci[1][ky]) * g.fld_n[0];
        double v[4];
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) v[kx] = cb[row + ci[0][kx]];
        const double wzy = cw[2][kz] * cw[1][ky];
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) s3 += wzy * cw[0][kx] * v[kx];
      }
    }
    if (s3 == 0.0) return;
    if (count == 1) parent_bar[pc] += s3;            // the parent cell's only writer here
    else atomicAdd(parent_bar + pc, s3);
  }
}

hipError_t launch_adj_restrict(const GridDesc* grids, int32_t first, int32_t count,
                               const int64_t* begin, int64_t nblocks, const double* child_bar,
                               double* parent_bar, int fs, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (fs == 1)
    hipLaunchKernelGGL(k_adj_restrict<1>, dim3((unsigned)nblocks), dim3(kBlock), 0, s, grids, first,
                       count, begin, child_bar, parent_bar);
  else
    hipLaunchKernelGGL(k_adj_restrict<4>, dim3((unsigned)nblocks), dim3(kBlock), 0, s, grids, first,
                       count, begin, child_bar, parent_bar);
  return hipGetLastError();
}

// ---- deposit transpose, grid side ------------------------------------------------------
// kGmfPer GMF cells of a grid per thread: the level's FP64 key-box cotangent +=
// gmf_bar / dx^3 (on a level of one grid a store, and the binning box's one-cell shell
// set to zero here rather than cleared before); own gas (active cells) += gmf_bar; the
// parent's gas += gmf_bar on ghost cells.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_deposit_grid(AdjIO<T> io, const DepLevel* __restrict__ tab) {
  const int lb = batch_of(io.fin_blk0, io.nlev, blockIdx.x);
  const DepLevel L = load_global(tab + lb);
  const int64_t blk = blockIdx.x - io.fin_blk0[lb];
  const gptr<int64_t> bbeg = as_global<int64_t>(L.block_begin);
  int lo = 0, hi = L.ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bbeg[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  // the grid's descriptor as values read once, and global-space pointers: through
  // plain pointers every store below could alias the descriptors, which then had to be
  // read again after it (generic loads and stores, each waiting on the last)
  const GridDesc g = load_global(L.grids + lo);
  const int64_t cells = (int64_t)g.gmf_n[0] * g.gmf_n[1] * g.gmf_n[2];
  const int64_t first = (blk - bbeg[lo]) * (int64_t)(kBlock * kGmfPer) + threadIdx.x;
  const gptr<T> gin = as_global<T>(io.gmf_bar[lb]) + g.gmf_offset;
  double gbv[kGmfPer];
#pragma unroll
  for (int k = 0; k < kGmfPer; ++k) {               // the loads first
    const int64_t local = first + (int64_t)k * kBlock;
    gbv[k] = local < cells ? (double)gin[local] : 0.0;
  }
  const double inv_vol = 1.0 / (L.dx * L.dx * L.dx);   // exact: dx is a power of two
  const int64_t kx = L.key_n[0], kxy = (int64_t)L.key_n[0] * L.key_n[1];
  const bool single = L.ngrids == 1;
  const gmut<double> acc = as_global_mut<double>(L.accum);
  const gmut<double> gbar = io.gas_bar[lb] ? as_global_mut<double>(io.gas_bar[lb]) + g.gas_offset
                                           : nullptr;
  const gmut<double> pbar = io.pgas_bar[lb] && g.parent >= 0
                                ? as_global_mut<double>(io.pgas_bar[lb]) + g.parent_gas_offset
                                : nullptr;
#pragma unroll
  for (int k = 0; k < kGmfPer; ++k) {
    const double gb = gbv[k];
    const int64_t local = first + (int64_t)k * kBlock;
    if (local >= cells) continue;
    int lx, ly, lz;
    box_cell(local, g.gmf_n[0], g.gmf_n[1], lx, ly, lz);
    const int cx = g.gmf_lo[0] + lx, cy = g.gmf_lo[1] + ly, cz = g.gmf_lo[2] + lz;
    const gmut<double> kc = acc + (cz - L.key_lo[2]) * kxy + (int64_t)(cy - L.key_lo[1]) * kx +
                            (cx - L.key_lo[0]);
    if (single) {
      // One grid on the level: its GMF box is the binning box less a one-cell shell,
      // which is not cleared for this pass.  This thread is the cell's only writer, so
      // a store (zero included) gives the cleared grid's atomic sum, and the cells on
      // the GMF box's faces also zero the shell cells beside them.
      *kc = gb * inv_vol;
      const int x0 = lx == 0 ? -1 : 0, x1 = lx == g.gmf_n[0] - 1 ? 1 : 0;
      const int y0 = ly == 0 ? -1 : 0, y1 = ly == g.gmf_n[1] - 1 ? 1 : 0;
      const int z0 = lz == 0 ? -1 : 0, z1 = lz == g.gmf_n[2] - 1 ? 1 : 0;
      if (x0 | x1 | y0 | y1 | z0 | z1)
        for (int dz = z0; dz <= z1; ++dz)
          for (int dy = y0; dy <= y1; ++dy)
            for (int dx = x0; dx <= x1; ++dx)
              if (dx | dy | dz) kc[dz * kxy + (int64_t)dy * kx + dx] = 0.0;
      if (gb == 0.0) continue;
    } else {
      if (gb == 0.0) continue;
      global_add(kc, gb * inv_vol);
    }
    const bool active = cx >= g.lo[0] && cx < g.lo[0] + g.n[0] && cy >= g.lo[1] &&
                        cy < g.lo[1] + g.n[1] && cz >= g.lo[2] && cz < g.lo[2] + g.n[2];
    if (active) {
      // atomic: a finer level of the same launch adds its ghost cells to this array
      if (gbar)
        global_add(gbar + ((int64_t)(cz - g.lo[2]) * g.n[1] + (cy - g.lo[1])) * g.n[0] +
                       (cx - g.lo[0]),
                   gb);
    } else if (pbar) {
      const int px = (cx >> 1) - g.parent_lo[0], py = (cy >> 1) - g.parent_lo[1],
                pz = (cz >> 1) - g.parent_lo[2];
      global_add(pbar + ((int64_t)pz * g.parent_n[1] + py) * g.parent_n[0] + px, gb);
    }
  }
}

template <typename T>
hipError_t launch_adj_deposit_grid(const AdjIO<T>& io, const DepLevel* tab, hipStream_t s) {
  const int64_t nb = io.fin_blk0[io.nlev];
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_deposit_grid<T>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab);
  return hipGetLastError();
}

// ---- deposit transpose, particle side --------------------------------------------------
// Entry q of a level's tile runs: (sum_c w(c) A(c), m sum_c grad w(c) A(c)), A the
// level's key-box cotangent, stored in the level's slot at q (the levels are summed
// per particle at the end, so no atomics).  One block per deposit work item; a
// chunk of 64 entries or more reads the 10^3 key-box cells around its tile into LDS
// (zero outside the box, wrapped on a periodic root) and gathers from there.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_deposit_particles(AdjIO<T> io, const DepLevel* __restrict__ tab) {
  __shared__ double ta[kTH3];
  constexpr int kTH = kTile + 2;
  const int lb = batch_of(io.item_blk0, io.nlev, blockIdx.x);
  const DepLevel L = load_global(tab + lb);   // its fields as values, not re-read after stores
  const int64_t item = blockIdx.x - io.item_blk0[lb];
  const int32_t total = L.items[L.ntiles];
  const int4 wk = L.work[item];                     // in the table's room; read with the count
  if (item >= total) return;                        // uniform for the block
  const int tile = wk.x;
  const int64_t begin = wk.y, end = wk.z;
  int ox, oy, oz;
  tile_origin(L, tile, ox, oy, oz);
  const int nx = L.key_n[0], ny = L.key_n[1], nz = L.key_n[2];
  const gptr<double> acc_g = as_global<double>(L.accum);
  const bool staged = end - begin >= 64;            // uniform for the block
  if (staged) {
    for (int c = threadIdx.x; c < kTH3; c += kBlock) {
      int x = ox + c % kTH - 1, y = oy + (c / kTH) % kTH - 1, z = oz + c / (kTH * kTH) - 1;
      if (L.wrap) {                                  // periodic root: cells -1 and N
        x = wrap_cell(x + L.key_lo[0], L.wrap) - L.key_lo[0];
        y = wrap_cell(y + L.key_lo[1], L.wrap) - L.key_lo[1];
        z = wrap_cell(z + L.key_lo[2], L.wrap) - L.key_lo[2];
      }
      const bool in = x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
      const double a = acc_g[in ? ((int64_t)z * ny + y) * nx + x : 0];
      ta[c] = in ? a : 0.0;
    }
    __syncthreads();
  }
  for (int k = 0; k < 8; ++k) {
    const int64_t q = begin + threadIdx.x + (int64_t)k * kBlock;
    if (q >= end) break;
    const V4<T> v = level_rec<T>(L, q);
    const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
    const T tx = v.x - fx - (T)0.5, ty = v.y - fy - (T)0.5, tz = v.z - fz - (T)0.5;
    double wx[3], wy[3], wz[3], dwx[3], dwy[3], dwz[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      wx[d] = (double)tsc_w_a(d - 1, tx);
      wy[d] = (double)tsc_w_a(d - 1, ty);
      wz[d] = (double)tsc_w_a(d - 1, tz);
      dwx[d] = (double)tsc_dw_a(d - 1, tx);
      dwy[d] = (double)tsc_dw_a(d - 1, ty);
      dwz[d] = (double)tsc_dw_a(d - 1, tz);
    }
    double a27[27];
    if (staged) {
      const int ix = min(max((int)fx - L.key_lo[0] - ox, 0), kTile - 1),
                iy = min(max((int)fy - L.key_lo[1] - oy, 0), kTile - 1),
                iz = min(max((int)fz - L.key_lo[2] - oz, 0), kTile - 1);
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx)
            a27[(dz * 3 + dy) * 3 + dx] = ta[((iz + dz) * kTH + iy + dy) * kTH + ix + dx];
    } else {
      const int cx = (int)fx - L.key_lo[0], cy = (int)fy - L.key_lo[1], cz = (int)fz - L.key_lo[2];
      int ax_[3], ay_[3], az_[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int xx = cx + d - 1, yy = cy + d - 1, zz = cz + d - 1;
        if (L.wrap) {                                // periodic root: cells -1 and N
          xx = wrap_cell(xx + L.key_lo[0], L.wrap) - L.key_lo[0];
          yy = wrap_cell(yy + L.key_lo[1], L.wrap) - L.key_lo[1];
          zz = wrap_cell(zz + L.key_lo[2], L.wrap) - L.key_lo[2];
        }
        const bool ox_ = (xx >= 0) & (xx < nx), oy_ = (yy >= 0) & (yy < ny), oz_ = (zz >= 0) & (zz < nz);
        ax_[d] = ox_ ? xx : 0; ay_[d] = oy_ ? yy : 0; az_[d] = oz_ ? zz : 0;
        if (!ox_) { wx[d] = 0.0; dwx[d] = 0.0; }
        if (!oy_) { wy[d] = 0.0; dwy[d] = 0.0; }
        if (!oz_) { wz[d] = 0.0; dwz[d] = 0.0; }
      }
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx)
            a27[(dz * 3 + dy) * 3 + dx] = acc_g[((int64_t)az_[dz] * ny + ay_[dy]) * nx + ax_[dx]];
    }
    double sm = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const double a = a27[(dz * 3 + dy) * 3 + dx];
          sm += wx[dx] * wy[dy] * wz[dz] * a;
          gx += dwx[dx] * wy[dy] * wz[dz] * a;
          gy += wx[dx] * dwy[dy] * wz[dz] * a;
          gz += wx[dx] * wy[dy] * dwz[dz] * a;
        }
    const double m = (double)v.w * L.inv_dx;
    io.plev[lb][q] = V4<T>{(T)sm, (T)(m * gx), (T)(m * gy), (T)(m * gz)};   // sorted position
  }
}

template <typename T>
hipError_t launch_adj_deposit_particles(const AdjIO<T>& io, const DepLevel* tab, hipStream_t s) {
  const int64_t nb = io.item_blk0[io.nlev];
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_deposit_particles<T>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab);
  return hipGetLastError();
}

// ---- outputs -----------------------------------------------------------------------------
// One thread per entry q of the sorted list, for particle i = its original index:
// mbar, xbar = the sum over the levels whose tiles hold the particle of the deposit
// transpose, plus the interpolation transpose's position gradient and wbar Phi_p / 2
// (mass) for owned particles, formed in FP64 and rounded once into the record
// pout[i] (one 16 B write a particle; the four output arrays are then written
// coalesced by k_adj_unpack).  A level's tiles hold the particle when its tile
// floor(x / dx) / kTile lies in the level's tile box, as the tile runs do.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_finish(AdjIO<T> io, const DepLevel* __restrict__ tab, const T* __restrict__ pot) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= io.npart) return;
  const int2 r = load_i2(tab[0].sref, q);
  if (r.y < 0) return;                               // outside the domain: zero (unpack)
  const int64_t i = r.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const V4<T> w = load_v4<T>(tab[0].sorted, q);
  for (int l = 0; l < io.nlev; ++l) {
    const DepLevel& L = tab[l];
    const T sc = (T)L.inv_dx;
    const int cx = (int)floor(w.x * sc), cy = (int)floor(w.y * sc), cz = (int)floor(w.z * sc);
    static_assert(kTile == 8, "tile index by shift");
    const int tx = (cx >> 3) - L.tile_lo[0], ty = (cy >> 3) - L.tile_lo[1],
              tz = (cz >> 3) - L.tile_lo[2];
    if (tx < 0 || tx >= L.tiles_n[0] || ty < 0 || ty >= L.tiles_n[1] || tz < 0 ||
        tz >= L.tiles_n[2])
      continue;
    const V4<T> o = load_v4<T>(io.plev[l], q);
    s0 += (double)o.x; s1 += (double)o.y; s2 += (double)o.z; s3 += (double)o.w;
  }
  const V4<T> pi = load_v4<T>(io.pint, q);
  s1 += (double)pi.x; s2 += (double)pi.y; s3 += (double)pi.z;
  if (io.wbar != 0.0 && pot) s0 += io.wbar * 0.5 * (double)pot[i];
  if (io.rbar) s0 += as_global<double>(io.rbar)[0];   // periodic: the average density's
  io.pout[i] = V4<T>{(T)s0, (T)s1, (T)s2, (T)s3};
}

// The records -> the four gradient arrays (zero outside the domain: owner < 0).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_unpack(const V4<T>* __restrict__ pout, const int32_t* __restrict__ owner, int64_t n,
             T* __restrict__ xb, T* __restrict__ yb, T* __restrict__ zb, T* __restrict__ mb) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const V4<T> r = load_v4<T>(pout, i);
  const V4<T> v = owner[i] >= 0 ? r : V4<T>{0, 0, 0, 0};
  if (mb) mb[i] = v.x;
  if (xb) xb[i] = v.y;
  if (yb) yb[i] = v.z;
  if (zb) zb[i] = v.w;
}

// a[i] += scale * s[0] for i < n (a periodic root's gas cotangent: the average
// density's cotangent times dx_0^3 on every cell)
__global__ void __launch_bounds__(kBlock) k_add_scalar(double* __restrict__ a, int64_t n,
                                                       const double* __restrict__ s, double scale) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] += scale * as_global<double>(s)[0];
}

hipError_t launch_add_scalar(double* a, int64_t n, const double* s, double scale, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_scalar, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     a, n, s, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_finish(const AdjIO<T>& io, const DepLevel* tab, const int32_t* owner,
                             const T* pot, T* xb, T* yb, T* zb, T* mb, hipStream_t s) {
  if (io.npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((io.npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_adj_finish<T>), dim3(nb), dim3(kBlock), 0, s, io, tab, pot);
  hipLaunchKernelGGL((k_adj_unpack<T>), dim3(nb), dim3(kBlock), 0, s, io.pout, owner, io.npart, xb,
                     yb, zb, mb);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_to_t(const double* __restrict__ a, T* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = (T)a[i];
}

template <typename T>
hipError_t launch_to_t(const double* a, T* b, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_to_t<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     a, b, n);
  return hipGetLastError();
}

#define APM_INST_A(T)                                                                         \
  template hipError_t launch_adj_interp<T>(const AdjIO<T>&, const DepLevel*, const GridDesc*,   \
                                           hipStream_t);                                       \
  template hipError_t launch_adj_gas_seed<T>(const GridDesc*, const OwnerLevel*, int32_t,       \
                                             int32_t, int32_t, const int64_t*, int64_t,        \
                                             const T*, const V4<T>*, double, double*, int,     \
                                             double*, hipStream_t);                            \
  template hipError_t launch_adj_deposit_grid<T>(const AdjIO<T>&, const DepLevel*, hipStream_t); \
  template hipError_t launch_adj_deposit_particles<T>(const AdjIO<T>&, const DepLevel*,        \
                                                      hipStream_t);                            \
  template hipError_t launch_adj_finish<T>(const AdjIO<T>&, const DepLevel*, const int32_t*,    \
                                           const T*, T*, T*, T*, T*, hipStream_t);              \
  template hipError_t launch_to_t<T>(const double*, T*, int64_t, hipStream_t);
APM_INST_A(float)
APM_INST_A(double)

}  // namespace apm
