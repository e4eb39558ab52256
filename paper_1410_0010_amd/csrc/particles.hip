// Particle-side kernels: tile runs, TSC deposit (Sec. 2), owner grid, TSC
// interpolation.
//
// Deposit design: the particles, sorted once by the Morton code of their tile
// (sort.hip), form one contiguous run per 8^3-cell tile on every level; the tiles of a
// level are those covering its binning box (the union of its GMF boxes grown by one
// cell).  A work item is one tile's chunk of at most kChunk particles; its block
// counting-sorts the chunk by cell, sums the 27 TSC contributions of each same-cell
// run in registers, adds them to a 10^3 halo-extended tile in LDS with FP64 atomics,
// then adds the non-zero cells to an FP64 key-box grid with global atomics.  A finalize
// pass divides by dx^3, adds the gas and writes the GMF in the working precision.
// Heavy tiles (a Plummer core holds ~1e5 particles per tile on the root) are split
// across many blocks, so the load is balanced; FP64 accumulation keeps the result at
// the working precision's rounding of the exact sum.
#include <algorithm>
#include <type_traits>

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

// Batch level of block blockIdx.x in a launch whose levels own consecutive block
// ranges [blk0[b], blk0[b + 1]).
__device__ __forceinline__ int batch_level(const int64_t* blk0, int nlev, int64_t blk) {
  int b = 0;
  while (b + 1 < nlev && blk0[b + 1] <= blk) ++b;
  return b;
}

// TSC gather of the 27 cells around cell (ix, iy, iz) (box-relative) of a field box of
// dims n, with offsets t from the cell centre.  Branch-free: a cell outside the box
// gets weight 0 and a clamped (valid) address, so all 27 loads are issued together.
// wrap != 0 (a periodic root, whose field box is the whole domain): the stencil wraps
// around the box edges instead.
template <typename T>
__device__ __forceinline__ V4<T> tsc_gather(const V4<T>* __restrict__ F, int nx, int ny, int nz,
                                            int ix, int iy, int iz, T tx, T ty, T tz, int wrap) {
  const int n[3] = {nx, ny, nz};
  int cx[3], cy[3], cz[3];
  T wx[3], wy[3], wz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int x = ix + d - 1, y = iy + d - 1, z = iz + d - 1;
    if (wrap) {
      x = wrap_cell(x, nx);
      y = wrap_cell(y, ny);
      z = wrap_cell(z, nz);
    }
    const bool okx = (x >= 0) & (x < nx), oky = (y >= 0) & (y < ny), okz = (z >= 0) & (z < nz);
    cx[d] = okx ? x : 0;
    cy[d] = oky ? y : 0;
    cz[d] = okz ? z : 0;
    wx[d] = okx ? tsc_w(d - 1, tx) : (T)0;
    wy[d] = oky ? tsc_w(d - 1, ty) : (T)0;
    wz[d] = okz ? tsc_w(d - 1, tz) : (T)0;
  }
  V4<T> acc;
  acc.x = 0; acc.y = 0; acc.z = 0; acc.w = 0;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) {                   // a plane of 9 loads at a time
    V4<T> f[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const V4<T>* row = F + ((int64_t)cz[dz] * n[1] + cy[dy]) * n[0];
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) f[3 * dy + dx] = row[cx[dx]];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) pin4(f[k]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const T wzy = wz[dz] * wy[dy];
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const V4<T>& v = f[3 * dy + dx];
        const T w = wzy * wx[dx];
        acc.x += w * v.x; acc.y += w * v.y; acc.z += w * v.z; acc.w += w * v.w;
      }
    }
  }
  return acc;
}

// ---- clear: tile runs and FP64 mass grids of every level of the batch ------------------
__global__ void __launch_bounds__(kBlock) k_dep_clear(const DepLevel* __restrict__ tab) {
  const DepLevel& L = tab[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < L.ntiles; i += stride) {
    L.tbegin[i] = 0;
    L.tend[i] = 0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < L.key_cells; i += stride)
    L.accum[i] = 0.0;
}

hipError_t launch_dep_clear(const DepLevel* tab, int nlev, int64_t max_elems, hipStream_t s) {
  if (nlev == 0) return hipSuccess;
  const int64_t want = (max_elems + 4 * kBlock - 1) / (4 * kBlock);
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
  hipLaunchKernelGGL(k_dep_clear, dim3(nb, (unsigned)nlev), dim3(kBlock), 0, s, tab);
  return hipGetLastError();
}

// ---- per-level scans ------------------------------------------------------------------
// Each tile's work items, ceil(tile count / kChunk), get item starts and work-table
// entries.  Three short launches, all levels in each: per-block sums over kScanTiles
// tiles (one tile per thread), a scan of those sums per level, then every block scans
// its own tiles from its offset.
constexpr int kScanTiles = 256;                      // tiles per block (one per thread)
constexpr int kScanThreads = 1024;                   // threads of the per-level scan

// Exclusive prefix sums of two values over a block of NT threads (wavefront shuffles,
// then the wave totals); *tot gets the block sums.  sh holds 2 NT / 64 ints.
template <int NT>
__device__ static int2 block_scan2(int2 v, int32_t* sh, int2* tot) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int2 inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t ox = __shfl_up(inc.x, off, 64), oy = __shfl_up(inc.y, off, 64);
    if (lane >= off) { inc.x += ox; inc.y += oy; }
  }
  if (lane == 63) { sh[wave] = inc.x; sh[NW + wave] = inc.y; }
  __syncthreads();
  int2 base = make_int2(0, 0), sum = make_int2(0, 0);
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int32_t a = sh[w], b = sh[NW + w];
    if (w < wave) { base.x += a; base.y += b; }
    sum.x += a; sum.y += b;
  }
  __syncthreads();                                   // sh reused by the next call
  *tot = sum;
  return make_int2(base.x + inc.x - v.x, base.y + inc.y - v.y);
}

// tile t's particle count and work items
__device__ __forceinline__ int2 tile_count(const DepLevel& L, int32_t t) {
  const int32_t n = t < L.ntiles ? L.tend[t] - L.tbegin[t] : 0;
  return make_int2(n, (n + kChunk - 1) / kChunk);
}

__global__ void __launch_bounds__(kScanTiles) k_scan_tiles(const DepLevel* __restrict__ tab) {
  __shared__ int32_t sh[2 * kScanTiles / 64];
  const DepLevel& L = tab[blockIdx.y];
  if ((int64_t)blockIdx.x * kScanTiles >= L.ntiles) return;   // uniform for the block
  const int2 c = tile_count(L, (int32_t)(blockIdx.x * kScanTiles + threadIdx.x));
  int2 tot;
  block_scan2<kScanTiles>(c, sh, &tot);
  if (threadIdx.x == 0) L.bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(const DepLevel* __restrict__ tab) {
  __shared__ int32_t sh[2 * kScanThreads / 64];
  const DepLevel& L = tab[blockIdx.x];
  const int32_t nb = (L.ntiles + kScanTiles - 1) / kScanTiles;
  int2 carry = make_int2(0, 0);
  for (int32_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int32_t b = b0 + (int32_t)threadIdx.x;
    const int2 v = b < nb ? L.bsum[b] : make_int2(0, 0);
    int2 tot;
    const int2 ex = block_scan2<kScanThreads>(v, sh, &tot);
    if (b < nb) L.bsum[b] = make_int2(carry.x + ex.x, carry.y + ex.y);
    carry.x += tot.x;
    carry.y += tot.y;
  }
  if (threadIdx.x == 0) L.items[L.ntiles] = carry.y;
}

__global__ void __launch_bounds__(kScanTiles) k_scan_emit(const DepLevel* __restrict__ tab) {
  __shared__ int32_t sh[2 * kScanTiles / 64];
  const DepLevel& L = tab[blockIdx.y];
  if ((int64_t)blockIdx.x * kScanTiles >= L.ntiles) return;   // uniform for the block
  const int32_t t = (int32_t)(blockIdx.x * kScanTiles + threadIdx.x);
  const int2 c = tile_count(L, t);
  int2 tot;
  const int2 ex = block_scan2<kScanTiles>(c, sh, &tot);
  if (t >= L.ntiles) return;
  const int32_t istart = L.bsum[blockIdx.x].y + ex.y;
  const int32_t start = L.tbegin[t];
  L.items[t] = istart;
  for (int32_t q = 0; q < c.y; ++q) {                // the tile's work items
    const int32_t b = start + q * kChunk;
    L.work[istart + q] = make_int4(t, b, min(start + c.x, b + kChunk), 0);
  }
}

hipError_t launch_bin_scan(const DepLevel* tab, int nlev, int32_t max_tiles, hipStream_t s) {
  if (nlev == 0) return hipSuccess;
  const unsigned nb = (unsigned)((max_tiles + kScanTiles - 1) / kScanTiles);
  hipLaunchKernelGGL(k_scan_tiles, dim3(nb, (unsigned)nlev), dim3(kScanTiles), 0, s, tab);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nlev), dim3(kScanThreads), 0, s, tab);
  hipLaunchKernelGGL(k_scan_emit, dim3(nb, (unsigned)nlev), dim3(kScanTiles), 0, s, tab);
  return hipGetLastError();
}

// ---- deposit: work item = chunk of one tile ------------------------------------------
// The chunk is counting-sorted by cell in LDS; runs of one cell accumulate in registers
// and go to an LDS tile (the tile and its one-cell halo) once per run; then global
// atomics add the tile into the level's key-box grid.  Blocks past a level's item
// count exit at once.
//
// Two accumulations.  FP64: weights, run sums, the LDS tile and the key-box grid in
// FP64.  Compensated FP32 (COMP): weights in FP32, each sum a pair (s, e) whose exact
// value s + e tracks the exact sum: TwoSum recovers the rounding error of every FP32
// addition (in registers directly; in LDS and in the key-box grid from the value a
// returning atomic add found there), and the errors are summed in the low word.
__device__ __forceinline__ int find_grid(const int64_t* __restrict__ begin, int ngrids, int64_t b) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (as_global<int64_t>(begin)[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kTH = kTile + 2;
constexpr int kTH3 = kHaloCells;

// s + e == a + b exactly (Knuth's TwoSum; round to nearest)
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
  const float s = a + b;
  const float bp = s - a;
  e = (a - (s - bp)) + (b - bp);
  return s;
}
// A pair (hi, lo) takes (v + c) with a returning atomic add of v to hi: it gives the
// value v was added to, so the rounding error of that addition is known exactly and
// joins c in the low word (an ordinary atomic add).  The returning adds of a batch of
// cells are all issued before any error add, so their round trips overlap.

template <typename T, bool COMP>
__global__ void __launch_bounds__(kBlock) k_deposit_tiles(DepIO<T> io, const DepLevel* __restrict__ tab) {
  using A = typename std::conditional<COMP, float, double>::type;   // accumulation type
  constexpr int kCells = kTile * kTile * kTile;
  __shared__ double acc_raw[kTH3];                   // FP64 sums, or (hi, lo) FP32 pairs
  __shared__ int32_t cstart[kCells];                 // per-cell counts, then starts
  __shared__ uint16_t sidx[kChunk];                  // the chunk's entries, sorted by cell
  double* acc = acc_raw;
  float2* accp = reinterpret_cast<float2*>(acc_raw);
  const int lb = batch_level(io.item_blk0, io.nlev, blockIdx.x);
  const DepLevel L = load_global(tab + lb);   // its fields as values, not re-read after stores
  const int64_t item = blockIdx.x - io.item_blk0[lb];
  const int32_t total = L.items[L.ntiles];
  const int4 wk = L.work[item];                     // in the table's room; read with the count
  if (item >= total) return;                        // uniform for the block
  const int tile = wk.x;
  const int64_t begin = wk.y, end = wk.z;
  const int n = (int)(end - begin);                  // 1 .. kChunk
  for (int c = threadIdx.x; c < kTH3; c += kBlock) acc[c] = 0.0;   // both words zero
  for (int c = threadIdx.x; c < kCells; c += kBlock) cstart[c] = 0;
  int ox, oy, oz;
  tile_origin(L, tile, ox, oy, oz);
  const int bx = L.key_lo[0] + ox, by = L.key_lo[1] + oy, bz = L.key_lo[2] + oz;
  static_assert(kChunk == 8 * kBlock, "a chunk is eight records per thread");
  V4<T> rec[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {                      // the whole chunk's loads first
    const int64_t q = begin + threadIdx.x + (int64_t)k * kBlock;
    rec[k] = level_rec<T>(L, q < end ? q : begin);   // begin < end: a valid record
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) pin4(rec[k]);
  __syncthreads();                                   // tile and counters cleared
  // TSC weights of offset t = x - cell - 1/2 (exact in T: x and its cell share an
  // exponent range), in the accumulation type
  auto weights = [](T t, A w[3]) {
    const A u = (A)t;
    w[0] = (A)0.5 * ((A)0.5 - u) * ((A)0.5 - u);
    w[1] = (A)0.75 - u * u;
    w[2] = (A)0.5 * ((A)0.5 + u) * ((A)0.5 + u);
  };
  if (n <= kBlock) {
    // a small chunk (at most one record per thread): each record's 27 weighted masses
    // go straight to the LDS tile; sorting would cost more than it saves
    if ((int)threadIdx.x < n) {
      const V4<T> v = rec[0];
      const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
      const int ix = min(max((int)fx - bx, 0), kTile - 1), iy = min(max((int)fy - by, 0), kTile - 1),
                iz = min(max((int)fz - bz, 0), kTile - 1);
      A wx[3], wy[3], wz[3];
      weights(v.x - fx - (T)0.5, wx);
      weights(v.y - fy - (T)0.5, wy);
      weights(v.z - fz - (T)0.5, wz);
      const A m = (A)v.w;
      const int base = (iz * kTH + iy) * kTH + ix;
      A w27[27];
#pragma unroll
      for (int c = 0; c < 27; ++c) w27[c] = m * wz[c / 9] * wy[(c / 3) % 3] * wx[c % 3];
      if constexpr (COMP) {
        float old[27];                                 // returning adds first, as in flush
#pragma unroll
        for (int c = 0; c < 27; ++c)
          old[c] = atomicAdd(&accp[base + ((c / 9) * kTH + (c / 3) % 3) * kTH + c % 3].x, w27[c]);
#pragma unroll
        for (int c = 0; c < 27; ++c) {
          float e;
          two_sum(old[c], w27[c], e);
          atomicAdd(&accp[base + ((c / 9) * kTH + (c / 3) % 3) * kTH + c % 3].y, e);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 27; ++c)
          atomicAdd(acc + base + ((c / 9) * kTH + (c / 3) % 3) * kTH + c % 3, (double)w27[c]);
      }
    }
  } else {
    // counting sort of the chunk by cell of the tile (cells clamped into the tile
    // defensively; every particle of a tile's run has its cell inside the tile)
    int cell[8], rk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cell[k] = -1;
      rk[k] = 0;
      if ((int)threadIdx.x + k * kBlock < n) {
        const int ix = min(max((int)floor(rec[k].x) - bx, 0), kTile - 1),
                  iy = min(max((int)floor(rec[k].y) - by, 0), kTile - 1),
                  iz = min(max((int)floor(rec[k].z) - bz, 0), kTile - 1);
        cell[k] = (iz * kTile + iy) * kTile + ix;
        rk[k] = atomicAdd(&cstart[cell[k]], 1);
      }
    }
    __syncthreads();
    {                                                  // exclusive scan of the 512 counts
      static_assert(kCells == 2 * kBlock, "two cells per thread");
      const int a = cstart[2 * threadIdx.x], b = cstart[2 * threadIdx.x + 1];
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      int incl = a + b;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
      }
      __shared__ int wsum[kBlock / 64];
      if (lane == 63) wsum[wave] = incl;
      __syncthreads();
      int wbase = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) wbase += w < wave ? wsum[w] : 0;
      const int ex = wbase + incl - (a + b);
      cstart[2 * threadIdx.x] = ex;
      cstart[2 * threadIdx.x + 1] = ex + a;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (cell[k] >= 0) sidx[cstart[cell[k]] + rk[k]] = (uint16_t)(threadIdx.x + k * kBlock);
    __syncthreads();
    // eight consecutive sorted records per thread: a run of one cell accumulates its
    // 27 weighted masses in registers and adds them to the tile once
    A a27[27], e27[27];                                // sums (and, COMP, their errors)
#pragma unroll
    for (int c = 0; c < 27; ++c) { a27[c] = 0; e27[c] = 0; }
    int cur = -1;
    auto flush = [&](int cl) {
      const int ix = cl % kTile, iy = (cl / kTile) % kTile, iz = cl / (kTile * kTile);
      const int base = (iz * kTH + iy) * kTH + ix;     // halo tile index of cell i0 + d - 1
      if constexpr (COMP) {
        // the 27 returning adds first (independent cells), then the error adds
        float old[27];
#pragma unroll
        for (int c = 0; c < 27; ++c)
          old[c] = atomicAdd(&accp[base + ((c / 9) * kTH + (c / 3) % 3) * kTH + c % 3].x, a27[c]);
#pragma unroll
        for (int c = 0; c < 27; ++c) {
          float e;
          two_sum(old[c], a27[c], e);
          atomicAdd(&accp[base + ((c / 9) * kTH + (c / 3) % 3) * kTH + c % 3].y, e + e27[c]);
          a27[c] = 0;
          e27[c] = 0;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 27; ++c) {
          atomicAdd(acc + base + ((c / 9) * kTH + (c / 3) % 3) * kTH + c % 3, (double)a27[c]);
          a27[c] = 0;
        }
      }
    };
    // this thread's eight sorted entries, re-read from the chunk's records (cache
    // hits: the block read them above) so the LDS holds 2 B per entry, not a record
    V4<T> sv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = min((int)threadIdx.x * 8 + j, n - 1);
      sv[j] = level_rec<T>(L, begin + sidx[e]);
    }
    for (int j = 0; j < 8; ++j) {
      const int e = (int)threadIdx.x * 8 + j;
      if (e >= n) break;
      const V4<T> v = sv[j];
      const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
      const int ix = min(max((int)fx - bx, 0), kTile - 1), iy = min(max((int)fy - by, 0), kTile - 1),
                iz = min(max((int)fz - bz, 0), kTile - 1);
      const int cl = (iz * kTile + iy) * kTile + ix;
      if (cl != cur) {
        if (cur >= 0) flush(cur);
        cur = cl;
      }
      A wx[3], wy[3], wz[3];
      weights(v.x - fx - (T)0.5, wx);
      weights(v.y - fy - (T)0.5, wy);
      weights(v.z - fz - (T)0.5, wz);
      const A m = (A)v.w;
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const A mz = m * wz[dz];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const A mzy = mz * wy[dy];
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const int c = (dz * 3 + dy) * 3 + dx;
            if constexpr (COMP) {
              float err;
              a27[c] = two_sum(a27[c], mzy * wx[dx], err);
              e27[c] += err;
            } else {
              a27[c] += mzy * wx[dx];
            }
          }
        }
      }
    }
    if (cur >= 0) flush(cur);
  }
  __syncthreads();
  // flush: consecutive threads take consecutive halo-tile cells, so a wave's atomics
  // fall on a few rows of the key-box grid; on a periodic root the cells one past the
  // box edges (-1 and N) are cells N - 1 and 0
  const int tx0 = ox - 1, ty0 = oy - 1, tz0 = oz - 1;
  constexpr int kPer = (kTH3 + kBlock - 1) / kBlock;   // halo cells per thread
  int64_t gidx[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int c = threadIdx.x + k * kBlock;
    gidx[k] = -1;
    if (c >= kTH3 || acc[c] == 0.0) continue;        // both words zero (or an exact zero)
    int gx = tx0 + c % kTH, gy = ty0 + (c / kTH) % kTH, gz = tz0 + c / (kTH * kTH);
    if (L.wrap) {
      gx = wrap_cell(gx + L.key_lo[0], L.wrap) - L.key_lo[0];
      gy = wrap_cell(gy + L.key_lo[1], L.wrap) - L.key_lo[1];
      gz = wrap_cell(gz + L.key_lo[2], L.wrap) - L.key_lo[2];
    }
    if (gx < 0 || gx >= L.key_n[0] || gy < 0 || gy >= L.key_n[1] || gz < 0 || gz >= L.key_n[2])
      continue;
    gidx[k] = ((int64_t)gz * L.key_n[1] + gy) * L.key_n[0] + gx;
  }
  if constexpr (COMP) {
    // every returning add of the thread first, then the error adds
    float* cells = reinterpret_cast<float*>(L.accum);
    float old[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      old[k] = gidx[k] >= 0
                   ? global_add(as_global_mut<float>(cells + 2 * gidx[k]), accp[threadIdx.x + k * kBlock].x)
                   : 0.f;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (gidx[k] < 0) continue;
      const float2 v = accp[threadIdx.x + k * kBlock];
      float e;
      two_sum(old[k], v.x, e);
      global_add(as_global_mut<float>(cells + 2 * gidx[k] + 1), e + v.y);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (gidx[k] >= 0) global_add(as_global_mut<double>(L.accum) + gidx[k], acc[threadIdx.x + k * kBlock]);
  }
}

template <typename T>
hipError_t launch_deposit_tiles(const DepIO<T>& io, const DepLevel* tab, hipStream_t s) {
  const int64_t nb = io.item_blk0[io.nlev];
  if (nb <= 0) return hipSuccess;
  if constexpr (std::is_same<T, float>::value) {
    if (io.comp) {
      hipLaunchKernelGGL((k_deposit_tiles<T, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_deposit_tiles<T, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab);
  return hipGetLastError();
}

// ---- finalize: GMF cell = accumulated mass / dx^3 + gas ------------------------------
// (own gas on active cells, the parent's copied onto ghost cells); kGmfPer GMF cells
// per thread over every grid of every level of the batch.  COMP: the pair's sum,
// scaled by 1/dx^3 (a power of two: exact) in FP32.
template <typename T, bool COMP>
__global__ void __launch_bounds__(kBlock) k_deposit_finalize(DepIO<T> io, const DepLevel* __restrict__ tab) {
  const int lb = batch_level(io.fin_blk0, io.nlev, blockIdx.x);
  // the descriptors as values read once, and global-space pointers (generic loads
  // of their fields in the loops would each wait on the previous memory operation)
  const DepLevel L = load_global(tab + lb);
  const int64_t blk = blockIdx.x - io.fin_blk0[lb];
  const int gi = find_grid(L.block_begin, L.ngrids, blk);
  const GridDesc g = load_global(L.grids + gi);
  const int64_t cells = (int64_t)g.gmf_n[0] * g.gmf_n[1] * g.gmf_n[2];
  const int64_t first = (blk - as_global<int64_t>(L.block_begin)[gi]) * (int64_t)(kBlock * kGmfPer) +
                        threadIdx.x;
  const gptr<T> gas = io.gas[lb] ? as_global<T>(io.gas[lb]) : nullptr;
  const gptr<T> pgas = io.pgas[lb] ? as_global<T>(io.pgas[lb]) : nullptr;
  const gmut<T> out = as_global_mut<T>(io.gmf[lb]) + g.gmf_offset;
  int cx[kGmfPer], cy[kGmfPer], cz[kGmfPer];
  double mass[kGmfPer];
  T add[kGmfPer];
#pragma unroll
  for (int k = 0; k < kGmfPer; ++k) {               // every load first
    const int64_t local = first + (int64_t)k * kBlock;
    const int64_t lc = local < cells ? local : 0;   // a valid cell; not written below
    int lx, ly, lz;
    box_cell(lc, g.gmf_n[0], g.gmf_n[1], lx, ly, lz);
    cx[k] = g.gmf_lo[0] + lx; cy[k] = g.gmf_lo[1] + ly; cz[k] = g.gmf_lo[2] + lz;
    const int64_t kc = ((int64_t)(cz[k] - L.key_lo[2]) * L.key_n[1] + (cy[k] - L.key_lo[1])) *
                           L.key_n[0] + (cx[k] - L.key_lo[0]);
    if constexpr (COMP) {
      const nvec2<float> p = as_global<nvec2<float>>(L.accum)[kc];
      mass[k] = (double)((p.x + p.y) * (float)(L.inv_dx * L.inv_dx * L.inv_dx));
    } else {
      mass[k] = as_global<double>(L.accum)[kc] / (L.dx * L.dx * L.dx);
    }
    const bool active = cx[k] >= g.lo[0] && cx[k] < g.lo[0] + g.n[0] && cy[k] >= g.lo[1] &&
                        cy[k] < g.lo[1] + g.n[1] && cz[k] >= g.lo[2] && cz[k] < g.lo[2] + g.n[2];
    add[k] = (T)0;
    if (active) {
      if (gas)
        add[k] = gas[g.gas_offset + ((int64_t)(cz[k] - g.lo[2]) * g.n[1] + (cy[k] - g.lo[1])) * g.n[0] +
                     (cx[k] - g.lo[0])];
    } else if (pgas && g.parent >= 0) {
      const int px = (cx[k] >> 1) - g.parent_lo[0], py = (cy[k] >> 1) - g.parent_lo[1],
                pz = (cz[k] >> 1) - g.parent_lo[2];
      add[k] = pgas[g.parent_gas_offset + ((int64_t)pz * g.parent_n[1] + py) * g.parent_n[0] + px];
    }
  }
#pragma unroll
  for (int k = 0; k < kGmfPer; ++k) {
    const int64_t local = first + (int64_t)k * kBlock;
    if (local < cells) out[local] = (T)mass[k] + add[k];
  }
}

template <typename T>
hipError_t launch_deposit_finalize(const DepIO<T>& io, const DepLevel* tab, hipStream_t s) {
  const int64_t nb = io.fin_blk0[io.nlev];
  if (nb <= 0) return hipSuccess;
  if constexpr (std::is_same<T, float>::value) {
    if (io.comp) {
      hipLaunchKernelGGL((k_deposit_finalize<T, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, io,
                         tab);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_deposit_finalize<T, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab);
  return hipGetLastError();
}

// ---- owner grid -------------------------------------------------------------------
template <typename T>
__global__ void k_owner(const OwnerLevel* __restrict__ om, int32_t nlev, const T* __restrict__ x,
                        const T* __restrict__ y, const T* __restrict__ z, int64_t npart,
                        int32_t* __restrict__ owner, T* __restrict__ ax, T* __restrict__ ay,
                        T* __restrict__ az, T* __restrict__ pot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npart) return;
  const T px = x[i], py = y[i], pz = z[i];
  const int32_t best = in_domain(px, py, pz) ? owner_lookup(om, nlev, px, py, pz) : -1;
  owner[i] = best;
  if (best < 0 && ax) {
    ax[i] = 0; ay[i] = 0; az[i] = 0;
    if (pot) pot[i] = 0;
  }
}

template <typename T>
hipError_t launch_owner(const OwnerLevel* om, int32_t nlev, const T* x, const T* y, const T* z,
                        int64_t npart, int32_t* owner, T* ax, T* ay, T* az, T* pot, hipStream_t s) {
  if (npart == 0) return hipSuccess;
  const unsigned nb = (unsigned)((npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_owner<T>), dim3(nb), dim3(kBlock), 0, s, om, nlev, x, y, z, npart, owner,
                     ax, ay, az, pot);
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
  const T fx = floor(sx), fy = floor(sy), fz = floor(sz);
  const int64_t off = g.fld_offset;
  const int nx = g.fld_n[0], ny = g.fld_n[1], nz = g.fld_n[2];
  const V4<T> a = tsc_gather<T>(field + off, nx, ny, nz, (int)fx - g.fld_lo[0],
                                (int)fy - g.fld_lo[1], (int)fz - g.fld_lo[2], sx - fx - (T)0.5,
                                sy - fy - (T)0.5, sz - fz - (T)0.5, g.wrap);
  ax[i] = a.x; ay[i] = a.y; az[i] = a.z;
  if (pot) pot[i] = a.w;
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

// Tile-staged interpolation, one block per deposit work item (a tile's chunk of at most
// kChunk sorted entries): on a level of one grid, for chunks of 64 entries or more, the
// 10^3 field cells around the tile (zero outside the field box; wrapped on a periodic
// root) are read into LDS once and every entry's 27-cell gather reads LDS.  The sums
// run in the same order as tsc_gather's, over the same values (a cell outside the box
// contributes an exact zero either way).  Other chunks gather from global memory
// (tsc_gather).  Each owned entry writes one 16 B record at its particle's index.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_interp_tiles(InterpIO<T> io, const DepLevel* __restrict__ tab,
                                                         const GridDesc* __restrict__ grids) {
  __shared__ V4<T> tf[kTH3];
  const int lb = batch_level(io.item_blk0, io.nlev, blockIdx.x);
  const DepLevel L = load_global(tab + lb);   // its fields as values, not re-read after stores
  const int64_t item = blockIdx.x - io.item_blk0[lb];
  const int32_t total = L.items[L.ntiles];
  const int4 wk = L.work[item];                     // in the table's room; read with the count
  if (item >= total) return;                        // uniform for the block
  const int tile = wk.x;
  const int64_t begin = wk.y, end = wk.z;
  int ox, oy, oz;
  tile_origin(L, tile, ox, oy, oz);
  // staged when the level has one grid and the chunk is not sparse (a few entries
  // read fewer bytes with their own gathers than the 10^3 tile)
  const bool staged = L.ngrids == 1 && end - begin >= 64;   // uniform for the block
  const V4<T>* F = io.fld[lb];
  if (staged) {
    const GridDesc& g = grids[L.first];
    const V4<T>* Fg = F + g.fld_offset;
    // halo cell (lx, ly, lz) of the tile is level cell key_lo + o + l - 1
    for (int c = threadIdx.x; c < kTH3; c += kBlock) {
      int x = L.key_lo[0] + ox + c % kTH - 1 - g.fld_lo[0];
      int y = L.key_lo[1] + oy + (c / kTH) % kTH - 1 - g.fld_lo[1];
      int z = L.key_lo[2] + oz + c / (kTH * kTH) - 1 - g.fld_lo[2];
      if (g.wrap) {
        x = wrap_cell(x, g.fld_n[0]);
        y = wrap_cell(y, g.fld_n[1]);
        z = wrap_cell(z, g.fld_n[2]);
      }
      const bool in = x >= 0 && x < g.fld_n[0] && y >= 0 && y < g.fld_n[1] && z >= 0 &&
                      z < g.fld_n[2];
      V4<T> v = load_v4<T>(Fg, in ? ((int64_t)z * g.fld_n[1] + y) * g.fld_n[0] + x : 0);
      if (!in) v = V4<T>{0, 0, 0, 0};
      tf[c] = v;
    }
    __syncthreads();
  }
  const int bx = L.key_lo[0] + ox, by = L.key_lo[1] + oy, bz = L.key_lo[2] + oz;
  for (int k = 0; k < 8; ++k) {
    const int64_t q = begin + threadIdx.x + (int64_t)k * kBlock;
    if (q >= end) break;
    const int2 r = level_ref(L, q);
    if (r.y < 0) continue;
    const V4<T> v = level_rec<T>(L, q);
    const T fx = floor(v.x), fy = floor(v.y), fz = floor(v.z);
    const T tx = v.x - fx - (T)0.5, ty = v.y - fy - (T)0.5, tz = v.z - fz - (T)0.5;
    V4<T> a;
    if (staged) {
      // the entry's cell inside the tile (its run's tile; clamped defensively)
      const int ix = min(max((int)fx - bx, 0), kTile - 1), iy = min(max((int)fy - by, 0), kTile - 1),
                iz = min(max((int)fz - bz, 0), kTile - 1);
      const T wx[3] = {tsc_w(-1, tx), tsc_w(0, tx), tsc_w(1, tx)};
      const T wy[3] = {tsc_w(-1, ty), tsc_w(0, ty), tsc_w(1, ty)};
      const T wz[3] = {tsc_w(-1, tz), tsc_w(0, tz), tsc_w(1, tz)};
      a.x = 0; a.y = 0; a.z = 0; a.w = 0;
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const T wzy = wz[dz] * wy[dy];
          const V4<T>* row = tf + ((iz + dz) * kTH + iy + dy) * kTH + ix;
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const V4<T> f = row[dx];
            const T w = wzy * wx[dx];
            a.x += w * f.x; a.y += w * f.y; a.z += w * f.z; a.w += w * f.w;
          }
        }
    } else {
      const GridDesc& g = grids[r.y];
      a = tsc_gather<T>(F + g.fld_offset, g.fld_n[0], g.fld_n[1], g.fld_n[2], (int)fx - g.fld_lo[0],
                        (int)fy - g.fld_lo[1], (int)fz - g.fld_lo[2], tx, ty, tz, g.wrap);
    }
    io.res[r.x] = a;                              // one 16 B record at the particle's index
  }
}

template <typename T>
hipError_t launch_interp_tiles(const InterpIO<T>& io, const DepLevel* tab, const GridDesc* grids,
                               hipStream_t s) {
  const int64_t nb = io.item_blk0[io.nlev];
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_interp_tiles<T>), dim3((unsigned)nb), dim3(kBlock), 0, s, io, tab, grids);
  return hipGetLastError();
}

// Records -> the four output arrays: particle i's record, written at index i by its
// owner level's interpolation, is read coalesced (zero where owner < 0).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_unpack(InterpIO<T> io, const DepLevel* __restrict__ tab,
                                                   const int32_t* __restrict__ owner, int64_t npart,
                                                   T* __restrict__ ax, T* __restrict__ ay,
                                                   T* __restrict__ az, T* __restrict__ pot) {
  (void)tab;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= npart) return;
  const int32_t og = owner[i];
  const V4<T> r = load_v4<T>(io.res, i);
  const V4<T> v = og >= 0 ? r : V4<T>{0, 0, 0, 0};
  ax[i] = v.x; ay[i] = v.y; az[i] = v.z;
  if (pot) pot[i] = v.w;
}

template <typename T>
hipError_t launch_unpack(const InterpIO<T>& io, const DepLevel* tab, const int32_t* owner,
                         int64_t npart, T* ax, T* ay, T* az, T* pot, hipStream_t s) {
  if (npart <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((npart + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_unpack<T>), dim3(nb), dim3(kBlock), 0, s, io, tab, owner, npart, ax, ay, az,
                     pot);
  return hipGetLastError();
}


// ---- subcycled evolution -------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_assign(SubIO<T> io) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= io.npart || io.lev[i] < io.level) return;
  const T px = io.x[i], py = io.y[i], pz = io.z[i];
  const int o = in_domain(px, py, pz) ? owner_lookup(io.om, io.nlev, px, py, pz) : -1;
  io.lev[i] = max(io.level, o >= 0 ? io.grids[o].level : 0);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_predict(SubIO<T> io) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= io.npart) return;
  const T d = (T)(io.tm - io.clock[io.lev[i]]);
  io.xp[i] = io.x[i] + io.vx[i] * d;
  io.yp[i] = io.y[i] + io.vy[i] * d;
  io.zp[i] = io.z[i] + io.vz[i] * d;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_move(SubIO<T> io) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= io.npart || io.lev[i] != io.level) return;
  const T px = io.xp[i], py = io.yp[i], pz = io.zp[i];
  const int o = in_domain(px, py, pz) ? owner_lookup(io.om, io.level + 1, px, py, pz) : -1;
  V4<T> a{0, 0, 0, 0};
  if (o >= 0) {
    const GridDesc& g = io.grids[o];
    const T s = (T)(1.0 / g.dx);
    const T sx = px * s, sy = py * s, sz = pz * s;
    const T fx = floor(sx), fy = floor(sy), fz = floor(sz);
    a = tsc_gather<T>(io.fld[g.level] + g.fld_offset, g.fld_n[0], g.fld_n[1], g.fld_n[2],
                      (int)fx - g.fld_lo[0], (int)fy - g.fld_lo[1], (int)fz - g.fld_lo[2],
                      sx - fx - (T)0.5, sy - fy - (T)0.5, sz - fz - (T)0.5, g.wrap);
  }
  const T h = (T)io.h, hh = (T)(0.5 * io.h);
  const T vx = io.vx[i] + h * a.x, vy = io.vy[i] + h * a.y, vz = io.vz[i] + h * a.z;
  io.vx[i] = vx; io.vy[i] = vy; io.vz[i] = vz;
  io.x[i] = px + hh * vx;
  io.y[i] = py + hh * vy;
  io.z[i] = pz + hh * vz;
}

template <typename T> hipError_t launch_sub_assign(const SubIO<T>& io, hipStream_t s) {
  if (io.npart <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sub_assign<T>), dim3((unsigned)((io.npart + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, io);
  return hipGetLastError();
}
template <typename T> hipError_t launch_sub_predict(const SubIO<T>& io, hipStream_t s) {
  if (io.npart <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sub_predict<T>), dim3((unsigned)((io.npart + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, io);
  return hipGetLastError();
}
template <typename T> hipError_t launch_sub_move(const SubIO<T>& io, hipStream_t s) {
  if (io.npart <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sub_move<T>), dim3((unsigned)((io.npart + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, io);
  return hipGetLastError();
}

#define APM_INST(T)                                                                          \
  template hipError_t launch_deposit_tiles<T>(const DepIO<T>&, const DepLevel*, hipStream_t);  \
  template hipError_t launch_deposit_finalize<T>(const DepIO<T>&, const DepLevel*, hipStream_t); \
  template hipError_t launch_sub_assign<T>(const SubIO<T>&, hipStream_t);                     \
  template hipError_t launch_sub_predict<T>(const SubIO<T>&, hipStream_t);                    \
  template hipError_t launch_sub_move<T>(const SubIO<T>&, hipStream_t);                       \
  template hipError_t launch_owner<T>(const OwnerLevel*, int32_t, const T*, const T*, const T*, \
                                      int64_t, int32_t*, T*, T*, T*, T*, hipStream_t);          \
  template hipError_t launch_interp_tiles<T>(const InterpIO<T>&, const DepLevel*,               \
                                             const GridDesc*, hipStream_t);                     \
  template hipError_t launch_unpack<T>(const InterpIO<T>&, const DepLevel*, const int32_t*,     \
                                       int64_t, T*, T*, T*, T*, hipStream_t);                   \
  template hipError_t launch_interp<T>(const GridDesc*, int32_t, const V4<T>*, const T*,       \
                                       const T*, const T*, const int32_t*, int64_t, T*, T*, T*, \
                                       T*, hipStream_t);
APM_INST(float)
APM_INST(double)

}  // namespace apm
