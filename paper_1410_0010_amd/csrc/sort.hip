// The particle sort shared by every level's deposit and interpolation (Sec. 2: the
// TSC assignment visits particles tile by tile).
//
// Each particle gets the Morton code of its kTile^3 tile on the sort's finest level
// (floor(x N_f) / kTile per axis, bits interleaved with x lowest).  A particle outside
// [0, 1)^3 takes the code of the last tile and a record of zero mass at a point of
// that tile's last cell, so it adds nothing to any grid, and its owner -1 keeps it out
// of the interpolation.  A stable least-significant-digit radix sort of (key, index)
// pairs, at most 9 bits a pass, orders the particles; a gather then writes the sorted
// records and references.  A tile s levels coarser holds the finest tiles whose codes
// share all but the lowest 3 s bits, so its particles form one run of the list;
// k_tile_ranges finds every level's runs in one read of the sorted keys.
//
// A pass is three steps: per-block digit counts (kRadixTile keys a block), their
// exclusive scan in digit-major order (so each block knows where its keys of each
// digit go), and the scatter.  There each wave ranks its quarter of the block's keys
// stably in 16 rounds of 64: wavefront ballots give a lane's rank among the lanes
// with its digit, and a per-wave count of each digit in LDS carries over between
// rounds, so no barrier is needed until the block combines its waves' counts; the
// keys are then sorted by digit in LDS and each digit's run is written with
// consecutive threads on consecutive addresses.  No global atomics: the per-level
// counting by global atomics that this replaces serialised the many blocks of a dense
// core on the same few counters.
#include <algorithm>

#include "apm_kernels.hpp"

namespace apm {

namespace {

constexpr int kMaxRadixBits = 9, kMaxDigits = 1 << kMaxRadixBits;
constexpr int kRadixWaves = kRadixBlock / 64;
constexpr int kWaveItems = kRadixTile / kRadixWaves;   // keys per wave (16 rounds of 64)
constexpr int kScanChunk = 4096;                    // digit counts per scan block
constexpr int kScanMid = 1024;                      // threads of the partials' scan
static_assert(kMaxDigits == 2 * kRadixBlock, "two digits per thread");

template <typename K> __device__ __forceinline__ K spread3(uint32_t v, int nb) {
  K r = 0;
  for (int j = 0; j < nb; ++j) r |= (K)((v >> j) & 1u) << (3 * j);
  return r;
}
template <typename K> __device__ __forceinline__ int32_t compact3(K c, int nb) {
  uint32_t r = 0;
  for (int j = 0; j < nb; ++j) r |= (uint32_t)((c >> (3 * j)) & 1u) << j;
  return (int32_t)r;
}
template <typename K> __device__ __forceinline__ K shr(K k, int s) {
  return s >= (int)(8 * sizeof(K)) ? (K)0 : (K)(k >> s);
}

template <typename T>
__device__ __forceinline__ bool in_unit_box(T x, T y, T z) {
  return x >= (T)0 && x < (T)1 && y >= (T)0 && y < (T)1 && z >= (T)0 && z < (T)1;
}

// ---- keys, owners, packed records -----------------------------------------------------
template <typename T, typename K>
__global__ void __launch_bounds__(kBlock) k_sort_keys(SortIO<T> io) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= io.npart) return;
  const T x = io.x[i], y = io.y[i], z = io.z[i], m = io.m[i];
  const bool in = in_unit_box(x, y, z);
  const int nb = io.nbits / 3;
  // outside: the last cell, 1 - 1/N_f per axis (exact for N_f <= 2^24), zero mass
  const T s = (T)io.cells_f, edge = (T)1 - (T)1 / s;
  const T px = in ? x : edge, py = in ? y : edge, pz = in ? z : edge;
  // x N_f is exact (a power of two) and below N_f for x < 1
  const uint32_t tx = (uint32_t)(int32_t)floor(px * s) / kTile,
                 ty = (uint32_t)(int32_t)floor(py * s) / kTile,
                 tz = (uint32_t)(int32_t)floor(pz * s) / kTile;
  const K key = spread3<K>(tx, nb) | (spread3<K>(ty, nb) << 1) | (spread3<K>(tz, nb) << 2);
  if (io.om) io.owner[i] = in ? owner_lookup(io.om, io.om_nlev, x, y, z) : -1;
  reinterpret_cast<K*>(io.key[0])[i] = key;
  io.idx[0][i] = in ? (int32_t)i : ~(int32_t)i;      // outside: the complement (negative)
  as_global_mut<nvec4<T>>(io.prec)[i] = nvec4<T>{px, py, pz, in ? m : (T)0};
}

// ---- per-block digit counts ------------------------------------------------------------
template <typename K>
__global__ void __launch_bounds__(kRadixBlock) k_radix_hist(const K* __restrict__ key, int64_t n,
                                                            int shift, int rb,
                                                            uint32_t* __restrict__ hist,
                                                            int64_t nblk) {
  __shared__ uint32_t h[kMaxDigits];
  const int nd = 1 << rb;
  for (int d = threadIdx.x; d < nd; d += kRadixBlock) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  const gptr<K> kg = as_global<K>(key);
  K k[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {            // all loads first
    const int64_t q = base + r * kRadixBlock + threadIdx.x;
    k[r] = q < n ? kg[q] : (K)0;
  }
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t q = base + r * kRadixBlock + threadIdx.x;
    if (q < n) atomicAdd(&h[(uint32_t)(k[r] >> shift) & (uint32_t)(nd - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nd; d += kRadixBlock) hist[(int64_t)d * nblk + blockIdx.x] = h[d];
}

// ---- exclusive scan of the counts (three launches) ---------------------------------------
// Exclusive prefix sum over a block of NT threads of one value each; *tot = block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* sh, uint32_t* tot) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t base = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t a = sh[w];
    base += w < wave ? a : 0u;
    sum += a;
  }
  __syncthreads();                                   // sh reused by the next call
  *tot = sum;
  return base + inc - v;
}

constexpr int kScanPer = kScanChunk / kRadixBlock;  // 16 counts per thread

__global__ void __launch_bounds__(kRadixBlock) k_hscan_reduce(const uint32_t* __restrict__ a,
                                                              int64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t sh[kRadixWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) s += base + j < n ? a[base + j] : 0u;
  uint32_t tot;
  block_exscan<kRadixBlock>(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanMid) k_hscan_mid(uint32_t* __restrict__ sums, int64_t n) {
  __shared__ uint32_t sh[kScanMid / 64];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < n; b0 += kScanMid) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < n ? sums[b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exscan<kScanMid>(v, sh, &tot);
    if (b < n) sums[b] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(kRadixBlock) k_hscan_down(uint32_t* __restrict__ a, int64_t n,
                                                            const uint32_t* __restrict__ sums) {
  __shared__ uint32_t sh[kRadixWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer], s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    v[j] = base + j < n ? a[base + j] : 0u;
    s += v[j];
  }
  uint32_t tot;
  uint32_t o = sums[blockIdx.x] + block_exscan<kRadixBlock>(s, sh, &tot);
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    if (base + j < n) a[base + j] = o;
    o += v[j];
  }
}

// ---- stable scatter by one digit ------------------------------------------------------------
// Key j of the block (input position base + j) is taken by wave j / kWaveItems in round
// (j % kWaveItems) / 64, lane j % 64: (wave, round, lane) order is input order.
template <typename K>
__global__ void __launch_bounds__(kRadixBlock)
k_radix_scatter(const K* __restrict__ kin, const int32_t* __restrict__ iin, K* __restrict__ kout,
                int32_t* __restrict__ iout, int64_t n, int shift, int rb,
                const uint32_t* __restrict__ offs, int64_t nblk) {
  __shared__ K sk[kRadixTile];
  __shared__ int32_t si[kRadixTile];
  __shared__ uint32_t wc[kRadixWaves][kMaxDigits];  // per-wave digit counts, then starts
  __shared__ uint32_t ls[kMaxDigits], gs[kMaxDigits];   // block-local and global digit starts
  __shared__ uint32_t sh[kRadixWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nd = 1 << rb;
  const uint32_t dmask = (uint32_t)nd - 1;
  const int64_t blk0 = (int64_t)blockIdx.x * kRadixTile;
  const int64_t base = blk0 + (int64_t)wave * kWaveItems;
  const gptr<K> kg = as_global<K>(kin);
  const gptr<int32_t> ig = as_global<int32_t>(iin);
  K k[kRadixItems];
  int32_t id[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t q = base + r * 64 + lane;
    k[r] = q < n ? kg[q] : (K)0;
    id[r] = q < n ? ig[q] : 0;
  }
  for (int d = threadIdx.x; d < nd; d += kRadixBlock) {
#pragma unroll
    for (int w = 0; w < kRadixWaves; ++w) wc[w][d] = 0;
    gs[d] = offs[(int64_t)d * nblk + blockIdx.x];
  }
  __syncthreads();
  uint32_t* mine = wc[wave];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));   // lanes below this one
  uint32_t rank[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const bool valid = base + r * 64 + lane < n;
    const uint32_t d = (uint32_t)(k[r] >> shift) & dmask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < rb; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t lr = (uint32_t)__popcll(peers & lt);
    // the wave's earlier keys of this digit; the digit's leader (lowest lane) then
    // adds the round's count (the wave's LDS accesses complete in program order)
    const uint32_t prior = mine[d];
    rank[r] = prior + lr;
    if (valid && lr == 0) mine[d] = prior + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {                                                  // digits 2t, 2t + 1 of thread t
    const int d0 = 2 * threadIdx.x, d1 = d0 + 1;
    uint32_t c0[kRadixWaves], c1[kRadixWaves], t0 = 0, t1 = 0;
#pragma unroll
    for (int w = 0; w < kRadixWaves; ++w) {
      c0[w] = d0 < nd ? wc[w][d0] : 0u;
      c1[w] = d1 < nd ? wc[w][d1] : 0u;
      t0 += c0[w];
      t1 += c1[w];
    }
    uint32_t tot;
    const uint32_t s0 = block_exscan<kRadixBlock>(t0 + t1, sh, &tot), s1 = s0 + t0;
    if (d0 < nd) ls[d0] = s0;
    if (d1 < nd) ls[d1] = s1;
    uint32_t a0 = s0, a1 = s1;
#pragma unroll
    for (int w = 0; w < kRadixWaves; ++w) {       // wave w's first local position per digit
      if (d0 < nd) wc[w][d0] = a0;
      if (d1 < nd) wc[w][d1] = a1;
      a0 += c0[w];
      a1 += c1[w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    if (base + r * 64 + lane < n) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & dmask;
      const uint32_t p = mine[d] + rank[r];
      sk[p] = k[r];
      si[p] = id[r];
    }
  }
  __syncthreads();
  const int cnt = n - blk0 < kRadixTile ? (int)(n - blk0) : kRadixTile;
  for (int j = threadIdx.x; j < cnt; j += kRadixBlock) {
    const K kk = sk[j];
    const uint32_t d = (uint32_t)(kk >> shift) & dmask;
    const int64_t o = (int64_t)gs[d] + (j - (int64_t)ls[d]);
    kout[o] = kk;
    iout[o] = si[j];
  }
}

// ---- sorted records and references ---------------------------------------------------------
// The owner grid is looked up again from the record (the particle's own position when
// inside the domain), not read back at the particle's index: one random read a
// particle instead of two.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sort_gather(SortIO<T> io, const int32_t* __restrict__ idx) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= io.npart) return;
  const int32_t e = as_global<int32_t>(idx)[q];
  const bool in = e >= 0;
  const int32_t p = in ? e : ~e;
  const V4<T> v = load_v4<T>(io.prec, p);
  const int32_t o = (io.om && in) ? owner_lookup(io.om, io.om_nlev, v.x, v.y, v.z) : -1;
  as_global_mut<nvec4<T>>(io.sorted)[q] = nvec4<T>{v.x, v.y, v.z, v.w};
  as_global_mut<nvec2<int32_t>>(io.sref)[q] = nvec2<int32_t>{p, o};
}

// ---- every level's tile runs -----------------------------------------------------------------
// Thread q: for each level of the batch, entry q starts (ends) a run when the previous
// (next) key differs in the bits above the level's shift; the run's code is decoded to
// the level's tile, whose begin (end) the thread writes when the tile lies in the
// level's tile box.
template <typename K>
__global__ void __launch_bounds__(kBlock) k_tile_ranges(const DepLevel* __restrict__ tab, int nlev,
                                                        const K* __restrict__ key, int nbits,
                                                        int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const gptr<K> kg = as_global<K>(key);
  const K k = kg[q];
  const bool has_prev = q > 0, has_next = q + 1 < n;
  const K kp = has_prev ? kg[q - 1] : (K)0, kn = has_next ? kg[q + 1] : (K)0;
  for (int b = 0; b < nlev; ++b) {
    const DepLevel& L = tab[b];
    const int s = L.shift;
    const K c = shr(k, s);
    const bool start = !has_prev || shr(kp, s) != c;
    const bool end = !has_next || shr(kn, s) != c;
    if (!start && !end) continue;
    const int nb = (nbits - s) / 3;
    const int tx = compact3<K>(c, nb) - L.tile_lo[0], ty = compact3<K>(c >> 1, nb) - L.tile_lo[1],
              tz = compact3<K>(c >> 2, nb) - L.tile_lo[2];
    if (tx < 0 || tx >= L.tiles_n[0] || ty < 0 || ty >= L.tiles_n[1] || tz < 0 ||
        tz >= L.tiles_n[2])
      continue;
    const int t = (tz * L.tiles_n[1] + ty) * L.tiles_n[0] + tx;
    if (start) L.tbegin[t] = (int32_t)q;
    if (end) L.tend[t] = (int32_t)(q + 1);
  }
}

template <typename T, typename K>
hipError_t sort_impl(const SortIO<T>& io, int* which, hipStream_t s) {
  const int64_t n = io.npart;
  *which = 0;
  if (n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_sort_keys<T, K>), dim3(nb), dim3(kBlock), 0, s, io);
  const int64_t nblk = (n + kRadixTile - 1) / kRadixTile;
  const int passes = sort_passes(io.nbits);
  const int rb = passes > 0 ? (io.nbits + passes - 1) / passes : 0;
  const int64_t nh = nblk << rb;
  const int64_t nsum = (nh + kScanChunk - 1) / kScanChunk;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * rb;
    const K* kin = (const K*)io.key[cur];
    hipLaunchKernelGGL((k_radix_hist<K>), dim3((unsigned)nblk), dim3(kRadixBlock), 0, s, kin, n,
                       shift, rb, io.hist, nblk);
    hipLaunchKernelGGL(k_hscan_reduce, dim3((unsigned)nsum), dim3(kRadixBlock), 0, s, io.hist, nh,
                       io.hsum);
    hipLaunchKernelGGL(k_hscan_mid, dim3(1), dim3(kScanMid), 0, s, io.hsum, nsum);
    hipLaunchKernelGGL(k_hscan_down, dim3((unsigned)nsum), dim3(kRadixBlock), 0, s, io.hist, nh,
                       io.hsum);
    hipLaunchKernelGGL((k_radix_scatter<K>), dim3((unsigned)nblk), dim3(kRadixBlock), 0, s, kin,
                       io.idx[cur], (K*)io.key[1 - cur], io.idx[1 - cur], n, shift, rb, io.hist,
                       nblk);
    cur = 1 - cur;
  }
  hipLaunchKernelGGL((k_sort_gather<T>), dim3(nb), dim3(kBlock), 0, s, io, io.idx[cur]);
  *which = cur;
  return hipGetLastError();
}

}  // namespace

int64_t sort_hist_elems(int64_t npart) {
  return std::max<int64_t>(1, (npart + kRadixTile - 1) / kRadixTile) * kMaxDigits;
}
int64_t sort_sum_elems(int64_t npart) {
  return (sort_hist_elems(npart) + kScanChunk - 1) / kScanChunk;
}

template <typename T>
hipError_t launch_particle_sort(const SortIO<T>& io, int* which, hipStream_t s) {
  if (io.nbits < 0 || io.nbits > kMaxMortonBits || io.nbits % 3 != 0) return hipErrorInvalidValue;
  return sort_key64(io.nbits) ? sort_impl<T, uint64_t>(io, which, s)
                              : sort_impl<T, uint32_t>(io, which, s);
}

hipError_t launch_tile_ranges(const DepLevel* tab, int nlev, const void* skey, int nbits,
                              int64_t npart, hipStream_t s) {
  if (npart <= 0 || nlev == 0) return hipSuccess;
  const unsigned nb = (unsigned)((npart + kBlock - 1) / kBlock);
  if (sort_key64(nbits))
    hipLaunchKernelGGL((k_tile_ranges<uint64_t>), dim3(nb), dim3(kBlock), 0, s, tab, nlev,
                       (const uint64_t*)skey, nbits, npart);
  else
    hipLaunchKernelGGL((k_tile_ranges<uint32_t>), dim3(nb), dim3(kBlock), 0, s, tab, nlev,
                       (const uint32_t*)skey, nbits, npart);
  return hipGetLastError();
}

template hipError_t launch_particle_sort<float>(const SortIO<float>&, int*, hipStream_t);
template hipError_t launch_particle_sort<double>(const SortIO<double>&, int*, hipStream_t);

}  // namespace apm
