// Launcher interfaces between the ABI layer and the kernels (all on one stream).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "apm_internal.hpp"
#include "device_common.hpp"

namespace apm {

// Optional timing hook called around every kernel launch (phase 0 before, 1 after).
struct LaunchHook {
  void (*fn)(void* user, const char* name, int phase) = nullptr;
  void* user = nullptr;
  void operator()(const char* name, int phase) const { if (fn) fn(user, name, phase); }
};

constexpr int kMaxLevels = 21;
template <typename T> struct LevelPtrs {
  const T* gmf[kMaxLevels];        // packed GMF buffer of each level
  V4<T>* fld[kMaxLevels];          // packed (own) field buffer of each level
};

// The five transform passes of a grid's convolution, and the five of its transpose
// (each adjoint pass runs one forward pass backwards, with that pass's launch shape).
enum { PASS_X_FWD = 0, PASS_Y_FWD = 1, PASS_Z_CONV = 2, PASS_Y_INV = 3, PASS_X_INV = 4,
       PASS_AX = 5, PASS_AY = 6, PASS_AZ = 7, PASS_AYI = 8, PASS_AXI = 9,
       // potential-only transposes (zero acceleration cotangents)
       PASS_APX = 10, PASS_APY = 11, PASS_APZ = 12 };
// forward pass whose launch shape an adjoint pass shares
inline int mirror_pass(int pass) {
  switch (pass) {
    case PASS_AX: return PASS_X_INV;
    case PASS_AY: return PASS_Y_INV;
    case PASS_AZ: return PASS_Z_CONV;
    case PASS_AYI: return PASS_Y_FWD;
    case PASS_AXI: return PASS_X_FWD;
    case PASS_APX: return PASS_X_FWD;
    case PASS_APY: return PASS_Y_FWD;
    case PASS_APZ: return PASS_Z_CONV;
  }
  return pass;
}

// Spectrum and z-buffer rows are stored in tiles of kYT rows along ky: row (plane p,
// ky) of a region of np planes sits kYT ((ky / kYT) np + p) + ky % kYT rows from the
// region's start.  A column along the planes (the z pass) then steps kYT rows, so it
// crosses a few memory pages instead of one per plane (a 1024-plane column of a
// plane-major 1024^2 spectrum touched over a thousand pages per block, and the
// address translation, not HBM, set the z pass's pace); a line along ky steps one row
// within a tile and np kYT rows between tiles.  Every FFT length is a multiple of kYT.
constexpr int kYT = 16;
__host__ __device__ __forceinline__ int64_t tile_row(int p, int ky, int np) {
  return ((int64_t)(ky / kYT) * np + p) * kYT + (ky % kYT);
}

// One grid in one pass: GMF (dims g) zero-padded into FFT box M, outputs on the field
// box (dims f) whose first cell sits at transform index off (cyclic).  Offsets are
// in elements of the level GMF buffer, the level field buffer (cells) and the
// shared spectrum, z-output (3 fz My W per grid) and y-output (4 fz fy W per grid)
// buffers (complex values).
constexpr int kRowAlign = 16;      // row pitch granularity (complex values): 128 B or more
struct ConvJob {
  int64_t blk0;                    // first block of this job in its launch
  int32_t level;
  int32_t g[3], M[3], f[3], off[3];
  int32_t pitch;                   // complex values per row of the spectrum, z and y
                                   // buffers: W = Mx/2 + 1 rounded up to kRowAlign
  int64_t gmf_off, fld_off, spec_off, z_off, y_off;
  const void* kern;                // octant table: kstride values per entry, Gf first
  int32_t kstride;                 // 2: (Gf, Gp) pairs; 1: Gf alone, the potential's kernel
                                   // too (spectral gradient): then the z pass writes two
                                   // arrays and the y inverse pass three lines per column
  int32_t kpot;                    // offset of the potential's kernel in an entry (1 or 0)
  const void* dsym[3];             // gradient symbols per axis index
  const double* mean;              // periodic plans, subgrids: device scalar, the average
                                   // density subtracted from the GMF; else null
};
int64_t pass_blocks(int pass, const int g[3], const int M[3], const int f[3], int nl);
template <typename T> int default_lines(int pass, int L);
// threads per block of the passes that hold two sets of line values per thread (the z
// passes, the y inverse pass): 512 keeps the FP64 kernels free of spills
template <typename T> constexpr int kTwoSetThreads = sizeof(T) == 4 ? 1024 : 512;
constexpr int kMaxLDS = 163840;           // dynamic LDS per workgroup on gfx950
hipError_t allow_lds_forward();           // raise every transform kernel's LDS limit
hipError_t allow_lds_adjoint();
// nc: lines per column of the y inverse pass: 3 with single-kernel tables (kstride 1,
// the z pass then writes two arrays), else 4
template <typename T> size_t pass_lds(int pass, int L, int nl, int nc = 4);  // 0: not launchable
template <typename T> int pass_row_stride(int pass, int L, int nl); // LDS line stride
int pass_threads(int pass, int L, int nl, int nc = 4);
template <typename T>
hipError_t launch_pass(int pass, int L, int nl, int nc, const ConvJob* jobs, int njobs,
                       int64_t nblocks, const LevelPtrs<T>& lp, C2<T>* spec, C2<T>* zbuf,
                       C2<T>* ybuf, const void* tw, hipStream_t s);
// Working octant tables (the kernel values the z passes multiply by) are tiled for
// those passes' reads: entry (kx, |ky|, |kz|) of an Mx x My x Mz box sits at
// ((|ky| NT + kx / kOctKx) Oz + |kz|) kOctKx + kx mod kOctKx, NT = ceil((Mx/2 + 1) /
// kOctKx), Oz = Mz/2 + 1.  A block's kOctKx neighbouring columns and a wavefront's
// consecutive kz then read one contiguous run instead of one short piece per kz.
constexpr int kOctKx = 4;
__host__ __device__ __forceinline__ int oct_tiles(int Mx) { return (Mx / 2 + kOctKx) / kOctKx; }
__host__ __device__ __forceinline__ int64_t oct_entries(int Mx, int My, int Mz) {
  return (int64_t)oct_tiles(Mx) * kOctKx * (My / 2 + 1) * (Mz / 2 + 1);
}
// offset of column kx's run of |ky| row kyo (entry |kz| follows at kz kOctKx)
__host__ __device__ __forceinline__ int64_t oct_col(int kx, int kyo, int Mx, int Mz) {
  return ((int64_t)kyo * oct_tiles(Mx) + kx / kOctKx) * (Mz / 2 + 1) * kOctKx + kx % kOctKx;
}
// The working table from the FP64 (Gf, Gp) pairs in natural order (index (|kz| (My/2+1)
// + |ky|) (Mx/2+1) + kx): KS = 1 takes value comp of each pair, KS = 2 both.
template <typename T, int KS>
hipError_t launch_table_tiles(const double* pairs, T* out, int Mx, int My, int Mz, int comp,
                              hipStream_t s);

// Buffers of the transposed convolution: GMF cotangents out (working precision) and
// FP64 field-box cotangents in (field layout: 4 per cell, or the Phi one alone for the
// potential-only passes), per level.
template <typename T> struct AdjPtrs {
  T* gmf[kMaxLevels];
  const double* fbar[kMaxLevels];
};
template <typename T>
hipError_t launch_adj_pass(int pass, int L, int nl, const ConvJob* jobs, int njobs, int64_t nblocks,
                           const AdjPtrs<T>& ap, C2<T>* spec, C2<T>* zbuf, C2<T>* ybuf,
                           const void* tw, hipStream_t s);

// Green's functions (FP64): octant table of (force, potential) times `norm`.
struct InfluenceParams {
  int Mx, My, Mz;
  double dx, a_l, a_lm1;   // a_lm1 < 0: root (S_{-1} = 0)
  double G, norm;
  int bz, grad;
  const double* james;     // isolated root: octant of the doubled-mesh reference kernel
                           // (null with a_lm1 < 0: the periodic root)
};
hipError_t launch_influence(const InfluenceParams& p, double2* out, hipStream_t s);
hipError_t launch_james(int N, double dx, double a0, double G, const double* costab,
                        double* buf0, double* buf1, double** result, hipStream_t s);

// Owner lookup (finest grid whose active box holds a point, lowest index on that level):
// per level either its single grid's active box or, for several grids, a table over
// the bounding box of their active boxes with the lowest-index grid of every cell.
struct OwnerLevel {
  double inv_dx;
  int32_t lo[3], n[3];             // box (level cells)
  int32_t single;                  // the grid if the level has one, else -1
  const int32_t* table;            // n[0] n[1] n[2] grid indices (-1: none), or null
};
__device__ __forceinline__ int owner_lookup(const OwnerLevel* __restrict__ om, int nlev, double px,
                                            double py, double pz) {
  for (int l = nlev - 1; l >= 0; --l) {
    const OwnerLevel& o = om[l];
    const int cx = (int)floor(px * o.inv_dx) - o.lo[0];
    const int cy = (int)floor(py * o.inv_dx) - o.lo[1];
    const int cz = (int)floor(pz * o.inv_dx) - o.lo[2];
    if (cx < 0 || cx >= o.n[0] || cy < 0 || cy >= o.n[1] || cz < 0 || cz >= o.n[2]) continue;
    const int g = o.single >= 0 ? o.single : o.table[((int64_t)cz * o.n[1] + cy) * o.n[0] + cx];
    if (g >= 0) return g;
  }
  return -1;
}

// Particles: one sort of every particle by the Morton code (bits interleaved, x in
// the lowest) of its kTile^3-cell tile on the sort's finest level, tiles aligned at
// multiples of kTile cells on every level.  A tile s levels coarser is a cube of 2^(3s)
// finest tiles whose codes form one aligned range, so on every level each tile's
// particles are one contiguous run of the sorted list: the levels share the list,
// each finds its tiles' runs, and the tile-wise TSC deposit reads them.  Every
// per-level stage is one launch over a batch of consecutive levels.
constexpr int kTile = 8;
constexpr int kHaloCells = (kTile + 2) * (kTile + 2) * (kTile + 2);   // tile + one-cell halo
constexpr int kChunk = 2048;       // particles per deposit work item
constexpr int kMaxMortonBits = 63; // tiles per axis of the sort's finest level up to 2^21

// Static part of one level (device table, rewritten only when buffers move).
struct DepLevel {
  double inv_dx, dx;
  int32_t key_lo[3], key_n[3];     // binning box (cells): the level's GMF boxes grown by one
  int32_t tile_lo[3];              // global index of the first tile covering the box
  int32_t tiles_n[3];              // tiles per axis
  int32_t ntiles;
  int32_t shift;                   // Morton bits below the level's tiles: 3 (sort's finest
                                   // level - level)
  int32_t first, ngrids;           // the level's grids: [first, first + ngrids)
  int32_t wrap;                    // periodic root: cells per axis (clouds wrap), else 0
  int64_t key_cells;
  int32_t* tbegin;                 // ntiles: first sorted position of each tile's run
  int32_t* tend;                   // ntiles: one past its last (both 0: empty tile)
  int32_t* items;                  // ntiles + 1: scanned work-item counts
  int4* work;                      // work item -> (tile, first entry, end entry, 0); room
                                   // for ntiles + ceil(npart / kChunk) items
  int2* bsum;                      // per 256 tiles: (count, items) sums, then their starts
  const int2* sref;                // the shared sorted list: (original index, owner grid)
  const void* sorted;              // the shared sorted list: (x, y, z, m), world units
  double* accum;                   // key_cells FP64 mass (the reverse sweep: GMF cotangent)
  const GridDesc* grids;           // the level's grids
  const int64_t* block_begin;      // first finalize block of each grid (ngrids + 1)
};

// First cell of tile t of a level, relative to the level's binning box (between
// 1 - kTile and 0 for the first tile of an axis).
__host__ __device__ __forceinline__ void tile_origin(const DepLevel& L, int t, int& ox, int& oy,
                                                     int& oz) {
  ox = (L.tile_lo[0] + t % L.tiles_n[0]) * kTile - L.key_lo[0];
  oy = (L.tile_lo[1] + (t / L.tiles_n[0]) % L.tiles_n[1]) * kTile - L.key_lo[1];
  oz = (L.tile_lo[2] + t / (L.tiles_n[0] * L.tiles_n[1])) * kTile - L.key_lo[2];
}
// Entry q of the sorted list in the level's cell units (exact: dx is a power of two).
template <typename T> __device__ __forceinline__ V4<T> level_rec(const DepLevel& L, int64_t q) {
  V4<T> v = load_v4<T>(L.sorted, q);
  const T s = (T)L.inv_dx;
  v.x *= s; v.y *= s; v.z *= s;
  return v;
}
// (original index, owner grid when that grid is on the level, else -1) of entry q
__device__ __forceinline__ int2 level_ref(const DepLevel& L, int64_t q) {
  int2 r = load_i2(L.sref, q);
  if (r.y < L.first || r.y >= L.first + L.ngrids) r.y = -1;
  return r;
}

// The particle sort (sort.hip), once per solve or deposit, before any level's tiles.
// Keys are 32-bit while nbits < 32, else 64-bit.
constexpr int kRadixBlock = 256, kRadixItems = 16, kRadixTile = kRadixBlock * kRadixItems;
template <typename T> struct SortIO {
  const T* x; const T* y; const T* z; const T* m;
  int64_t npart;
  double cells_f;                      // cells per axis of the sort's finest level
  int32_t nbits;                       // Morton bits of its tiles (3 per axis)
  const OwnerLevel* om;                // owner lookup of every level, or null (no owners:
  int32_t om_nlev;                     // the sorted references hold -1)
  int32_t* owner;                      // out (with om): owner grid per particle, -1 outside
  void* key[2];                        // npart each: ping-pong keys
  int32_t* idx[2];                     // npart each: ping-pong original indices (their
                                       // complement for particles outside [0, 1)^3)
  void* prec;                          // npart records (x, y, z, m) in input order (outside
                                       // [0, 1)^3: a point of the last tile, mass 0)
  uint32_t* hist;                      // sort_hist_elems(npart): digit counts, then their
                                       // exclusive scan (digit-major)
  uint32_t* hsum;                      // scan partials, sort_sum_elems(npart)
  void* sorted;                        // out: npart records (x, y, z, m), sorted
  int2* sref;                          // out: npart (original index, owner grid)
};
int64_t sort_hist_elems(int64_t npart);
int64_t sort_sum_elems(int64_t npart);
inline bool sort_key64(int nbits) { return nbits > 32; }
// radix passes of at most 9 bits over the nbits key bits; the sorted keys end in
// ping-pong slot passes % 2
inline int sort_passes(int nbits) { return (nbits + 8) / 9; }
// The whole sort on s; *which gets the ping-pong slot (0 or 1) holding the sorted keys.
template <typename T> hipError_t launch_particle_sort(const SortIO<T>& io, int* which,
                                                      hipStream_t s);

// Per-call part: the batch's block offsets and its in/out buffers (index b = level -
// first level of the batch).
template <typename T> struct DepIO {
  int64_t npart;
  int32_t nlev;
  int32_t comp;                        // T = float: 1 = compensated FP32 accumulation (the
                                       // key-box grid holds (sum, error) FP32 pairs)
  int64_t item_blk0[kMaxLevels + 1];   // deposit-tile blocks of level b: [item_blk0[b], [b+1])
  int64_t fin_blk0[kMaxLevels + 1];    // finalize blocks of level b
  const T* gas[kMaxLevels];            // level active gas (packed) or null
  const T* pgas[kMaxLevels];           // parent level active gas (packed) or null
  T* gmf[kMaxLevels];
};
hipError_t launch_dep_clear(const DepLevel* tab, int nlev, int64_t max_elems, hipStream_t s);
// each tile's run of the sorted keys (sorted by launch_particle_sort with nbits) on
// every level of the batch; tbegin and tend cleared before (launch_dep_clear)
hipError_t launch_tile_ranges(const DepLevel* tab, int nlev, const void* skey, int nbits,
                              int64_t npart, hipStream_t s);
hipError_t launch_bin_scan(const DepLevel* tab, int nlev, int32_t max_tiles, hipStream_t s);
template <typename T> hipError_t launch_deposit_tiles(const DepIO<T>& io, const DepLevel* tab,
                                                      hipStream_t s);
template <typename T> hipError_t launch_deposit_finalize(const DepIO<T>& io, const DepLevel* tab,
                                                         hipStream_t s);

// owner grid of every particle; where the outputs are given, particles outside the
// domain (owner -1) get zero acceleration and potential there
template <typename T> hipError_t launch_owner(const OwnerLevel* om, int32_t nlev, const T* x,
                                              const T* y, const T* z, int64_t npart,
                                              int32_t* owner, T* ax, T* ay, T* az, T* pot,
                                              hipStream_t s);
template <typename T> hipError_t launch_interp(const GridDesc* grids, int32_t level,
                                               const V4<T>* field, const T* x, const T* y,
                                               const T* z, const int32_t* owner, int64_t npart,
                                               T* ax, T* ay, T* az, T* pot, hipStream_t s);
// TSC interpolation over the tile-sorted lists of a batch of levels (one launch):
// entry q of level b is interpolated from the composed field fld[b] of its owner
// grid when that grid is on level b, and written to the particle's original slot.
template <typename T> struct InterpIO {
  int32_t nlev;
  int64_t item_blk0[kMaxLevels + 1];   // work-item blocks of level b (the deposit's items)
  const V4<T>* fld[kMaxLevels];
  V4<T>* res;                          // (a_x, a_y, a_z, Phi) of every owned particle,
                                       // at its own index
};
// interpolation of every level's owned particles, one block per deposit work item
// (the tile's field in LDS where it pays)
template <typename T> hipError_t launch_interp_tiles(const InterpIO<T>& io, const DepLevel* tab,
                                                     const GridDesc* grids, hipStream_t s);
// the records (res, particle order) -> the four per-particle output arrays (zero
// where owner < 0); pot may be null
template <typename T> hipError_t launch_unpack(const InterpIO<T>& io, const DepLevel* tab,
                                               const int32_t* owner, int64_t npart, T* ax, T* ay,
                                               T* az, T* pot, hipStream_t s);
// ---- reverse sweep (adjoint.hip) ----
struct ZeroList {                      // FP64 ranges to clear in one launch
  double* p[48];
  int64_t n[48];
  int32_t count;
};
hipError_t launch_zero_ranges(const ZeroList& zl, hipStream_t s);
template <typename T> struct AdjIO {
  int32_t nlev;                        // levels of the batch (b = level - first)
  int32_t c0;                          // first non-zero cotangent component (3: Phi only)
  int64_t npart;
  double wbar;                         // weight of W in the loss
  const T* abx; const T* aby; const T* abz;   // acceleration cotangents (npart)
  const T* phib;                       // potential cotangents (npart) or null
  int64_t item_blk0[kMaxLevels + 1];   // interpolation-transpose blocks (deposit items)
  int64_t fin_blk0[kMaxLevels + 1];    // GMF-cell blocks
  const V4<T>* fld[kMaxLevels];        // forward composed fields
  double* fbar[kMaxLevels];            // field cotangents, FP64: 4 per field cell, or
                                       // the Phi one alone (dense) when c0 == 3
  const T* gmf_bar[kMaxLevels];        // GMF cotangents
  double* gas_bar[kMaxLevels];         // own-gas cotangent of the level, or null
  double* pgas_bar[kMaxLevels];        // the parent level's gas cotangent, or null
  // Per-entry partial results, in the working precision T (each is one term of a
  // sum over at most a few levels, formed in FP64 and rounded once), stored at the
  // entry's position in the sorted list (coalesced):
  V4<T>* pint;                         // the interpolation transpose's position gradient
                                       // (x, y, z; owned entries)
  V4<T>* plev[kMaxLevels];             // per level: the deposit transpose's
                                       // (mbar, xbar, ybar, zbar) (entries of the level's
                                       // tiles)
  V4<T>* pout;                         // per particle (original index): the gradient
                                       // record (mbar, xbar, ybar, zbar)
  const double* rbar;                  // periodic: device scalar, the cotangent of the
                                       // average density (added to every in-domain
                                       // particle's mass cotangent); else null
};
template <typename T> hipError_t launch_adj_interp(const AdjIO<T>& io, const DepLevel* tab,
                                                   const GridDesc* grids, hipStream_t s);
template <typename T> hipError_t launch_adj_gas_seed(const GridDesc* grids, const OwnerLevel* om,
                                                     int32_t nlev, int32_t first, int32_t count,
                                                     const int64_t* begin, int64_t nblocks,
                                                     const T* gas, const V4<T>* field, double wbar,
                                                     double* fbar, int fs, double* gas_bar,
                                                     hipStream_t s);
hipError_t launch_adj_restrict(const GridDesc* grids, int32_t first, int32_t count,
                               const int64_t* begin, int64_t nblocks, const double* child_bar,
                               double* parent_bar, int fs, hipStream_t s);   // fs: 4 or 1 per cell
template <typename T> hipError_t launch_adj_deposit_grid(const AdjIO<T>& io, const DepLevel* tab,
                                                         hipStream_t s);
template <typename T> hipError_t launch_adj_deposit_particles(const AdjIO<T>& io,
                                                              const DepLevel* tab, hipStream_t s);
// the particle gradients (two launches: sums in sorted order into io.pout, then the
// four arrays in particle order, zero where owner < 0); any output may be null
template <typename T> hipError_t launch_adj_finish(const AdjIO<T>& io, const DepLevel* tab,
                                                   const int32_t* owner, const T* pot, T* xb,
                                                   T* yb, T* zb, T* mb, hipStream_t s);
template <typename T> hipError_t launch_to_t(const double* a, T* b, int64_t n, hipStream_t s);
hipError_t launch_add_scalar(double* a, int64_t n, const double* s, double scale, hipStream_t st);

// field = own + P(parent) on every grid of a level (own may be field: in place); with
// pprev, P((1 - alpha) pprev + alpha parent), the parent taken linearly in time
template <typename T> hipError_t launch_compose(const GridDesc* grids, const int64_t* block_begin,
                                                int32_t ngrids, const V4<T>* own,
                                                const V4<T>* parent, V4<T>* field,
                                                int64_t nblocks, hipStream_t s,
                                                const V4<T>* pprev = nullptr, double alpha = 1.0);
// ---- subcycled evolution (particles.hip) ----
template <typename T> struct SubIO {
  int64_t npart;
  T* x; T* y; T* z; T* vx; T* vy; T* vz;
  T* xp; T* yp; T* zp;                 // positions predicted to the step's mid-time
  int32_t* lev;                        // level each particle moves with
  double clock[kMaxLevels];            // the levels' clocks
  int32_t level;                       // the stepping level
  double h, tm;                        // its step and mid-step time
  const OwnerLevel* om;
  int32_t nlev;
  const GridDesc* grids;
  const V4<T>* fld[kMaxLevels];        // latest composed field of every level <= level
};
// particles of level >= io.level: level = max(io.level, level of the owner grid)
template <typename T> hipError_t launch_sub_assign(const SubIO<T>& io, hipStream_t s);
// every particle: xp = x + v (tm - clock[lev])
template <typename T> hipError_t launch_sub_predict(const SubIO<T>& io, hipStream_t s);
// particles of io.level: v += h a(xp) (finest grid of level <= io.level holding xp),
// x = xp + v h / 2
template <typename T> hipError_t launch_sub_move(const SubIO<T>& io, hipStream_t s);
// Deterministic FP64 reductions: per-block partials (part, kMaxParts per quantity),
// then one block sums them in a fixed order into out.
constexpr int kMaxParts = 1024;
template <typename T> hipError_t launch_sum_scaled(const T* a, int64_t n, double scale,
                                                   double* part, double* out, hipStream_t s);
template <typename T> hipError_t launch_particle_totals(const T* m, const int32_t* owner,
                                                        int64_t npart, const T* ax, const T* ay,
                                                        const T* az, const T* pot, double* part,
                                                        double* out, hipStream_t s);
// Totals of a solve in two launches: every level's GMF sum and the particle sums
// leave partials at part[q kMaxParts + b] (q < nlev: levels, then W_p and sum m a);
// then one block per quantity writes out[0..nlev + 5) in a fixed order: scaled level
// masses, W (+ *gas_w), sum m a, W_gas (*gas_w, or 0).
template <typename T> struct TotalsIO {
  int32_t nlev;
  const T* gmf[kMaxLevels];
  int64_t gmf_n[kMaxLevels];
  double vol[kMaxLevels];              // dx^3 of the level
  const T* m; const int32_t* owner; int64_t npart;
  const T* ax; const T* ay; const T* az; const T* pot;
  const double* gas_w;                 // device scalar W_gas, or null
  double* part;                        // (nlev + 4) kMaxParts doubles
  double* out;                         // nlev + 5 doubles
};
template <typename T> hipError_t launch_totals(const TotalsIO<T>& io, hipStream_t s);
// number and mass of the particles outside [0, 1)^3 or with a NaN coordinate, added to
// out[0] (the count, as a double) and out[1]; partials in part (2 kMaxParts doubles)
template <typename T> hipError_t launch_dropped(const T* x, const T* y, const T* z, const T* m,
                                                int64_t npart, double* part, double* out,
                                                hipStream_t s);
// out[q] += scale * sum_{b < nparts} part[q * kMaxParts + b], q < nq (fixed order;
// with nq = 1 any nparts)
hipError_t launch_sum_parts(const double* part, int nparts, int nq, double scale, double* out,
                            hipStream_t s);
// Average density of a periodic system: (sum of the in-domain particle masses + sum
// of the root gas times vol) over the unit box, into out[0] (written, not added);
// per-block partials in part (kMaxParts doubles).  gas may be null.
template <typename T> hipError_t launch_mean_density(const T* x, const T* y, const T* z,
                                                     const T* m, int64_t npart, const T* gas,
                                                     int64_t ngas, double vol, double* part,
                                                     double* out, hipStream_t s);
// time integration and energy terms (dynamics.hip); wrap != 0: drifted positions are
// taken modulo 1 (periodic box)
template <typename T> hipError_t launch_kick_drift(int64_t n, T* x, T* y, T* z, T* vx, T* vy,
                                                   T* vz, const T* ax, const T* ay, const T* az,
                                                   double hk, double hd, int wrap, hipStream_t s);
template <typename T> hipError_t launch_kinetic(const T* m, const T* vx, const T* vy, const T* vz,
                                                int64_t n, double* part, double* out,
                                                hipStream_t s);
template <typename T> hipError_t launch_gas_energy(const GridDesc* grids, const OwnerLevel* om,
                                                   int32_t nlev, int32_t first, int32_t count,
                                                   const int64_t* begin, int64_t nblocks,
                                                   const T* gas, const V4<T>* field, double* part,
                                                   double* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, hipStream_t s);  // one value
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);

constexpr int kBlock = 256;
// GMF cells per thread in the deposit's finalize pass and in its transpose (the grid
// side): kGmfPer coalesced rows of a block, their loads issued together, so each thread
// keeps several reads in flight and a block's table lookups serve more cells; the
// per-grid block tables count kBlock kGmfPer cells
constexpr int kGmfPer = 8;

}  // namespace apm
