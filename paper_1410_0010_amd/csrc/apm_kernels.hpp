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
constexpr int kZConvMaxThreads = 512;     // keeps the FP64 z passes free of spills
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
// one value of every octant pair (comp 0: Gf) in the working precision
template <typename T> hipError_t launch_table_pick(const double* pairs, T* out, int64_t n, int comp,
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
hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s);

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

// Particles: binning by 8^3 tile of the particle's cell i0 = floor(x/dx) inside the
// level's binning box (union of GMF boxes grown by one cell), then the tile-wise
// TSC deposit.  Every stage is one launch over a batch of consecutive levels.
constexpr int kTile = 8;
constexpr int kHaloCells = (kTile + 2) * (kTile + 2) * (kTile + 2);   // tile + one-cell halo
constexpr int kMaxRep = 16;        // counter replicas per tile, at most (a power of two)
constexpr int kChunk = 2048;       // particles per deposit work item

// Static part of one level (device table, rewritten only when buffers move).
struct DepLevel {
  double inv_dx, dx;
  int32_t key_lo[3], key_n[3];     // binning box (cells)
  int32_t tiles_n[3];              // tiles per axis
  int32_t ntiles, rep;             // rep: counter replicas per tile (power of two)
  int32_t first, ngrids;           // the level's grids: [first, first + ngrids)
  int32_t wrap;                    // periodic root: cells per axis (clouds wrap), else 0
  int64_t key_cells;
  int32_t* count;                  // ntiles * rep + 1; replica r of tile t at t rep + r;
                                   // scanned in place into start offsets
  int32_t* items;                  // ntiles + 1: scanned work-item counts
  int4* work;                      // work item -> (tile, first entry, end entry, 0); room
                                   // for ntiles + ceil(npart / kChunk) items
  int2* bsum;                      // per 256 tiles: (count, items) sums, then their starts
  int32_t* key;                    // npart: counter slot or -1
  int32_t* rank;                   // npart: rank within the slot
  int2* sref;                      // sorted position -> (original index, owner grid if
                                   // that grid is on this level, else -1)
  void* sorted;                    // npart records (x/dx, y/dx, z/dx, m); x/dx is exact
  double* accum;                   // key_cells FP64 mass (the reverse sweep: GMF cotangent)
  const GridDesc* grids;           // the level's grids
  const int64_t* block_begin;      // first finalize block of each grid (ngrids + 1)
  int32_t* binned;                 // number of particles binned on the level
};

// Per-call part: the particles, the batch's block offsets and its in/out buffers
// (index b = level - first level of the batch).
template <typename T> struct DepIO {
  const T* x; const T* y; const T* z; const T* m;
  const int32_t* owner;                // owner grid per particle, or null (no owners)
  const OwnerLevel* om;                // or the owner lookup of every level (om_nlev), the
  int32_t om_nlev;                     // owner computed in the scatter, and written to
  int32_t* owner_out;                  // owner_out (if not null) by the root level's blocks
  int64_t npart;
  int32_t nlev;
  int64_t item_blk0[kMaxLevels + 1];   // deposit-tile blocks of level b: [item_blk0[b], [b+1])
  int64_t fin_blk0[kMaxLevels + 1];    // finalize blocks of level b
  const T* gas[kMaxLevels];            // level active gas (packed) or null
  const T* pgas[kMaxLevels];           // parent level active gas (packed) or null
  T* gmf[kMaxLevels];
};
hipError_t launch_dep_clear(const DepLevel* tab, int nlev, int64_t max_elems, hipStream_t s);
template <typename T> hipError_t launch_bin_count(const DepIO<T>& io, const DepLevel* tab,
                                                  hipStream_t s);
hipError_t launch_bin_scan(const DepLevel* tab, int nlev, int32_t max_tiles, hipStream_t s);
template <typename T> hipError_t launch_bin_scatter(const DepIO<T>& io, const DepLevel* tab,
                                                    hipStream_t s);
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
  int64_t part_blk0[kMaxLevels + 1];   // sorted-list blocks
  const V4<T>* fld[kMaxLevels];        // forward composed fields
  double* fbar[kMaxLevels];            // field cotangents, FP64: 4 per field cell, or
                                       // the Phi one alone (dense) when c0 == 3
  const T* gmf_bar[kMaxLevels];        // GMF cotangents
  double* gas_bar[kMaxLevels];         // own-gas cotangent of the level, or null
  double* pgas_bar[kMaxLevels];        // the parent level's gas cotangent, or null
  // Per-entry partial results, in the working precision T (each is one term of a
  // sum over at most a few levels, formed in FP64 and rounded once), stored at the
  // entry's tile-sorted position on its level (coalesced):
  V4<T>* pint[kMaxLevels];             // per level: the interpolation transpose's
                                       // position gradient (x, y, z; owned entries)
  V4<T>* plev[kMaxLevels];             // per level: the deposit transpose's
                                       // (mbar, xbar, ybar, zbar) (binned entries)
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
template <typename T> hipError_t launch_adj_finish(const AdjIO<T>& io, const DepLevel* tab,
                                                   const int32_t* owner, const T* pot, T* xb,
                                                   T* yb, T* zb, T* mb, hipStream_t s);
template <typename T> hipError_t launch_to_t(const double* a, T* b, int64_t n, hipStream_t s);
hipError_t launch_add_scalar(double* a, int64_t n, const double* s, double scale, hipStream_t st);

template <typename T> hipError_t launch_compose(const GridDesc* grids, const int64_t* block_begin,
                                                int32_t ngrids, const V4<T>* own,
                                                const V4<T>* parent, V4<T>* field,
                                                int64_t nblocks, hipStream_t s);
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

}  // namespace apm
