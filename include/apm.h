/*
 * apm.h -- C ABI of the adaptive particle-mesh (APM) gravity solve on static
 * nested grids for AMD MI355X (gfx950), after Passy & Bryan, "An adaptive
 * particle-mesh gravity solver for ENZO".
 *
 * The library computes, per grid of a static hierarchy (level 0 = root covering
 * the unit box, each level refined by 2):
 *   apm_deposit      TSC mass assignment of particles plus gas into the grid's
 *                    GravitatingMassField (GMF)                       (Sec. 2)
 *   apm_solve_level  zero-padded FFT convolution with the optimal influence
 *                    function and differencing in Fourier space: the grid's own
 *                    (short-range) acceleration and potential   (Sec. 2.2, Eq. 2-9)
 *   apm_accel        composition with the parent: parent field interpolated onto
 *                    the grid plus its own short-range field        (Sec. 2.2)
 *   apm_interp       TSC interpolation of the composed field to the particles
 * plus host-side planning, the owner-grid query and FP64 totals.
 *
 * Conventions (all calls):
 *  - Units: box [0,1)^3, gravitational constant G from apm_config (code units).
 *  - Indices: level-l cell c spans [c, c+1) * dx_l, dx_l = 1/(root_n 2^l).
 *    Boxes are (lo[3], n[3]) in level-l global cell indices, (x, y, z) order.
 *  - 3-D arrays are x-fastest: element (x, y, z) of a box of dims (nx, ny, nz)
 *    sits at ((z * ny) + y) * nx + x.
 *  - "Packed level buffer": the grids of one level, in grid-index order, each
 *    at the offset that apm_plan_grid reports.
 *  - Field buffers hold 4 values per cell, interleaved: (a_x, a_y, a_z, Phi).
 *  - dtype APM_F32 or APM_F64 applies to every floating array of a call.
 *  - Array arguments of the compute calls are DEVICE pointers on the context's
 *    device, owned by the caller.  The library never frees or retains them and
 *    overwrites outputs.  It owns only the plan, the context, the cached Green's
 *    functions and its workspace.
 *  - Compute calls are asynchronous on the context's stream unless stated.
 *  - Every call returns an apm_status; on error apm_last_error() (thread-local)
 *    describes it.  No call aborts the process.
 *  - A context is used by one host thread at a time (calls on it are not
 *    synchronised with each other); different contexts may be used concurrently.
 *    apm_solve may run part of its work on a second stream of the context, forked
 *    from and joined back to the context's stream within the call.
 */
#ifndef APM_H
#define APM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APM_OK = 0,
  APM_ERR_INVALID = 1,      /* bad argument, descriptor or nesting            */
  APM_ERR_OOM = 2,          /* device allocation failed or workspace limit    */
  APM_ERR_DEVICE = 3,       /* no usable device / HIP runtime error           */
  APM_ERR_RANGE = 4,        /* size beyond a supported maximum                */
  APM_ERR_UNSUPPORTED = 5,  /* valid request the library does not support     */
  APM_ERR_STATE = 6         /* call out of order (e.g. missing parent field)  */
} apm_status;

typedef enum { APM_F32 = 1, APM_F64 = 2 } apm_dtype;

/* Gradient operator D of Eq. 5 and of the differencing (Sec. 2.2 names both). */
typedef enum {
  APM_GRAD_SPECTRAL = 0,    /* D(k) = -i k (default)                            */
  APM_GRAD_FD2 = 1          /* two-point central difference, -i sin(k dx)/dx  */
} apm_gradient;

/* Boundary condition of the root grid (Sec. 2.1 gives the Green's function of both;
 * the sine wave test of Sec. 3 uses the periodic one). */
typedef enum {
  APM_BC_ISOLATED = 0,      /* isolated: the root's kernel made isolated on the
                               doubled mesh (James), FFT length 2 root_n (default)  */
  APM_BC_PERIODIC = 1       /* periodic: the root's kernel is Eq. 5 taken directly
                               in Fourier space on the root's own mesh, zero at
                               k = 0; FFT length root_n; the average density of the
                               system is subtracted from every grid's GMF before its
                               convolution (zero net mass); the root's TSC clouds
                               and interpolation stencils wrap at the box edges    */
} apm_boundary;

/* Accumulation of the FP32 deposit (apm_deposit, apm_solve with APM_F32; the FP64
 * dtype always accumulates in FP64).  Sec. 2 sums each particle's TSC weights into
 * the 27 cells around it; both modes give the exact sum to well below FP32 rounding
 * before the GMF is rounded once. */
typedef enum {
  APM_ACC_F64 = 0,          /* sums in FP64 registers, LDS and key-box grid       */
  APM_ACC_F32_COMP = 1      /* FP32 throughout: TwoSum-compensated (sum, error)
                               pairs in registers, in LDS and in the level's
                               key-box grid (Kahan-style compensation)            */
} apm_accum;

typedef struct {
  double G;                 /* gravitational constant [1.0]                       */
  int32_t root_n;           /* root cells per axis, power of two in [8, 512]
                               (isolated) or [8, 1024] (periodic)                 */
  double a_cells;           /* S2 softening a_l = a_cells * dx_l [3.4] (Sec. 2.2) */
  double pad_factor;        /* subgrid zero padding p = ceil(pad_factor * 2 *
                               a_cells) cells per axis [0.65] (Sec. 2.2)           */
  int32_t ghost;            /* GMF ghost width of subgrids [3]                    */
  int32_t brillouin;        /* alias zones n in [-b, b]^3 in Eq. 5 [1] (Eq. 6)    */
  int32_t gradient;         /* apm_gradient [APM_GRAD_SPECTRAL]                   */
  int64_t workspace_limit;  /* bytes of device workspace allowed, 0 = no limit    */
  int32_t boundary;         /* apm_boundary of the root [APM_BC_ISOLATED]         */
  int32_t strict;           /* [0] 1: apm_deposit and apm_solve return APM_ERR_RANGE
                               (after writing their outputs, and synchronising) when
                               a particle has a coordinate outside [0,1) or NaN;
                               0: such particles are left out silently (see
                               apm_dropped)                                        */
  int32_t deposit_accum;    /* apm_accum of the FP32 deposit [APM_ACC_F64]        */
} apm_config;

/* One grid of the static hierarchy.  Grid 0 must be the root: level 0, parent
 * -1, lo = 0, n = root_n.  A subgrid has level >= 1, a parent of level-1 with a
 * smaller index, even lo and n >= 2 even, and its GMF box (active box grown by
 * `ghost` cells) must lie over its parent's active box: parent cells
 * floor((lo-ghost)/2) .. floor((lo+n+ghost-1)/2) on every axis (with ghost = 3:
 * 2 parent cells of margin). */
typedef struct {
  int32_t level;
  int32_t parent;
  int32_t lo[3];
  int32_t n[3];
} apm_grid;

/* Derived layout of one grid (apm_plan_grid). */
typedef struct {
  int32_t level, parent;
  int32_t lo[3], n[3];       /* active box                                        */
  int32_t gmf_lo[3], gmf_n[3];  /* GMF box: active (root) or active +- ghost     */
  int32_t fld_lo[3], fld_n[3];  /* field box: active (root) or active +- 1       */
  int32_t fft_n[3];          /* FFT lengths M (root: 2 root_n isolated, root_n
                                periodic; subgrids: zero-padded)                  */
  int64_t gmf_offset;        /* element offset in the level's packed GMF buffer   */
  int64_t fld_offset;        /* cell offset in the level's packed field buffer    */
  int64_t gas_offset;        /* element offset in the level's packed gas buffer   */
  double dx;                 /* cell size of the grid's level                      */
} apm_grid_layout;

typedef struct {
  int32_t ngrids;            /* grids on this level                               */
  int32_t first_grid;        /* index of its first grid (grids sorted by level)   */
  int64_t gmf_elems;         /* scalars in the packed GMF buffer                  */
  int64_t fld_cells;         /* cells in the packed field buffer (x4 values)       */
  int64_t gas_elems;         /* scalars in the packed active-gas buffer           */
  double dx;
} apm_level_layout;

typedef struct apm_plan_s* apm_plan;
typedef struct apm_ctx_s* apm_ctx;

/* ---------------------------------------------------------------- host only -- */

/* Fill cfg with the defaults in brackets above (root_n = 0: must be set). */
void apm_config_default(apm_config* cfg);

/* Validate a hierarchy and compute its layout (no device needed).
 * grids: host array of ngrids descriptors, sorted by level, parents first.
 * On success *out owns a plan to release with apm_plan_destroy.
 * Errors: APM_ERR_INVALID (descriptor / nesting), APM_ERR_RANGE (FFT length
 * beyond 1024, index space beyond int32, or a finest level of more than 2^24
 * cells per axis: root_n 2^maxlevel <= 2^24). */
apm_status apm_plan_create(const apm_config* cfg, const apm_grid* grids, int32_t ngrids,
                           apm_plan* out);
apm_status apm_plan_destroy(apm_plan plan);
int32_t apm_plan_nlevels(apm_plan plan);                     /* -1 if plan is NULL */
int32_t apm_plan_ngrids(apm_plan plan);
apm_status apm_plan_grid(apm_plan plan, int32_t grid, apm_grid_layout* out);
apm_status apm_plan_level(apm_plan plan, int32_t level, apm_level_layout* out);

/* Thread-local description of the last error of this thread; never NULL. */
const char* apm_last_error(void);

/* -------------------------------------------------------------- device side -- */

/* Bind a copy of `plan` to HIP device `device` and stream `stream` (a
 * hipStream_t, NULL = default stream).  Allocates the workspace lazily.
 * Errors: APM_ERR_DEVICE when no device is visible or it cannot be used. */
apm_status apm_create(apm_plan plan, int32_t device, void* stream, apm_ctx* out);
apm_status apm_destroy(apm_ctx ctx);
apm_status apm_set_stream(apm_ctx ctx, void* stream);

/* Finest grid whose active box holds each particle, lowest index among grids of
 * that level; -1 for particles with a coordinate outside [0,1) or NaN.
 * Owner of the TSC interpolation (Sec. 3.1, 3.2: particles take the force of the
 * grid they live on).  x, y, z: npart values; owner: npart int32 (device). */
apm_status apm_owner(apm_ctx ctx, apm_dtype dtype, const void* x, const void* y,
                     const void* z, int64_t npart, int32_t* owner);

/* GravitatingMassField of every grid of `level` (Sec. 2): the TSC density
 * sum_p m_p W(x_c - x_p) / dx^3 of every in-domain particle whose cloud overlaps
 * the grid's GMF box (clouds clipped at the box; the modified deposition of Sec. 2
 * that also takes the parent's and its siblings' particles), plus gas: `gas` on
 * active cells, `parent_gas` copied piecewise-constant onto the ghost cells.
 *   x, y, z, m  npart positions (box units) and masses
 *   gas         packed active-gas buffer of `level` or NULL (no own gas)
 *   parent_gas  packed active-gas buffer of level-1 or NULL (no ghost gas)
 *   gmf         out: packed GMF buffer of `level` (gmf_elems scalars)
 * The TSC weights and the accumulation are FP64 for both dtypes (the mass of a
 * cell is summed in FP64 and rounded once to the dtype), so the FP32 result is
 * the FP32 rounding of the FP64 sum up to the order of additions.  The level's
 * library-owned binning is rebuilt for these particles, so the state that
 * apm_solve_adjoint needs is gone until the next apm_solve.
 * Periodic plans: at level 0 the clouds wrap around the box edges, and the call
 * also records in the context the average density of the system, (sum of the
 * in-domain particle masses + sum of `gas` dx_0^3) / 1, that apm_solve_level of a
 * subgrid level subtracts. */
apm_status apm_deposit(apm_ctx ctx, apm_dtype dtype, int32_t level, const void* x,
                       const void* y, const void* z, const void* m, int64_t npart,
                       const void* gas, const void* parent_gas, void* gmf);

/* Own field of every grid of `level` (Sec. 2.2, Eq. 2, 5-9): the GMF zero-padded to
 * the FFT box, transformed, multiplied by the level's influence function and
 * transformed back, the potential Phi = IDFT(G rho_hat) with Eq. 5's kernel G and
 * the three acceleration components differenced in Fourier space
 * (a_i = IDFT(-i d_i G rho_hat)).  With APM_GRAD_FD2, where Eq. 5's kernel is
 * unbounded next to the Nyquist corners, the potential takes Hockney and
 * Eastwood's potential-optimal kernel instead.  Root: isolated boundary
 * on the doubled mesh, or periodic (kernel zero at k = 0); subgrids: short-range
 * reference S_l^2 - S_{l-1}^2.  Periodic plans: a subgrid level's GMF is convolved
 * minus the average density recorded by the last level-0 apm_deposit or apm_solve
 * of this context (APM_ERR_STATE if there was none).
 *   gmf    packed GMF buffer of `level` (input, not modified)
 *   field  out: packed field buffer of `level`, 4 values per cell
 * The Green's functions are generated in FP64 on the device on first use and
 * cached (Sec. 2.2: cached Green's functions). */
apm_status apm_solve_level(apm_ctx ctx, apm_dtype dtype, int32_t level, const void* gmf,
                           void* field);

/* Composition with the parent (Sec. 2.2): on every cell of the field boxes of
 * `level`, field = own + P(parent_field), P = trilinear interpolation between
 * cell centres.  At level 0 parent_field must be NULL and field = own.
 * own and field may be the same buffer. */
apm_status apm_accel(apm_ctx ctx, apm_dtype dtype, int32_t level, const void* own,
                     const void* parent_field, void* field);

/* TSC interpolation of the composed field of `level` to the particles whose owner
 * grid is on `level` (Sec. 2: particles take their acceleration from the mesh with
 * the assignment's own TSC weights, which gives no self-force on one level, as the
 * self-force test of Sec. 3.1 relies on; Sec. 3.2: the force on a particle is that
 * of the finest grid it lies on).  Stencils wrap at the box edges on a periodic
 * root.  field: the level's composed field (apm_accel output layout); x, y, z:
 * npart positions; owner: npart owner grids (apm_owner); writes a_x, a_y, a_z and
 * Phi of those particles only (others untouched); pot may be NULL.  Errors:
 * APM_ERR_INVALID for a NULL array, APM_ERR_RANGE for npart outside [0, 2^31). */
apm_status apm_interp(apm_ctx ctx, apm_dtype dtype, int32_t level, const void* field,
                      const void* x, const void* y, const void* z, const int32_t* owner,
                      int64_t npart, void* ax, void* ay, void* az, void* pot);

/* FP64 totals.  out[0 .. nlevels-1]: deposited mass per level (sum over the level's
 * GMF cells of rho dx^3, i.e. particles + gas, clouds clipped);
 * out[nlevels + 0] = 1/2 sum_p m_p Phi_p over owned particles,
 * out[nlevels + 1..3] = sum_p m_p a_p over owned particles.
 * gmf: host array of nlevels device pointers; m, ax, ay, az, pot, owner as above.
 * Synchronises the stream (results are on the host on return). */
apm_status apm_totals(apm_ctx ctx, apm_dtype dtype, const void* const* gmf, const void* m,
                      const int32_t* owner, int64_t npart, const void* ax, const void* ay,
                      const void* az, const void* pot, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): apm_totals with its results
 * written to out_dev (nlevels + 4 FP64 values, a device array the caller owns, same
 * layout as apm_totals' out) in stream order, without synchronising and without any
 * allocation: the reduction partials live in a fixed device array of the library,
 * (21 + 4) * 1024 doubles (200 KiB), one per device, held until the process ends and
 * shared by every call on that device.  Each call rewrites every partial it reads,
 * so nothing carries over between calls; calls that overlap on one device (other
 * streams, other contexts, other threads) race on the array and must be ordered by
 * the caller.  Arguments as in apm_totals.  Errors: APM_ERR_INVALID for NULL
 * arguments, APM_ERR_RANGE for npart < 0 or more levels than the array holds. */
apm_status apm_totals_noalloc(apm_ctx ctx, apm_dtype dtype, const void* const* gmf,
                              const void* m, const int32_t* owner, int64_t npart, const void* ax,
                              const void* ay, const void* az, const void* pot, double* out_dev);

/* The particles a deposit leaves out: those with a coordinate outside [0,1) or NaN
 * (Sec. 2 deposits the particles that lie on the grids; they get no acceleration).
 * Their number into *count and their total mass (FP64) into *mass, from npart
 * positions and masses (device arrays of dtype).  The deposited mass itself is the
 * per-level sum of apm_totals / apm_solve_totals.  Synchronises.  Errors:
 * APM_ERR_INVALID for NULL arguments, APM_ERR_RANGE for npart < 0. */
apm_status apm_dropped(apm_ctx ctx, apm_dtype dtype, const void* x, const void* y, const void* z,
                       const void* m, int64_t npart, int64_t* count, double* mass);

/* The whole forward solve in one call: owner, deposit, solve, composition and
 * interpolation of every level, in the paper's order, into library-owned level
 * buffers (periodic plans: the average density is computed from the particles and
 * the root's gas first and subtracted from every subgrid GMF; the root's kernel
 * removes it from the root).  gas: host array of nlevels device pointers (or NULL entries / NULL).
 * ax, ay, az, pot: npart outputs (pot may be NULL).  Fields of level l can be
 * read back with apm_field_ptr after the call. */
apm_status apm_solve(apm_ctx ctx, apm_dtype dtype, const void* x, const void* y,
                     const void* z, const void* m, int64_t npart, const void* const* gas,
                     void* ax, void* ay, void* az, void* pot);

/* Totals of the last apm_solve of `dtype` over its library-owned GMFs, owner grids
 * and composed fields; m, gas, ax, ay, az, pot as passed to it (gas may be NULL).
 * out has nlevels + 5 entries: out[0..nlevels) deposited mass per level as in
 * apm_totals; out[nlevels] the potential energy W = 1/2 sum_p m_p Phi_p (owned
 * particles) + 1/2 sum rho_gas Phi dx^3 (active gas cells owned by their grid:
 * no finer grid and no lower-index grid of the level contains the cell centre);
 * out[nlevels + 1..3] sum_p m_p a_p; out[nlevels + 4] the gas part of W.
 * Synchronises. */
apm_status apm_solve_totals(apm_ctx ctx, apm_dtype dtype, const void* m, int64_t npart,
                            const void* const* gas, const void* ax, const void* ay,
                            const void* az, const void* pot, double* out);

/* apm_solve_totals without the synchronisation: the same nlevels + 5 FP64 values are
 * written to out_dev, a device array the caller owns, in stream order (so a step
 * loop can keep them on the GPU and read them when it needs them).  The library's
 * totals scratch is reused by the next totals call: calls on one context are
 * ordered by its stream.  APM_ERR_INVALID for a NULL out_dev; APM_ERR_STATE as for
 * apm_solve_totals.  Asynchronous. */
apm_status apm_solve_totals_async(apm_ctx ctx, apm_dtype dtype, const void* m, int64_t npart,
                                  const void* const* gas, const void* ax, const void* ay,
                                  const void* az, const void* pot, double* out_dev);

/* Gas part of the potential energy of one level (as in apm_solve_totals) from its
 * packed active gas and its composed field (apm_accel output layout).  Written to
 * *out; synchronises. */
apm_status apm_gas_energy(apm_ctx ctx, apm_dtype dtype, int32_t level, const void* gas,
                          const void* field, double* out);

/* ------------------------------------------------------------- adjoint ------ */

/* Reverse sweep of the last apm_solve on this context (same dtype, npart, x, y, z, m
 * pointers and gas pointers of every level, with unchanged contents; APM_ERR_STATE
 * otherwise): the gradient of
 *     L = wbar W + sum_p abar_p . a_p + sum_p phibar_p Phi_p
 * (W as in apm_solve_totals, a and Phi the solve's outputs) with respect to the
 * particle positions, masses and the gas.  Each forward step is transposed in
 * reverse order: the TSC interpolation (its weights' derivatives give the position
 * terms), the level composition (Sec. 2.2, trilinear prolongation), each grid's
 * convolution (Eq. 2 with Fourier-space differencing; the transposed kernel has
 * multipliers +i d_i Gf and Gp), the deposit (Sec. 2).  Owner grids are held fixed.
 * The transposes are linear, so nothing of the forward spectra is kept: the reverse
 * sweep reads the forward composed fields and tile-sorted particles that apm_solve
 * leaves in the context.  Field, GMF and gas cotangents accumulate in FP64 for both
 * dtypes; each particle's per-level terms are rounded to dtype before their FP64 sum.
 * gas: as passed to apm_solve.  pot: the solve's potentials (needed if wbar != 0).
 * abar_x/y/z, phibar: npart values each, or NULL for zero.
 * xbar, ybar, zbar, mbar: npart outputs (any may be NULL).  gas_bar: NULL or host
 * array of nlevels device pointers, a packed active-gas cotangent of a level for
 * each level with gas (NULL entries skipped).  Asynchronous.
 * Periodic plans: the root's transposes wrap like its stencils, and the average
 * density's cotangent (minus the sum of the subgrids' GMF cotangents) is added to
 * the mass cotangent of every in-domain particle and, times dx_0^3, to the root's
 * gas cotangent. */
apm_status apm_solve_adjoint(apm_ctx ctx, apm_dtype dtype, const void* x, const void* y,
                             const void* z, const void* m, int64_t npart, const void* const* gas,
                             const void* pot, const void* abar_x, const void* abar_y,
                             const void* abar_z, const void* phibar, double wbar, void* xbar,
                             void* ybar, void* zbar, void* mbar, void* const* gas_bar);

/* ------------------------------------------------------ time integration ---- */

/* Leapfrog pieces (Sec. 2 time-centring; every level on one step, no subcycling,
 * Sec. 3.1, 3.5).  apm_kick: v += h a.  apm_drift: x += h v, then, for periodic
 * plans, x - floor(x) (a value that rounds to 1 becomes 0).  Arrays are npart
 * device values of `dtype`, updated in place; asynchronous. */
apm_status apm_kick(apm_ctx ctx, apm_dtype dtype, int64_t npart, void* vx, void* vy, void* vz,
                    const void* ax, const void* ay, const void* az, double h);
apm_status apm_drift(apm_ctx ctx, apm_dtype dtype, int64_t npart, void* x, void* y, void* z,
                     const void* vx, const void* vy, const void* vz, double h);

/* Kinetic energy 1/2 sum_p m_p |v_p|^2 in FP64 into *out; synchronises. */
apm_status apm_kinetic_energy(apm_ctx ctx, apm_dtype dtype, const void* m, const void* vx,
                              const void* vy, const void* vz, int64_t npart, double* out);

/* nsteps kick-drift-kick steps of size h: an initial apm_solve at x, then per step
 * v += (h/2) a; x += h v; apm_solve; v += (h/2) a.  x..vz are updated in place; on
 * return ax, ay, az, pot hold the accelerations and potentials at the final
 * positions (pot may be NULL: a library buffer is used).  gas as in apm_solve,
 * held fixed.  energy (host, NULL or nsteps + 1 values) receives the total energy
 * K + W after the initial solve and after every step, W as in apm_solve_totals.
 * Synchronises once at the end. */
apm_status apm_leapfrog(apm_ctx ctx, apm_dtype dtype, void* x, void* y, void* z, void* vx,
                        void* vy, void* vz, const void* m, int64_t npart, const void* const* gas,
                        double h, int32_t nsteps, void* ax, void* ay, void* az, void* pot,
                        double* energy);

/* Subcycled evolution (Sec. 2: levels advance with their own steps, Eq. 10 taken
 * with equality, dt_l = h0 / 2^l; Sec. 3.1 and 3.5 evolve the self-force and orbit
 * tests this way).  nroot root steps of h0; the levels step recursively (a step of
 * level l, then two of level l + 1, and so on).  A step of size h on level l, from
 * its clock t_l: (i) each particle of level l or finer joins level max(l, level of
 * its owner grid); (ii) every particle is deposited at x + v (t_l + h/2 - t_own),
 * its position predicted to the mid-step time from its own level's clock (the
 * time-centred density of Sec. 2); the level's grids are solved and each adds its
 * parent's composed field taken linearly in time through the parent's two latest
 * solves to this mid-step time (the parent's latest alone before it has solved
 * twice); (iii) the level's own particles move about the predicted position:
 * v += h a, x = x_mid + v h/2, a interpolated from the finest grid of level <= l
 * holding x_mid (zero outside the domain).  With one level the step is a
 * drift-kick-drift leapfrog.  x..vz are updated in place; gas as in apm_solve,
 * held fixed.  energy (host, NULL or nroot + 1 values) receives K + W (W as in
 * apm_solve_totals) from a solve at the synchronised positions before the first
 * and after every root step.  Isolated root only (APM_ERR_UNSUPPORTED otherwise);
 * replaces the state an apm_solve_adjoint would read.  Synchronises at the end. */
apm_status apm_evolve_subcycled(apm_ctx ctx, apm_dtype dtype, void* x, void* y, void* z,
                                void* vx, void* vy, void* vz, const void* m, int64_t npart,
                                const void* const* gas, double h0, int32_t nroot,
                                double* energy);

/* Device pointer to the library-owned composed field (or GMF) of `level` written
 * by the last apm_solve; NULL on error. */
const void* apm_field_ptr(apm_ctx ctx, apm_dtype dtype, int32_t level);
const void* apm_gmf_ptr(apm_ctx ctx, apm_dtype dtype, int32_t level);

/* ------------------------------------------- batching, graphs, autotuning ---- */

/* apm_solve runs each transform pass as one launch per FFT length over all grids
 * of all levels (uneven, non-cubic grids share a launch through a job table) and,
 * unless disabled here, records its whole launch sequence in a hipGraph on the
 * second call with identical arguments and library buffers, replaying the graph
 * on the context's stream afterwards.  A change of any argument pointer, of npart
 * or a library reallocation drops the graph.  enable = 0 keeps every call eager. */
apm_status apm_set_graph(apm_ctx ctx, int32_t enable);

/* Autotuner: for every (transform pass, FFT length) of the plan in `dtype`, times
 * the candidate launch shapes (lines per block) over `reps` launches on the job
 * tables and buffers of the last apm_solve of that dtype and keeps the fastest for
 * later calls.  FFT sizes themselves are part of the numeric contract and are not
 * tuned.  The choices and timings (microseconds per launch) are written as a JSON
 * object to `report` (cap bytes, NUL-terminated, may be NULL).  Synchronises.
 * The trial launches overwrite the library-owned level fields, so
 * apm_solve_adjoint, the gas term of apm_solve_totals and apm_field_ptr's contents
 * need a new apm_solve after this call (the first two return APM_ERR_STATE until
 * then).  Errors: APM_ERR_STATE if no apm_solve of this dtype ran yet. */
apm_status apm_autotune(apm_ctx ctx, apm_dtype dtype, int32_t reps, char* report, int32_t cap);

/* ------------------------------------------------------- kernel timing ------ */

/* Measurement support: while enabled (enable != 0), every kernel launch of the
 * compute calls is bracketed by HIP events recorded on the context's stream, and
 * the elapsed times are accumulated per kernel name (e.g. "fft_z_conv",
 * "deposit").  Enabling clears previous totals; disabling keeps them for reading.
 * The events add a few microseconds per launch, so leave it off for timing whole
 * steps. */
apm_status apm_profile(apm_ctx ctx, int32_t enable);
/* Number of kernel names with accumulated time (waits for pending events); -1 on
 * error. */
int32_t apm_profile_count(apm_ctx ctx);
/* Name (NUL-terminated, truncated to cap bytes), total milliseconds and launch
 * count of the i-th kernel name, i < apm_profile_count. */
apm_status apm_profile_entry(apm_ctx ctx, int32_t i, char* name, int32_t cap, double* total_ms,
                             int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* APM_H */
