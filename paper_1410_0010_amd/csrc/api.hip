// C ABI of the device side: context, workspace, cached Green's functions and the
// hot-path entry points declared in include/apm.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "apm_kernels.hpp"

using namespace apm;

// Fixed scratch of apm_totals_noalloc: the FP64 reduction partials, one row of
// kMaxParts per quantity (a level's mass, then W_p and sum m a), for callers that
// cannot allocate.  Each device holds its own copy for the life of the process; host
// code reaches it only through the per-device address taken in apm_create.
constexpr int64_t kNoAllocScratch = (int64_t)(apm::kMaxLevels + 4) * apm::kMaxParts;
static __device__ __align__(256) double scratch[kNoAllocScratch];

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

constexpr double kPiD = 3.14159265358979323846;

}  // namespace

struct apm_ctx_s {
  Plan plan;
  int device = 0;
  hipStream_t stream = nullptr;
  size_t used = 0;
  GridDesc* d_grids = nullptr;
  std::vector<int64_t*> d_dep_begin, d_cmp_begin, d_act_begin;     // per level: first block
  std::vector<int64_t> dep_blocks, cmp_blocks, act_blocks;         // of each grid, and total
  OwnerLevel* d_owner_map = nullptr;                               // owner lookup per level
  std::vector<int64_t*> d_foot_begin;                              // restriction footprints
  std::vector<int64_t> foot_blocks;
  // reverse sweep: FP64 field and gas cotangents per level, GMF cotangents by dtype,
  // FP64 per-particle accumulators; the forward state it needs is the last apm_solve's
  std::vector<DevBuf> adj_fbar, adj_gas, adj_gmf[3];
  DevBuf adj_pacc;
  std::vector<uintptr_t> last_solve;                               // (dtype, n, x, y, z, m,
                                                                  // gas pointer per level)
  // periodic plans: the average density (partials, then the value at kMaxParts and the
  // reverse sweep's cotangent of it at kMaxParts + 1), set by a level-0 deposit or a
  // solve; allocated once, so job tables may hold it
  DevBuf meanbuf;
  bool mean_set = false;
  std::map<std::pair<int, int>, void*> tw;                        // (dtype, L)
  std::map<std::tuple<int, int, int>, void*> dsym;                // (dtype, level, M)
  std::map<std::tuple<int, int, int, int, int>, void*> kern;      // (dtype, level, Mx, My, Mz)
  std::vector<void*> owned;                                       // every table allocation
  DevBuf spec, zbuf, ybuf, pres, owner, totals, gpart, energy, lf_pot;
  // the particle sort shared by the levels: ping-pong keys and indices, packed input
  // records, digit counts and scan partials, the sorted records and references
  DevBuf skey[2], sidx[2], sprec, shist, shsum, ssorted, ssref;
  // subcycled evolution: level of each particle, predicted positions, accelerations
  // of the synchronised solves, and two composed fields per level (latest, previous)
  DevBuf sc_lev, sc_pred, sc_acc;
  std::vector<DevBuf> sc_fld[3];
  int sort_nbits = 0;                                             // of the last sort
  // per level: tile runs, work items, scan sums, FP64 mass grid
  struct LevelBufs { DevBuf tbegin, tend, items, work, bsum, accum; };
  std::vector<LevelBufs> lvb;
  std::vector<DepLevel> dep_host;                                 // level table, host copy
  std::vector<unsigned char> dep_dev_copy;                        // bytes last uploaded
  DevBuf dep_tab;                                                 // level table, device
  std::vector<DevBuf> gmf[3], fld[3];                             // solve-owned, by dtype
  size_t spec_elems = 0, z_elems = 0, y_elems = 0;               // complex elements (sum)
  std::vector<int64_t> spec_off, z_off, y_off;                    // per grid
  struct JobList { ConvJob* d = nullptr; int n = 0; int64_t blocks = 0; };
  // (dtype, pass, L, level or -1, lines per block) -> jobs
  std::map<std::tuple<int, int, int, int, int>, JobList> jobs;
  std::map<std::tuple<int, int, int>, int> lines;                 // autotuned (dtype, pass, L)
  std::string tune_report;
  // hipGraph of apm_solve: captured on the second identical call, replayed after
  uint64_t epoch = 0;                                             // bumps on reallocation
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  // second branch of the solve: the subgrid levels' transforms run beside the root's
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<uintptr_t> gkey;
  uint64_t gkey_epoch = ~0ull;
  int gkey_seen = 0;
  hipGraphExec_t gexec = nullptr;
  // kernel timing: events around every launch while enabled
  struct Mark { std::string name; hipEvent_t a, b; };
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  hipEvent_t ev_open = nullptr;
  std::vector<Mark> marks;
  std::vector<std::string> prof_names;
  std::map<std::string, std::pair<double, int64_t>> prof_acc;
};

namespace {

std::mutex& device_setup_mutex() {
  static std::mutex m;
  return m;
}
std::vector<int>& setup_done() {                    // devices set up (under the mutex)
  static std::vector<int> v;
  return v;
}
std::map<int, double*>& scratch_ptrs() {            // device -> address of `scratch`
  static std::map<int, double*> v;
  return v;
}

apm_status hip_fail(hipError_t e, const char* where) {
  std::ostringstream s;
  s << where << ": " << hipGetErrorString(e);
  return fail(APM_ERR_DEVICE, s.str());
}

#define HIP_TRY(expr, where)                       \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

#define APM_TRY(expr)                  \
  do {                                 \
    apm_status _s = (expr);            \
    if (_s != APM_OK) return _s;       \
  } while (0)

apm_status dev_alloc(apm_ctx c, void** p, size_t bytes, const char* what) {
  if (c->plan.cfg.workspace_limit > 0 && c->used + bytes > (size_t)c->plan.cfg.workspace_limit) {
    std::ostringstream s;
    s << what << ": workspace limit " << c->plan.cfg.workspace_limit << " B exceeded";
    return fail(APM_ERR_OOM, s.str());
  }
  hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    std::ostringstream s;
    s << what << ": hipMalloc(" << bytes << ") failed: " << hipGetErrorString(e);
    return fail(APM_ERR_OOM, s.str());
  }
  c->used += bytes;
  return APM_OK;
}

apm_status ensure(apm_ctx c, DevBuf& b, size_t bytes, const char* what) {
  if (b.p && b.bytes >= bytes) return APM_OK;
  if (b.p) {
    HIP_TRY(hipStreamSynchronize(c->stream), "ensure: sync");
    HIP_TRY(hipFree(b.p), "ensure: free");
    c->used -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  APM_TRY(dev_alloc(c, &b.p, bytes, what));
  b.bytes = bytes;
  c->epoch++;
  return APM_OK;
}

apm_status upload(apm_ctx c, void** dst, const void* src, size_t bytes, const char* what) {
  c->epoch++;
  APM_TRY(dev_alloc(c, dst, bytes, what));
  c->owned.push_back(*dst);
  HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), what);
  return APM_OK;
}

size_t esize(apm_dtype t) { return t == APM_F32 ? 4 : 8; }

apm_status check_dtype(apm_dtype t) {
  if (t != APM_F32 && t != APM_F64) return fail(APM_ERR_INVALID, "dtype must be APM_F32 or APM_F64");
  return APM_OK;
}

apm_status check_ctx(apm_ctx c) {
  if (!c) return fail(APM_ERR_INVALID, "NULL context");
  HIP_TRY(hipSetDevice(c->device), "hipSetDevice");
  return APM_OK;
}

apm_status check_level(apm_ctx c, int32_t level) {
  if (level < 0 || level >= (int32_t)c->plan.levels.size())
    return fail(APM_ERR_INVALID, "level out of range");
  return APM_OK;
}

hipEvent_t next_event(apm_ctx c) {
  if (c->ev_next == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_next++];
}

void prof_hook(void* user, const char* name, int phase) {
  apm_ctx c = (apm_ctx)user;
  if (!c->prof_on) return;
  hipEvent_t e = next_event(c);
  if (!e) return;
  (void)hipEventRecord(e, c->stream);
  if (phase == 0) {
    c->ev_open = e;
  } else if (c->ev_open) {
    c->marks.push_back({name, c->ev_open, e});
    c->ev_open = nullptr;
  }
}

LaunchHook hook_of(apm_ctx c) {
  LaunchHook h;
  if (c->prof_on) { h.fn = prof_hook; h.user = c; }
  return h;
}

// time one launcher call under `name`
template <typename F>
hipError_t timed(apm_ctx c, const char* name, F&& f) {
  LaunchHook h = hook_of(c);
  h(name, 0);
  hipError_t e = f();
  h(name, 1);
  return e;
}

apm_status prof_collect(apm_ctx c) {
  for (auto& m : c->marks) {
    HIP_TRY(hipEventSynchronize(m.b), "profile sync");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, m.a, m.b), "profile elapsed");
    auto& a = c->prof_acc[m.name];
    a.first += ms;
    a.second += 1;
  }
  c->marks.clear();
  c->ev_next = 0;
  c->prof_names.clear();
  for (auto& kv : c->prof_acc) c->prof_names.push_back(kv.first);
  return APM_OK;
}

// twiddles exp(-2 pi i q / L), q < L, computed in FP64 on the host
template <typename T>
apm_status twiddles(apm_ctx c, int L, const void** out) {
  auto key = std::make_pair((int)sizeof(T), L);
  auto it = c->tw.find(key);
  if (it != c->tw.end()) { *out = it->second; return APM_OK; }
  std::vector<C2<T>> h(L);
  for (int q = 0; q < L; ++q) {
    const double a = -2.0 * kPiD * (double)q / (double)L;
    h[q].x = (T)std::cos(a);
    h[q].y = (T)std::sin(a);
  }
  void* d = nullptr;
  APM_TRY(upload(c, &d, h.data(), sizeof(C2<T>) * L, "twiddles"));
  c->tw[key] = d;
  *out = d;
  return APM_OK;
}

// gradient symbols d(m), m in [0, M): k or sin(k dx)/dx for signed m, 0 at M/2
template <typename T>
apm_status grad_symbols(apm_ctx c, int level, int M, double dx, const T** out) {
  auto key = std::make_tuple((int)sizeof(T), level, M);
  auto it = c->dsym.find(key);
  if (it != c->dsym.end()) { *out = (const T*)it->second; return APM_OK; }
  std::vector<T> h(M);
  for (int m = 0; m < M; ++m) {
    const int ms = m > M / 2 ? m - M : m;
    const double k = 2.0 * kPiD * (double)ms / ((double)M * dx);
    double d = c->plan.cfg.gradient == APM_GRAD_FD2 ? std::sin(k * dx) / dx : k;
    if (2 * m == M) d = 0.0;
    h[m] = (T)d;
  }
  void* d = nullptr;
  APM_TRY(upload(c, &d, h.data(), sizeof(T) * M, "gradient symbols"));
  c->dsym[key] = d;
  *out = (const T*)d;
  return APM_OK;
}

// One kernel for force and potential (the spectral gradient: the potential is taken
// with Eq. 5's kernel itself); with the two-point gradient the tables hold pairs.
bool single_kernel(apm_ctx c) { return c->plan.cfg.gradient != APM_GRAD_FD2; }
int y_lines(apm_ctx c) { return single_kernel(c) ? 3 : 4; }   // y inverse lines per column

// Octant table of a grid shape in the working precision, scaled by 1/(Mx My Mz):
// (Gf, Gp) pairs, or Gf alone with one kernel.  Generated once as FP64 pairs (cached);
// the working table is derived from those.
apm_status kernel_table(apm_ctx c, apm_dtype dt, const GridDesc& g, const void** out) {
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  const bool single = single_kernel(c);
  auto k64 = std::make_tuple(8, g.level, Mx, My, Mz);                   // FP64 pairs
  auto kw = std::make_tuple((dt == APM_F32 ? 4 : 8) + (single ? 1 : 0), g.level, Mx, My, Mz);
  {
    auto it = c->kern.find(kw);
    if (it != c->kern.end()) { *out = it->second; return APM_OK; }
  }
  auto it64 = c->kern.find(k64);
  const int64_t oct = (int64_t)(Mx / 2 + 1) * (My / 2 + 1) * (Mz / 2 + 1);
  double2* t64 = nullptr;
  if (it64 != c->kern.end()) {
    t64 = (double2*)it64->second;
  } else {
    void* p = nullptr;
    APM_TRY(dev_alloc(c, &p, sizeof(double2) * oct, "green's function table"));
    c->owned.push_back(p);
    t64 = (double2*)p;
    const Plan& P = c->plan;
    InfluenceParams ip{};
    ip.Mx = Mx; ip.My = My; ip.Mz = Mz;
    ip.dx = g.dx;
    ip.a_l = P.cfg.a_cells * g.dx;
    ip.a_lm1 = g.level == 0 ? -1.0 : P.cfg.a_cells * g.dx * 2.0;
    ip.G = P.cfg.G;
    ip.norm = 1.0 / ((double)Mx * My * Mz);
    ip.bz = P.cfg.brillouin;
    ip.grad = P.cfg.gradient;
    ip.james = nullptr;
    void *b0 = nullptr, *b1 = nullptr, *ct = nullptr;
    const bool james = g.level == 0 && P.cfg.boundary == APM_BC_ISOLATED;
    if (james) {
      const int N = P.cfg.root_n;
      const size_t on = (size_t)(N + 1) * (N + 1) * (N + 1);
      std::vector<double> cosv(2 * N);
      for (int q = 0; q < 2 * N; ++q) cosv[q] = std::cos(kPiD * (double)q / (double)N);
      APM_TRY(dev_alloc(c, &b0, on * 8, "james buffer"));
      APM_TRY(dev_alloc(c, &b1, on * 8, "james buffer"));
      APM_TRY(dev_alloc(c, &ct, cosv.size() * 8, "cos table"));
      HIP_TRY(hipMemcpy(ct, cosv.data(), cosv.size() * 8, hipMemcpyHostToDevice), "cos table");
      double* res = nullptr;
      HIP_TRY(launch_james(N, g.dx, ip.a_l, P.cfg.G, (const double*)ct, (double*)b0, (double*)b1,
                           &res, c->stream), "james kernel");
      ip.james = res;
    }
    HIP_TRY(launch_influence(ip, t64, c->stream), "influence kernel");
    if (james) {
      HIP_TRY(hipStreamSynchronize(c->stream), "james sync");
      for (void* q : {b0, b1, ct}) {
        (void)hipFree(q);
      }
      c->used -= ((size_t)(P.cfg.root_n + 1) * (P.cfg.root_n + 1) * (P.cfg.root_n + 1) * 16 +
                  (size_t)2 * P.cfg.root_n * 8);
    }
    c->kern[k64] = t64;
  }
  // the working table: the transforms' tiled layout, in the working precision
  const size_t es = dt == APM_F32 ? 4 : 8;
  void* pw = nullptr;
  APM_TRY(dev_alloc(c, &pw, es * (single ? 1 : 2) * (size_t)oct_entries(Mx, My, Mz),
                    "green's function table (working)"));
  c->owned.push_back(pw);
  const double* src = (const double*)t64;
  hipError_t te;
  if (dt == APM_F32)
    te = single ? launch_table_tiles<float, 1>(src, (float*)pw, Mx, My, Mz, 0, c->stream)
                : launch_table_tiles<float, 2>(src, (float*)pw, Mx, My, Mz, 0, c->stream);
  else
    te = single ? launch_table_tiles<double, 1>(src, (double*)pw, Mx, My, Mz, 0, c->stream)
                : launch_table_tiles<double, 2>(src, (double*)pw, Mx, My, Mz, 0, c->stream);
  HIP_TRY(te, "green's function table layout");
  c->kern[kw] = pw;
  *out = pw;
  return APM_OK;
}

int pass_axis(int pass) {
  const int p = mirror_pass(pass);
  return p == PASS_Y_FWD || p == PASS_Y_INV ? 1 : (p == PASS_Z_CONV ? 2 : 0);
}
const char* pass_name(int pass) {
  static const char* n[] = {"fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv",
                            "adj_fft_x",  "adj_fft_y",  "adj_fft_z",  "adj_fft_y_inv",
                            "adj_fft_x_inv", "adj_fft_x",  "adj_fft_y",  "adj_fft_z"};
  return n[pass];
}

template <typename T>
int lines_for(apm_ctx c, int pass, int L) {
  // an adjoint pass takes the tuned value of the forward pass it reverses where its own
  // block holds that many lines (the y transpose keeps four lines per column at once,
  // the forward y inverse pass one at a time), else its default
  auto it = c->lines.find(std::make_tuple((int)sizeof(T), mirror_pass(pass), L));
  if (it == c->lines.end()) return default_lines<T>(pass, L);
  if (pass != mirror_pass(pass) && pass_lds<T>(pass, L, it->second) == 0)   // as launch_adj_pass checks
    return default_lines<T>(pass, L);
  return it->second;
}

// Grids of `level` (or of every level when level < 0).
// level >= 0: that level; kAllLevels: every level; kSubLevels: every level but the root
constexpr int kAllLevels = -1, kSubLevels = -2;
std::vector<int> grid_set(apm_ctx c, int level) {
  std::vector<int> v;
  for (const GridDesc& g : c->plan.grids)
    if (level == kAllLevels || g.level == level || (level == kSubLevels && g.level > 0))
      v.push_back(g.index);
  return v;
}

// Tables every grid of the set needs (Green's functions, gradient symbols,
// twiddles).  Allocates and launches on first use.
template <typename T>
apm_status prepare_tables(apm_ctx c, const std::vector<int>& set) {
  for (int gi : set) {
    const GridDesc& g = c->plan.grids[gi];
    const void* k = nullptr;
    APM_TRY(kernel_table(c, sizeof(T) == 4 ? APM_F32 : APM_F64, g, &k));
    for (int a = 0; a < 3; ++a) {
      const T* d = nullptr;
      const void* t = nullptr;
      APM_TRY(grad_symbols<T>(c, g.level, g.M[a], g.dx, &d));
      APM_TRY(twiddles<T>(c, g.M[a], &t));
    }
  }
  return APM_OK;
}

// Job list of one pass and line length over the grid set (cached).
template <typename T>
apm_status job_list(apm_ctx c, int pass, int L, int level, int nl, const apm_ctx_s::JobList** out) {
  auto key = std::make_tuple((int)sizeof(T), pass, L, level, nl);
  auto it = c->jobs.find(key);
  if (it != c->jobs.end()) { *out = &it->second; return APM_OK; }
  std::vector<ConvJob> v;
  int64_t blocks = 0;
  const apm_dtype dt = sizeof(T) == 4 ? APM_F32 : APM_F64;
  for (int gi : grid_set(c, level)) {
    const GridDesc& g = c->plan.grids[gi];
    if (g.M[pass_axis(pass)] != L) continue;
    ConvJob j{};
    j.blk0 = blocks;
    j.level = g.level;
    for (int a = 0; a < 3; ++a) {
      j.g[a] = g.gmf_n[a];
      j.M[a] = g.M[a];
      j.f[a] = g.fld_n[a];
      j.off[a] = ((g.fld_lo[a] - g.gmf_lo[a]) % g.M[a] + g.M[a]) % g.M[a];
    }
    j.pitch = (g.M[0] / 2 + 1 + kRowAlign - 1) / kRowAlign * kRowAlign;
    j.gmf_off = g.gmf_offset;
    j.fld_off = g.fld_offset;
    j.mean = (c->plan.cfg.boundary == APM_BC_PERIODIC && g.level > 0)
                 ? (const double*)c->meanbuf.p + kMaxParts
                 : nullptr;
    j.spec_off = c->spec_off[gi];
    j.z_off = c->z_off[gi];
    j.y_off = c->y_off[gi];
    APM_TRY(kernel_table(c, dt, g, &j.kern));
    j.kstride = single_kernel(c) ? 1 : 2;
    j.kpot = single_kernel(c) ? 0 : 1;
    for (int a = 0; a < 3; ++a) {
      const T* d = nullptr;
      APM_TRY(grad_symbols<T>(c, g.level, g.M[a], g.dx, &d));
      j.dsym[a] = d;
    }
    blocks += pass_blocks(pass, j.g, j.M, j.f, nl);
    v.push_back(j);
  }
  apm_ctx_s::JobList jl;
  jl.n = (int)v.size();
  jl.blocks = blocks;
  if (!v.empty()) {
    void* d = nullptr;
    APM_TRY(upload(c, &d, v.data(), v.size() * sizeof(ConvJob), "job table"));
    jl.d = (ConvJob*)d;
  }
  c->jobs[key] = jl;
  *out = &c->jobs[key];
  return APM_OK;
}

// Distinct line lengths a pass needs over the set.
std::vector<int> pass_lengths(apm_ctx c, int pass, int level) {
  std::vector<int> Ls;
  for (int gi : grid_set(c, level)) {
    const int L = c->plan.grids[gi].M[pass_axis(pass)];
    if (std::find(Ls.begin(), Ls.end(), L) == Ls.end()) Ls.push_back(L);
  }
  return Ls;
}

// One launch (or a fixed group of launches) on the context's current stream; a list of
// them is one branch of a solve, so two branches can be enqueued interleaved.
using Step = std::function<apm_status()>;

apm_status run_steps(const std::vector<Step>& steps) {
  for (const Step& f : steps) APM_TRY(f());
  return APM_OK;
}

// Own fields of the grid set: the five passes, one launch per (pass, L), as steps.
// Tables, buffers and job lists are resolved here on the host.
template <typename T>
apm_status convolve_steps_t(apm_ctx c, int level, const LevelPtrs<T>& lp, std::vector<Step>& out) {
  const std::vector<int> set = grid_set(c, level);
  APM_TRY(prepare_tables<T>(c, set));
  APM_TRY(ensure(c, c->spec, c->spec_elems * sizeof(C2<T>), "spectrum buffer"));
  APM_TRY(ensure(c, c->zbuf, c->z_elems * sizeof(C2<T>), "z-pass output buffer"));
  APM_TRY(ensure(c, c->ybuf, c->y_elems * sizeof(C2<T>), "y-pass output buffer"));
  for (int pass = PASS_X_FWD; pass <= PASS_X_INV; ++pass) {
    for (int L : pass_lengths(c, pass, level)) {
      const int nl = lines_for<T>(c, pass, L);
      const apm_ctx_s::JobList* jl = nullptr;
      APM_TRY(job_list<T>(c, pass, L, level, nl, &jl));
      const void* tw = nullptr;
      APM_TRY(twiddles<T>(c, L, &tw));
      const ConvJob* jobs = jl->d;
      const int njobs = jl->n;
      const int64_t blocks = jl->blocks;
      const int nc = y_lines(c);
      out.push_back([c, pass, L, nl, nc, jobs, njobs, blocks, lp, tw]() -> apm_status {
        HIP_TRY(timed(c, pass_name(pass), [&] {
                  return launch_pass<T>(pass, L, nl, nc, jobs, njobs, blocks, lp, (C2<T>*)c->spec.p,
                                        (C2<T>*)c->zbuf.p, (C2<T>*)c->ybuf.p, tw, c->stream);
                }), pass_name(pass));
        return APM_OK;
      });
    }
  }
  return APM_OK;
}

template <typename T>
apm_status convolve_t(apm_ctx c, int level, const LevelPtrs<T>& lp) {
  std::vector<Step> steps;
  APM_TRY(convolve_steps_t<T>(c, level, lp, steps));
  return run_steps(steps);
}

// The second stream and the fork / join events of a two-branch solve (created once).
apm_status prepare_branch_stream(apm_ctx c) {
  if (!c->aux_stream)
    HIP_TRY(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking), "second stream");
  if (!c->ev_fork) HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "fork event");
  if (!c->ev_join) HIP_TRY(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "join event");
  return APM_OK;
}

template <typename T>
apm_status solve_level_t(apm_ctx c, int32_t level, const T* gmf, T* field) {
  if (c->plan.cfg.boundary == APM_BC_PERIODIC && level > 0 && !c->mean_set)
    return fail(APM_ERR_STATE, "apm_solve_level: a periodic subgrid level needs the average "
                               "density of a level-0 apm_deposit or an apm_solve first");
  LevelPtrs<T> lp{};
  lp.gmf[level] = gmf;
  lp.fld[level] = (V4<T>*)field;
  return convolve_t<T>(c, level, lp);
}

// Uploads the level table if its bytes changed (buffers moved): the stream is
// drained first so no kernel still reads the old table.
apm_status sync_dep_table(apm_ctx c) {
  const size_t bytes = c->dep_host.size() * sizeof(DepLevel);
  const unsigned char* src = (const unsigned char*)c->dep_host.data();
  if (c->dep_tab.p && c->dep_dev_copy.size() == bytes &&
      std::memcmp(c->dep_dev_copy.data(), src, bytes) == 0)
    return APM_OK;
  APM_TRY(ensure(c, c->dep_tab, bytes, "level table"));
  HIP_TRY(hipStreamSynchronize(c->stream), "level table: sync");
  HIP_TRY(hipMemcpy(c->dep_tab.p, src, bytes, hipMemcpyHostToDevice), "level table upload");
  c->dep_dev_copy.assign(src, src + bytes);
  c->epoch++;
  return APM_OK;
}

// Morton bits of the tiles of level lf: 3 log2(N_lf / kTile), 0 when one tile spans
// the domain (N_lf is a power of two).
int sort_bits(const Plan& P, int lf) {
  const int64_t n = (int64_t)P.cfg.root_n << lf;
  int b = 0;
  while ((n >> (b + 3)) > 1) ++b;
  return 3 * b;
}
// ping-pong slot of the sorted keys
int sort_slot(int nbits) { return sort_passes(nbits) & 1; }

// Buffers and arguments of the particle sort by tiles of level lf; owner (or null: no
// owners) receives every particle's owner grid.
template <typename T>
apm_status sort_prepare_t(apm_ctx c, int lf, const T* x, const T* y, const T* z, const T* m,
                          int64_t npart, int32_t* owner, SortIO<T>* out) {
  const Plan& P = c->plan;
  const int nbits = sort_bits(P, lf);
  if (nbits > kMaxMortonBits)
    return fail(APM_ERR_RANGE, "particle sort: level " + std::to_string(lf) + " has more than "
                               "2^21 tiles of 8 cells per axis");
  const size_t np = (size_t)std::max<int64_t>(npart, 1);
  const size_t ks = sort_key64(nbits) ? 8 : 4;
  for (int k = 0; k < 2; ++k) {
    APM_TRY(ensure(c, c->skey[k], np * ks, "sort keys"));
    APM_TRY(ensure(c, c->sidx[k], np * 4, "sort indices"));
  }
  APM_TRY(ensure(c, c->sprec, np * sizeof(V4<T>), "packed particles"));
  APM_TRY(ensure(c, c->shist, (size_t)sort_hist_elems(npart) * 4, "sort digit counts"));
  APM_TRY(ensure(c, c->shsum, (size_t)std::max<int64_t>(sort_sum_elems(npart), 1) * 4,
                 "sort scan partials"));
  APM_TRY(ensure(c, c->ssorted, np * sizeof(V4<T>), "sorted particles"));
  APM_TRY(ensure(c, c->ssref, np * 8, "sorted particle references"));
  SortIO<T> io{};
  io.x = x; io.y = y; io.z = z; io.m = m;
  io.npart = npart;
  io.cells_f = (double)((int64_t)P.cfg.root_n << lf);
  io.nbits = nbits;
  io.om = owner ? c->d_owner_map : nullptr;
  io.om_nlev = (int32_t)P.levels.size();
  io.owner = owner;
  for (int k = 0; k < 2; ++k) {
    io.key[k] = c->skey[k].p;
    io.idx[k] = (int32_t*)c->sidx[k].p;
  }
  io.prec = c->sprec.p;
  io.hist = (uint32_t*)c->shist.p;
  io.hsum = (uint32_t*)c->shsum.p;
  io.sorted = c->ssorted.p;
  io.sref = (int2*)c->ssref.p;
  c->sort_nbits = nbits;
  *out = io;
  return APM_OK;
}

template <typename T>
apm_status sort_launch_t(apm_ctx c, const SortIO<T>& io) {
  int which = 0;
  HIP_TRY(timed(c, "sort", [&] { return launch_particle_sort<T>(io, &which, c->stream); }),
          "particle sort");
  if (io.npart > 0 && which != sort_slot(io.nbits))
    return fail(APM_ERR_DEVICE, "particle sort: sorted keys in an unexpected buffer");
  return APM_OK;
}

// A deposit batch: its launch arguments, prepared before any of its launches.
template <typename T> struct DepBatch {
  int l0 = 0, nlev = 0;
  DepIO<T> io{};
  int64_t max_elems = 0;
  int32_t max_tiles = 1;
  const void* skey = nullptr;                        // the sorted keys
  int nbits = 0;
};

// Buffers and level-table entries of levels [l0, l0 + nlev), whose tiles are runs of
// the list sorted by tiles of level lf (sort_prepare_t with lf, prepared before); the
// table itself is uploaded by sync_dep_table (once for every batch of a solve).
template <typename T>
apm_status deposit_prepare_t(apm_ctx c, int l0, int nlev, int lf, int64_t npart,
                             const T* const* gas, const T* const* pgas, T* const* gmf,
                             DepBatch<T>* out) {
  const Plan& P = c->plan;
  const int nl = (int)P.levels.size();
  c->lvb.resize(nl);
  if ((int)c->dep_host.size() != nl) {
    c->dep_host.resize(nl);
    std::memset((void*)c->dep_host.data(), 0, nl * sizeof(DepLevel));
  }
  DepIO<T> io{};
  io.npart = npart;
  io.nlev = nlev;
  io.comp = (std::is_same<T, float>::value && P.cfg.deposit_accum == APM_ACC_F32_COMP) ? 1 : 0;
  int64_t max_elems = 0, iblk = 0, fblk = 0;
  for (int b = 0; b < nlev; ++b) {
    const int l = l0 + b;
    const LevelDesc& L = P.levels[l];
    apm_ctx_s::LevelBufs& B = c->lvb[l];
    // the tiles (aligned at multiples of kTile cells) that cover the binning box
    int32_t tlo[3], tn[3];
    int64_t ntiles = 1;
    for (int a = 0; a < 3; ++a) {
      const int32_t lo = L.key_lo[a], hi = L.key_lo[a] + L.key_n[a] - 1;
      tlo[a] = lo >= 0 ? lo / kTile : -((-lo + kTile - 1) / kTile);
      const int32_t thi = hi >= 0 ? hi / kTile : -((-hi + kTile - 1) / kTile);
      tn[a] = thi - tlo[a] + 1;
      ntiles *= tn[a];
    }
    if (ntiles >= ((int64_t)1 << 31))
      return fail(APM_ERR_UNSUPPORTED, "deposit: level " + std::to_string(l) + " has 2^31 tiles or more");
    APM_TRY(ensure(c, B.tbegin, (size_t)ntiles * 4, "tile run starts"));
    APM_TRY(ensure(c, B.tend, (size_t)ntiles * 4, "tile run ends"));
    APM_TRY(ensure(c, B.items, (size_t)(ntiles + 1) * 4, "tile work items"));
    const int64_t nwork = ntiles + (npart + kChunk - 1) / kChunk;    // deposit blocks of the level
    APM_TRY(ensure(c, B.work, (size_t)std::max<int64_t>(nwork, 1) * sizeof(int4), "work table"));
    APM_TRY(ensure(c, B.bsum, (size_t)((ntiles + 255) / 256 + 1) * sizeof(int2), "scan block sums"));
    APM_TRY(ensure(c, B.accum, (size_t)L.key_cells * 8, "fp64 mass grid"));
    DepLevel d;
    std::memset((void*)&d, 0, sizeof d);
    d.inv_dx = 1.0 / L.dx;
    d.dx = L.dx;
    for (int a = 0; a < 3; ++a) {
      d.key_lo[a] = L.key_lo[a];
      d.key_n[a] = L.key_n[a];
      d.tile_lo[a] = tlo[a];
      d.tiles_n[a] = tn[a];
    }
    d.ntiles = (int32_t)ntiles;
    d.shift = 3 * (lf - l);
    d.first = L.first;
    d.ngrids = L.count;
    d.wrap = (l == 0 && P.cfg.boundary == APM_BC_PERIODIC) ? P.cfg.root_n : 0;
    d.key_cells = L.key_cells;
    d.tbegin = (int32_t*)B.tbegin.p;
    d.tend = (int32_t*)B.tend.p;
    d.items = (int32_t*)B.items.p;
    d.work = (int4*)B.work.p;
    d.bsum = (int2*)B.bsum.p;
    d.sref = (const int2*)c->ssref.p;
    d.sorted = c->ssorted.p;
    d.accum = (double*)B.accum.p;
    d.grids = c->d_grids + L.first;
    d.block_begin = c->d_dep_begin[l];
    std::memcpy((void*)&c->dep_host[l], &d, sizeof d);
    max_elems = std::max(max_elems, std::max(ntiles, (int64_t)L.key_cells));
    io.item_blk0[b] = iblk;
    iblk += ntiles + (npart + kChunk - 1) / kChunk;
    io.fin_blk0[b] = fblk;
    fblk += c->dep_blocks[l];
    io.gas[b] = gas ? gas[b] : nullptr;
    io.pgas[b] = pgas ? pgas[b] : nullptr;
    io.gmf[b] = gmf[b];
  }
  io.item_blk0[nlev] = iblk;
  io.fin_blk0[nlev] = fblk;
  out->l0 = l0;
  out->nlev = nlev;
  out->io = io;
  out->max_elems = max_elems;
  out->max_tiles = 1;
  for (int b = 0; b < nlev; ++b) out->max_tiles = std::max(out->max_tiles, c->dep_host[l0 + b].ntiles);
  out->nbits = c->sort_nbits;
  out->skey = c->skey[sort_slot(c->sort_nbits)].p;
  return APM_OK;
}

// TSC deposit of a prepared batch (Sec. 2) as five steps -- clear, tile runs, three
// scan launches, tile deposit, finalize -- on the context's stream at the time each
// step runs, after the particle sort.  The level table must be uploaded
// (sync_dep_table) before the steps are built.
template <typename T>
void deposit_steps_t(apm_ctx c, const DepBatch<T>& d, std::vector<Step>& out) {
  const DepIO<T> io = d.io;
  const int nlev = d.nlev;
  const int64_t max_elems = d.max_elems;
  const int32_t max_tiles = d.max_tiles;
  const void* skey = d.skey;
  const int nbits = d.nbits;
  const DepLevel* tab = (const DepLevel*)c->dep_tab.p + d.l0;
  out.push_back([=]() -> apm_status {
    HIP_TRY(timed(c, "bin_clear", [&] { return launch_dep_clear(tab, nlev, max_elems, c->stream); }),
            "clear");
    return APM_OK;
  });
  out.push_back([=]() -> apm_status {
    HIP_TRY(timed(c, "tile_ranges", [&] {
              return launch_tile_ranges(tab, nlev, skey, nbits, io.npart, c->stream);
            }), "tile runs");
    return APM_OK;
  });
  out.push_back([=]() -> apm_status {
    HIP_TRY(timed(c, "bin_scan", [&] { return launch_bin_scan(tab, nlev, max_tiles, c->stream); }),
            "bin scan");
    return APM_OK;
  });
  out.push_back([=]() -> apm_status {
    HIP_TRY(timed(c, "deposit_tiles", [&] { return launch_deposit_tiles<T>(io, tab, c->stream); }),
            "deposit tiles");
    return APM_OK;
  });
  out.push_back([=]() -> apm_status {
    HIP_TRY(timed(c, "deposit_finalize", [&] {
              return launch_deposit_finalize<T>(io, tab, c->stream);
            }), "deposit finalize");
    return APM_OK;
  });
}

template <typename T>
apm_status deposit_launch_t(apm_ctx c, const DepBatch<T>& d) {
  std::vector<Step> steps;
  deposit_steps_t<T>(c, d, steps);
  return run_steps(steps);
}

// Particle sort by tiles of level lf (the batch's finest level by default) and TSC
// deposit of levels [l0, l0 + nlev) in one batch.  gas/pgas/gmf are indexed by batch
// position; owner (or null) receives the owner grids.
template <typename T>
apm_status deposit_levels_t(apm_ctx c, int l0, int nlev, const T* x, const T* y, const T* z,
                            const T* m, int64_t npart, int32_t* owner, const T* const* gas,
                            const T* const* pgas, T* const* gmf, int lf = -1) {
  if (lf < l0 + nlev - 1) lf = l0 + nlev - 1;        // the sort's finest level
  SortIO<T> so{};
  APM_TRY(sort_prepare_t<T>(c, lf, x, y, z, m, npart, owner, &so));
  DepBatch<T> d;
  APM_TRY(deposit_prepare_t<T>(c, l0, nlev, lf, npart, gas, pgas, gmf, &d));
  APM_TRY(sync_dep_table(c));
  APM_TRY(sort_launch_t<T>(c, so));
  return deposit_launch_t<T>(c, d);
}

template <typename T>
__global__ void k_fill_t(T* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

template <typename T>
apm_status zero_t(apm_ctx c, T* p, int64_t n) {
  if (!p || n == 0) return APM_OK;
  hipLaunchKernelGGL((k_fill_t<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, p, n);
  HIP_TRY(hipGetLastError(), "zero fill");
  return APM_OK;
}

// Average density of a periodic system from the particles and the root gas into the
// context's scalar (read by the subgrids' forward x pass).
template <typename T>
apm_status mean_density_t(apm_ctx c, const T* x, const T* y, const T* z, const T* m,
                          int64_t npart, const T* root_gas) {
  const int64_t N = c->plan.cfg.root_n;
  const double dx = c->plan.grids[0].dx;
  double* mb = (double*)c->meanbuf.p;
  HIP_TRY(timed(c, "mean_density", [&] {
            return launch_mean_density<T>(x, y, z, m, npart, root_gas, N * N * N, dx * dx * dx, mb,
                                          mb + kMaxParts, c->stream);
          }), "mean density");
  c->mean_set = true;
  return APM_OK;
}

template <typename T>
apm_status solve_body_t(apm_ctx c, apm_dtype dt, const T* x, const T* y, const T* z, const T* m,
                        int64_t npart, const void* const* gas, T* ax, T* ay, T* az, T* pot) {
  const Plan& P = c->plan;
  const int nl = (int)P.levels.size();
  const int di = (int)dt;
  c->gmf[di].resize(nl);
  c->fld[di].resize(nl);
  for (int l = 0; l < nl; ++l) {
    APM_TRY(ensure(c, c->gmf[di][l], (size_t)P.levels[l].gmf_elems * sizeof(T), "level gmf"));
    APM_TRY(ensure(c, c->fld[di][l], (size_t)P.levels[l].fld_cells * sizeof(V4<T>), "level field"));
  }
  APM_TRY(ensure(c, c->owner, (size_t)std::max<int64_t>(npart, 1) * 4, "owner"));
  int32_t* own = (int32_t*)c->owner.p;
  // owner grids: found by the particle sort
  if (P.cfg.boundary == APM_BC_PERIODIC) APM_TRY(mean_density_t<T>(c, x, y, z, m, npart,
                                                                   gas ? (const T*)gas[0] : nullptr));
  {
    const T* gl[kMaxLevels];
    const T* pg[kMaxLevels];
    T* gm[kMaxLevels];
    for (int l = 0; l < nl; ++l) {
      gl[l] = gas ? (const T*)gas[l] : nullptr;
      pg[l] = (gas && l > 0) ? (const T*)gas[l - 1] : nullptr;
      gm[l] = (T*)c->gmf[di][l].p;
    }
    // each grid's own field is written straight into the level field, then the
    // parent's composed field is added in place, level by level (the root has none)
    LevelPtrs<T> lp{};
    for (int l = 0; l < nl; ++l) {
      lp.gmf[l] = (const T*)c->gmf[di][l].p;
      lp.fld[l] = (V4<T>*)c->fld[di][l].p;
    }
    if (c->prof_on || nl < 2) {                      // one stream (kernels timed one by one)
      APM_TRY(deposit_levels_t<T>(c, 0, nl, x, y, z, m, npart, own, gl, pg, gm));
      APM_TRY(convolve_t<T>(c, kAllLevels, lp));
    } else {
      // One particle sort for every level; then the root's deposit and transforms, and
      // those of the subgrid levels, touch disjoint buffers until the composition: the
      // subgrid levels run on a second stream, forked from and joined back to the
      // context's stream (two branches of the captured graph).
      SortIO<T> so{};
      APM_TRY(sort_prepare_t<T>(c, nl - 1, x, y, z, m, npart, own, &so));
      DepBatch<T> d0, d1;
      APM_TRY(deposit_prepare_t<T>(c, 0, 1, nl - 1, npart, gl, pg, gm, &d0));
      APM_TRY(deposit_prepare_t<T>(c, 1, nl - 1, nl - 1, npart, gl + 1, pg + 1, gm + 1, &d1));
      APM_TRY(sync_dep_table(c));
      APM_TRY(prepare_branch_stream(c));
      APM_TRY(sort_launch_t<T>(c, so));
      std::vector<Step> root, sub;
      deposit_steps_t<T>(c, d0, root);
      APM_TRY(convolve_steps_t<T>(c, 0, lp, root));
      deposit_steps_t<T>(c, d1, sub);
      APM_TRY(convolve_steps_t<T>(c, kSubLevels, lp, sub));
      HIP_TRY(hipEventRecord(c->ev_fork, c->stream), "fork record");
      HIP_TRY(hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0), "fork wait");
      // the two branches' launches are enqueued (and captured) alternately, so both
      // branches start at once
      hipStream_t main = c->stream;
      apm_status st = APM_OK;
      for (size_t i = 0; st == APM_OK && i < std::max(root.size(), sub.size()); ++i) {
        if (i < root.size()) {
          c->stream = main;
          st = root[i]();
        }
        if (st == APM_OK && i < sub.size()) {
          c->stream = c->aux_stream;
          st = sub[i]();
        }
      }
      c->stream = main;
      // join in every case, so a capture never ends with the branch left open
      HIP_TRY(hipEventRecord(c->ev_join, c->aux_stream), "join record");
      HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_join, 0), "join wait");
      APM_TRY(st);
    }
  }
  for (int l = 1; l < nl; ++l) {
    const LevelDesc& L = P.levels[l];
    HIP_TRY(timed(c, "compose", [&] {
              return launch_compose<T>(c->d_grids + L.first, c->d_cmp_begin[l], L.count,
                                       (const V4<T>*)c->fld[di][l].p,
                                       (const V4<T>*)c->fld[di][l - 1].p,
                                       (V4<T>*)c->fld[di][l].p, c->cmp_blocks[l], c->stream);
            }), "compose");
  }
  InterpIO<T> io{};
  io.nlev = nl;
  for (int l = 0; l < nl; ++l) io.fld[l] = (const V4<T>*)c->fld[di][l].p;
  int64_t iblk = 0;                                  // one block per deposit work item
  for (int l = 0; l < nl; ++l) {
    io.item_blk0[l] = iblk;
    iblk += (int64_t)c->dep_host[l].ntiles + (npart + kChunk - 1) / kChunk;
  }
  io.item_blk0[nl] = iblk;
  // one record per particle, written by its owner level's interpolation
  APM_TRY(ensure(c, c->pres, (size_t)std::max<int64_t>(npart, 1) * sizeof(V4<T>), "particle results"));
  io.res = (V4<T>*)c->pres.p;
  HIP_TRY(timed(c, "interp", [&] {
            return launch_interp_tiles<T>(io, (const DepLevel*)c->dep_tab.p, c->d_grids, c->stream);
          }), "interp");
  HIP_TRY(timed(c, "unpack", [&] {
            return launch_unpack<T>(io, (const DepLevel*)c->dep_tab.p, own, npart, ax, ay, az, pot,
                                    c->stream);
          }), "unpack");
  return APM_OK;
}

// What the library-owned state of a solve belongs to: the particles and, since the
// composed fields depend on it, the gas of every level.
std::vector<uintptr_t> solve_key(apm_ctx c, apm_dtype dt, int64_t n, const void* x, const void* y,
                                 const void* z, const void* m, const void* const* gas) {
  std::vector<uintptr_t> k = {(uintptr_t)dt, (uintptr_t)n, (uintptr_t)x, (uintptr_t)y,
                              (uintptr_t)z, (uintptr_t)m};
  for (size_t l = 0; l < c->plan.levels.size(); ++l) k.push_back(gas ? (uintptr_t)gas[l] : 0);
  return k;
}

void drop_graph(apm_ctx c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
}

// apm_solve with graph capture: a call whose arguments and library buffers match
// the previous call is captured once (on an internal stream, since the caller's
// may be the legacy default stream) and replayed on the caller's stream after.
template <typename T>
apm_status solve_graph_t(apm_ctx c, apm_dtype dt, const T* x, const T* y, const T* z, const T* m,
                         int64_t npart, const void* const* gas, T* ax, T* ay, T* az, T* pot);

// The forward solve; records which inputs the library-owned state (sorted particles,
// owners, fields) belongs to, for the reverse sweep.
template <typename T>
apm_status solve_t(apm_ctx c, apm_dtype dt, const T* x, const T* y, const T* z, const T* m,
                   int64_t npart, const void* const* gas, T* ax, T* ay, T* az, T* pot) {
  c->last_solve.clear();
  apm_status st = solve_graph_t<T>(c, dt, x, y, z, m, npart, gas, ax, ay, az, pot);
  if (st == APM_OK) c->last_solve = solve_key(c, dt, npart, x, y, z, m, gas);
  return st;
}

template <typename T>
apm_status solve_graph_t(apm_ctx c, apm_dtype dt, const T* x, const T* y, const T* z, const T* m,
                         int64_t npart, const void* const* gas, T* ax, T* ay, T* az, T* pot) {
  if (!c->use_graph || c->prof_on)
    return solve_body_t<T>(c, dt, x, y, z, m, npart, gas, ax, ay, az, pot);
  std::vector<uintptr_t> key = {(uintptr_t)dt, (uintptr_t)npart, (uintptr_t)x, (uintptr_t)y,
                                (uintptr_t)z, (uintptr_t)m, (uintptr_t)ax, (uintptr_t)ay,
                                (uintptr_t)az, (uintptr_t)pot};
  for (size_t l = 0; l < c->plan.levels.size(); ++l)
    key.push_back(gas ? (uintptr_t)gas[l] : 0);
  if (c->gexec && key == c->gkey && c->epoch == c->gkey_epoch) {
    HIP_TRY(hipGraphLaunch(c->gexec, c->stream), "graph launch");
    return APM_OK;
  }
  if (key == c->gkey && c->epoch == c->gkey_epoch && c->gkey_seen >= 1) {
    drop_graph(c);
    if (!c->cap_stream)
      HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
    // the capture stream must see the caller's prior work: record on the caller's
    // stream, wait on the capture stream before capture begins
    hipStream_t user = c->stream;
    HIP_TRY(hipStreamSynchronize(user), "pre-capture sync");
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    c->stream = c->cap_stream;
    apm_status st = solve_body_t<T>(c, dt, x, y, z, m, npart, gas, ax, ay, az, pot);
    c->stream = user;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != APM_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(e, "end capture"); }
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { c->gexec = nullptr; return hip_fail(e, "graph instantiate"); }
    if (c->epoch != c->gkey_epoch) { drop_graph(c); return fail(APM_ERR_STATE, "allocation during capture"); }
    HIP_TRY(hipGraphLaunch(c->gexec, c->stream), "graph launch");
    return APM_OK;
  }
  drop_graph(c);
  apm_status st = solve_body_t<T>(c, dt, x, y, z, m, npart, gas, ax, ay, az, pot);
  c->gkey = key;
  c->gkey_epoch = c->epoch;
  c->gkey_seen = st == APM_OK ? 1 : 0;
  return st;
}

// Autotuner: lines per block of every (pass, L) of the plan, timed on the real job
// tables and buffers of the last apm_solve of this precision.
template <typename T>
apm_status autotune_t(apm_ctx c, apm_dtype dt, int reps) {
  const int di = (int)dt;
  const int nl = (int)c->plan.levels.size();
  if ((int)c->fld[di].size() != nl || !c->spec.p)
    return fail(APM_ERR_STATE, "apm_autotune: run apm_solve of this precision first");
  HIP_TRY(hipStreamSynchronize(c->stream), "autotune sync");
  LevelPtrs<T> lp{};
  for (int l = 0; l < nl; ++l) {
    lp.gmf[l] = (const T*)c->gmf[di][l].p;
    lp.fld[l] = (V4<T>*)c->fld[di][l].p;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "event");
  HIP_TRY(hipEventCreate(&e1), "event");
  std::ostringstream rep;
  rep << "{";
  bool first = true;
  for (int pass = PASS_X_FWD; pass <= PASS_X_INV; ++pass) {
    for (int L : pass_lengths(c, pass, -1)) {
      const int d0 = default_lines<T>(pass, L);
      const void* tw = nullptr;
      APM_TRY(twiddles<T>(c, L, &tw));
      int best = d0;
      float best_ms = 1e30f;
      std::ostringstream cand;
      for (int nlc : {d0 / 4, d0 / 2, d0, d0 * 2, d0 * 4}) {
        if (pass_lds<T>(pass, L, nlc, y_lines(c)) == 0) continue;
        const apm_ctx_s::JobList* jl = nullptr;
        APM_TRY(job_list<T>(c, pass, L, -1, nlc, &jl));
        HIP_TRY(launch_pass<T>(pass, L, nlc, y_lines(c), jl->d, jl->n, jl->blocks, lp,
                               (C2<T>*)c->spec.p,
                               (C2<T>*)c->zbuf.p, (C2<T>*)c->ybuf.p, tw, c->stream),
                "autotune warm-up");
        HIP_TRY(hipEventRecord(e0, c->stream), "event");
        for (int r = 0; r < reps; ++r)
          HIP_TRY(launch_pass<T>(pass, L, nlc, y_lines(c), jl->d, jl->n, jl->blocks, lp,
                               (C2<T>*)c->spec.p,
                                 (C2<T>*)c->zbuf.p, (C2<T>*)c->ybuf.p, tw, c->stream),
                  "autotune launch");
        HIP_TRY(hipEventRecord(e1, c->stream), "event");
        HIP_TRY(hipEventSynchronize(e1), "event");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "event");
        ms /= reps;
        cand << (cand.tellp() > 0 ? ", " : "") << "\"" << nlc << "\": " << ms * 1e3f;
        if (ms < best_ms) { best_ms = ms; best = nlc; }
      }
      c->lines[std::make_tuple((int)sizeof(T), pass, L)] = best;
      rep << (first ? "" : ", ") << "\"" << pass_name(pass) << "/" << L << "/"
          << (sizeof(T) == 4 ? "f32" : "f64") << "\": {\"lines\": " << best << ", \"us\": {"
          << cand.str() << "}}";
      first = false;
    }
  }
  rep << "}";
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tune_report = rep.str();
  drop_graph(c);
  c->gkey.clear();
  c->last_solve.clear();                            // the trial launches wrote the level fields
  return APM_OK;
}

}  // namespace

// =================================================================== C ABI ==========

// Gas energy of every level with gas into dev[0] (added); partials in c->gpart.
template <typename T>
apm_status gas_energy_levels_t(apm_ctx c, const void* const* gas, const V4<T>* const* fields,
                               double* dev) {
  const Plan& P = c->plan;
  int64_t maxb = 1;
  for (int64_t b : c->act_blocks) maxb = std::max(maxb, b);
  APM_TRY(ensure(c, c->gpart, (size_t)maxb * 8, "gas energy partials"));
  for (size_t l = 0; l < P.levels.size(); ++l) {
    if (!gas || !gas[l]) continue;
    const LevelDesc& L = P.levels[l];
    HIP_TRY(launch_gas_energy<T>(c->d_grids, c->d_owner_map, (int32_t)P.levels.size(), L.first,
                                 L.count, c->d_act_begin[l], c->act_blocks[l], (const T*)gas[l],
                                 fields[l], (double*)c->gpart.p, dev, c->stream),
            "gas energy");
  }
  return APM_OK;
}

// Energy terms of step slot e (6 doubles: K, W_particles, sum m a (3), W_gas) after a
// solve; all on the stream, no synchronisation.
template <typename T>
apm_status step_energy_t(apm_ctx c, apm_dtype dt, const T* m, const T* vx, const T* vy,
                         const T* vz, int64_t n, const T* ax, const T* ay, const T* az,
                         const T* pot, const void* const* gas, double* e) {
  double* part = (double*)c->totals.p + 8;
  HIP_TRY(launch_kinetic<T>(m, vx, vy, vz, n, part, e, c->stream), "leapfrog kinetic");
  HIP_TRY(launch_particle_totals<T>(m, (const int32_t*)c->owner.p, n, ax, ay, az, pot, part, e + 1,
                                    c->stream), "leapfrog particle energy");
  const int nl = (int)c->plan.levels.size();
  std::vector<const V4<T>*> f(nl);
  for (int l = 0; l < nl; ++l) f[l] = (const V4<T>*)c->fld[(int)dt][l].p;
  APM_TRY(gas_energy_levels_t<T>(c, gas, f.data(), e + 5));
  return APM_OK;
}

template <typename T>
apm_status leapfrog_t(apm_ctx c, apm_dtype dt, T* x, T* y, T* z, T* vx, T* vy, T* vz, const T* m,
                      int64_t n, const void* const* gas, double h, int32_t nsteps, T* ax, T* ay,
                      T* az, T* pot, double* energy) {
  const int nl = (int)c->plan.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(nl + 4 + 8 + 4 * kMaxParts) * 8, "totals"));
  if (!pot) {
    APM_TRY(ensure(c, c->lf_pot, (size_t)std::max<int64_t>(n, 1) * sizeof(T), "leapfrog potential"));
    pot = (T*)c->lf_pot.p;
  }
  const size_t ne = energy ? (size_t)(nsteps + 1) * 6 : 0;
  if (energy) {
    APM_TRY(ensure(c, c->energy, ne * 8, "leapfrog energies"));
    HIP_TRY(launch_fill_f64((double*)c->energy.p, (int64_t)ne, 0.0, c->stream), "energy fill");
  }
  double* E = (double*)c->energy.p;
  APM_TRY(solve_t<T>(c, dt, x, y, z, m, n, gas, ax, ay, az, pot));
  if (energy) APM_TRY(step_energy_t<T>(c, dt, m, vx, vy, vz, n, ax, ay, az, pot, gas, E));
  for (int32_t s = 0; s < nsteps; ++s) {
    HIP_TRY(timed(c, "kick_drift", [&] {
              return launch_kick_drift<T>(n, x, y, z, vx, vy, vz, ax, ay, az, 0.5 * h, h,
                                          c->plan.cfg.boundary == APM_BC_PERIODIC, c->stream);
            }), "leapfrog kick-drift");
    APM_TRY(solve_t<T>(c, dt, x, y, z, m, n, gas, ax, ay, az, pot));
    HIP_TRY(timed(c, "kick", [&] {
              return launch_kick_drift<T>(n, nullptr, nullptr, nullptr, vx, vy, vz, ax, ay, az,
                                          0.5 * h, 0.0, 0, c->stream);
            }), "leapfrog kick");
    if (energy)
      APM_TRY(step_energy_t<T>(c, dt, m, vx, vy, vz, n, ax, ay, az, pot, gas, E + 6 * (s + 1)));
  }
  if (energy) {
    std::vector<double> h6(ne);
    HIP_TRY(hipMemcpyAsync(h6.data(), E, ne * 8, hipMemcpyDeviceToHost, c->stream), "energy copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "leapfrog sync");
    for (int32_t s = 0; s <= nsteps; ++s) energy[s] = h6[6 * s] + h6[6 * s + 1] + h6[6 * s + 5];
  } else {
    HIP_TRY(hipStreamSynchronize(c->stream), "leapfrog sync");
  }
  return APM_OK;
}

// Subcycled evolution (see include/apm.h): the levels step recursively, level l with
// h0 / 2^l.  A level step reassigns the particles of its level and finer ones,
// deposits every particle at its position predicted to the mid-step time, solves
// the level's grids, adds the parent's composed field taken linearly in time through
// the parent's two latest solves, and moves the level's own particles about their
// predicted positions.
template <typename T>
apm_status evolve_subcycled_t(apm_ctx c, apm_dtype dt, T* x, T* y, T* z, T* vx, T* vy, T* vz,
                              const T* m, int64_t n, const void* const* gas, double h0,
                              int32_t nroot, double* energy) {
  const Plan& P = c->plan;
  const int nl = (int)P.levels.size();
  const int di = (int)dt;
  if (P.cfg.boundary == APM_BC_PERIODIC)
    return fail(APM_ERR_UNSUPPORTED, "apm_evolve_subcycled: isolated root only");
  const size_t np = (size_t)std::max<int64_t>(n, 1);
  APM_TRY(ensure(c, c->sc_lev, np * 4, "subcycling levels"));
  APM_TRY(ensure(c, c->sc_pred, np * 3 * sizeof(T), "predicted positions"));
  c->gmf[di].resize(nl);
  c->sc_fld[di].resize(2 * nl);
  for (int l = 0; l < nl; ++l) {
    APM_TRY(ensure(c, c->gmf[di][l], (size_t)P.levels[l].gmf_elems * sizeof(T), "level gmf"));
    for (int k = 0; k < 2; ++k)
      APM_TRY(ensure(c, c->sc_fld[di][2 * l + k], (size_t)P.levels[l].fld_cells * sizeof(V4<T>),
                     "subcycling fields"));
  }
  if (energy) {
    APM_TRY(ensure(c, c->sc_acc, np * 3 * sizeof(T), "subcycling accelerations"));
    APM_TRY(ensure(c, c->lf_pot, np * sizeof(T), "leapfrog potential"));
    APM_TRY(ensure(c, c->totals, (size_t)(nl + 4 + 8 + 4 * kMaxParts) * 8, "totals"));
    APM_TRY(ensure(c, c->energy, (size_t)(nroot + 1) * 6 * 8, "energies"));
    HIP_TRY(launch_fill_f64((double*)c->energy.p, (int64_t)(nroot + 1) * 6, 0.0, c->stream),
            "energy fill");
  }
  HIP_TRY(launch_fill_i32((int32_t*)c->sc_lev.p, n, 0, c->stream), "levels fill");
  SubIO<T> io{};
  io.npart = n;
  io.x = x; io.y = y; io.z = z; io.vx = vx; io.vy = vy; io.vz = vz;
  io.xp = (T*)c->sc_pred.p;
  io.yp = io.xp + np;
  io.zp = io.yp + np;
  io.lev = (int32_t*)c->sc_lev.p;
  io.om = c->d_owner_map;
  io.nlev = nl;
  io.grids = c->d_grids;
  std::vector<int> cur(nl, 0), solved(nl, 0);
  std::vector<double> t_cur(nl, 0.0), t_prev(nl, 0.0);
  auto field = [&](int l, int k) { return (V4<T>*)c->sc_fld[di][2 * l + k].p; };
  std::function<apm_status(int, double)> level_step = [&](int l, double h) -> apm_status {
    const LevelDesc& L = P.levels[l];
    io.level = l;
    HIP_TRY(launch_sub_assign<T>(io, c->stream), "subcycling: levels");
    io.tm = io.clock[l] + 0.5 * h;
    io.h = h;
    HIP_TRY(launch_sub_predict<T>(io, c->stream), "subcycling: prediction");
    const T* gl = gas ? (const T*)gas[l] : nullptr;
    const T* pg = (gas && l > 0) ? (const T*)gas[l - 1] : nullptr;
    T* gm = (T*)c->gmf[di][l].p;
    APM_TRY(deposit_levels_t<T>(c, l, 1, io.xp, io.yp, io.zp, m, n, nullptr, &gl, &pg, &gm, nl - 1));
    V4<T>* out = field(l, 1 - cur[l]);                // the older buffer takes the new field
    LevelPtrs<T> lp{};
    lp.gmf[l] = gm;
    lp.fld[l] = out;
    APM_TRY(convolve_t<T>(c, l, lp));
    if (l > 0) {
      const bool two = solved[l - 1] >= 2 && t_cur[l - 1] != t_prev[l - 1];
      const double al = two ? (io.tm - t_prev[l - 1]) / (t_cur[l - 1] - t_prev[l - 1]) : 1.0;
      HIP_TRY(timed(c, "compose", [&] {
                return launch_compose<T>(c->d_grids + L.first, c->d_cmp_begin[l], L.count, out,
                                         field(l - 1, cur[l - 1]), out, c->cmp_blocks[l],
                                         c->stream, two ? field(l - 1, 1 - cur[l - 1]) : nullptr,
                                         al);
              }), "subcycling: composition");
    }
    cur[l] = 1 - cur[l];
    solved[l]++;
    t_prev[l] = t_cur[l];
    t_cur[l] = io.tm;
    for (int k = 0; k <= l; ++k) io.fld[k] = field(k, cur[k]);
    io.level = l;
    io.tm = t_cur[l];
    io.h = h;
    HIP_TRY(launch_sub_move<T>(io, c->stream), "subcycling: move");
    io.clock[l] += h;
    if (l + 1 < nl)
      for (int r = 0; r < 2; ++r) APM_TRY(level_step(l + 1, 0.5 * h));
    return APM_OK;
  };
  double* E = (double*)c->energy.p;
  auto energy_at = [&](int r) -> apm_status {
    T* acc = (T*)c->sc_acc.p;
    T* pot = (T*)c->lf_pot.p;
    APM_TRY(solve_t<T>(c, dt, x, y, z, m, n, gas, acc, acc + np, acc + 2 * np, pot));
    return step_energy_t<T>(c, dt, m, vx, vy, vz, n, acc, acc + np, acc + 2 * np, pot, gas,
                            E + 6 * r);
  };
  if (energy) APM_TRY(energy_at(0));
  for (int32_t r = 0; r < nroot; ++r) {
    APM_TRY(level_step(0, h0));
    if (energy) APM_TRY(energy_at(r + 1));
  }
  if (energy) {
    std::vector<double> h6((size_t)(nroot + 1) * 6);
    HIP_TRY(hipMemcpyAsync(h6.data(), E, h6.size() * 8, hipMemcpyDeviceToHost, c->stream),
            "energy copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "subcycling sync");
    for (int32_t r = 0; r <= nroot; ++r) energy[r] = h6[6 * r] + h6[6 * r + 1] + h6[6 * r + 5];
  } else {
    HIP_TRY(hipStreamSynchronize(c->stream), "subcycling sync");
  }
  return APM_OK;
}

// Reverse sweep of the last apm_solve of this dtype (see include/apm.h).
// Transposed convolution passes of a grid set (see convolve_t).
template <typename T>
apm_status adj_convolve_t(apm_ctx c, int level, const AdjPtrs<T>& ap, bool pot_only) {
  const int seq_full[5] = {PASS_AX, PASS_AY, PASS_AZ, PASS_AYI, PASS_AXI};
  const int seq_pot[5] = {PASS_APX, PASS_APY, PASS_APZ, PASS_AYI, PASS_AXI};
  for (int pass : pot_only ? seq_pot : seq_full) {
    for (int L : pass_lengths(c, pass, level)) {
      const int nlines = lines_for<T>(c, pass, L);
      const apm_ctx_s::JobList* jl = nullptr;
      APM_TRY(job_list<T>(c, pass, L, level, nlines, &jl));
      const void* tw = nullptr;
      APM_TRY(twiddles<T>(c, L, &tw));
      HIP_TRY(timed(c, pass_name(pass), [&] {
                return launch_adj_pass<T>(pass, L, nlines, jl->d, jl->n, jl->blocks, ap,
                                          (C2<T>*)c->spec.p, (C2<T>*)c->zbuf.p, (C2<T>*)c->ybuf.p,
                                          tw, c->stream);
              }), pass_name(pass));
    }
  }
  return APM_OK;
}

// The subgrid levels' transposes on the second stream (as in the forward solve).
template <typename T>
apm_status adj_convolve_branches_t(apm_ctx c, const AdjPtrs<T>& ap, bool pot_only) {
  if (c->prof_on || c->plan.levels.size() < 2) return adj_convolve_t<T>(c, kAllLevels, ap, pot_only);
  APM_TRY(prepare_branch_stream(c));
  HIP_TRY(hipEventRecord(c->ev_fork, c->stream), "fork record");
  HIP_TRY(hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0), "fork wait");
  hipStream_t main = c->stream;
  c->stream = c->aux_stream;
  apm_status st = adj_convolve_t<T>(c, kSubLevels, ap, pot_only);
  c->stream = main;
  if (st == APM_OK) st = adj_convolve_t<T>(c, 0, ap, pot_only);
  HIP_TRY(hipEventRecord(c->ev_join, c->aux_stream), "join record");
  HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_join, 0), "join wait");
  return st;
}

template <typename T>
apm_status adjoint_t(apm_ctx c, apm_dtype dt, const T* x, const T* y, const T* z, const T* m,
                     int64_t n, const void* const* gas, const T* pot, const T* abx, const T* aby,
                     const T* abz, const T* phib, double wbar, T* xb, T* yb, T* zb, T* mb,
                     void* const* gas_bar) {
  const Plan& P = c->plan;
  const int nl = (int)P.levels.size();
  const int di = (int)dt;
  if (c->last_solve != solve_key(c, dt, n, x, y, z, m, gas) || (int)c->fld[di].size() != nl ||
      (int)c->lvb.size() != nl)
    return fail(APM_ERR_STATE, "apm_solve_adjoint: needs the apm_solve of the same particles, "
                               "gas and dtype as the last solve on this context");
  c->adj_fbar.resize(nl);
  c->adj_gas.resize(nl);
  c->adj_gmf[di].resize(nl);
  for (int l = 0; l < nl; ++l) {
    APM_TRY(ensure(c, c->adj_fbar[l], (size_t)P.levels[l].fld_cells * 32, "field cotangents"));
    APM_TRY(ensure(c, c->adj_gmf[di][l], (size_t)P.levels[l].gmf_elems * sizeof(T), "gmf cotangents"));
    if (gas && gas[l])
      APM_TRY(ensure(c, c->adj_gas[l], (size_t)std::max<int64_t>(P.levels[l].gas_elems, 1) * 8,
                     "gas cotangents"));
  }
  // per sorted entry, a 4-vector of T for each level's deposit transpose and one for
  // the interpolation transpose; per particle, the gradient record
  APM_TRY(ensure(c, c->adj_pacc, (size_t)std::max<int64_t>(n, 1) * sizeof(V4<T>) * (nl + 2),
                 "particle cotangents"));
  ZeroList zl{};
  hipError_t zerr = hipSuccess;
  auto add = [&](void* p, int64_t cnt) {            // cleared in batches of up to 48 ranges
    if (zl.count == 48) {
      if (zerr == hipSuccess) zerr = launch_zero_ranges(zl, c->stream);
      zl.count = 0;
    }
    zl.p[zl.count] = (double*)p;
    zl.n[zl.count] = cnt;
    zl.count++;
  };
  AdjIO<T> io{};
  io.nlev = nl;
  io.npart = n;
  io.wbar = wbar;
  io.abx = abx; io.aby = aby; io.abz = abz; io.phib = phib;
  const bool pot_only = !abx && !aby && !abz;       // the Phi cotangent alone flows back
  io.c0 = pot_only ? 3 : 0;
  // field cotangents per cell: all four components, or the Phi one alone, densely
  const int fs = pot_only ? 1 : 4;
  V4<T>* pacc = (V4<T>*)c->adj_pacc.p;
  for (int l = 0; l < nl; ++l) io.plev[l] = pacc + (int64_t)n * l;
  io.pint = pacc + (int64_t)n * nl;
  io.pout = pacc + (int64_t)n * (nl + 1);
  int64_t iblk = 0, fblk = 0;
  for (int l = 0; l < nl; ++l) {
    const DepLevel& d = c->dep_host[l];
    io.item_blk0[l] = iblk;
    iblk += (int64_t)d.ntiles + (n + kChunk - 1) / kChunk;
    io.fin_blk0[l] = fblk;
    fblk += c->dep_blocks[l];
    io.fld[l] = (const V4<T>*)c->fld[di][l].p;
    io.fbar[l] = (double*)c->adj_fbar[l].p;
    io.gmf_bar[l] = (const T*)c->adj_gmf[di][l].p;
    io.gas_bar[l] = (gas && gas[l]) ? (double*)c->adj_gas[l].p : nullptr;
    io.pgas_bar[l] = (l > 0 && gas && gas[l - 1]) ? (double*)c->adj_gas[l - 1].p : nullptr;
    add(io.fbar[l], P.levels[l].fld_cells * fs);
    // the GMF cotangent grid: on a level of one grid, the grid pass writes every cell
    if (P.levels[l].count > 1) add(c->lvb[l].accum.p, P.levels[l].key_cells);
    if (io.gas_bar[l]) add(io.gas_bar[l], P.levels[l].gas_elems);
  }
  io.item_blk0[nl] = iblk;
  io.fin_blk0[nl] = fblk;
  const DepLevel* tab = (const DepLevel*)c->dep_tab.p;
  HIP_TRY(zerr, "adjoint clear");
  HIP_TRY(timed(c, "adj_clear", [&] { return launch_zero_ranges(zl, c->stream); }), "adjoint clear");
  HIP_TRY(timed(c, "adj_interp", [&] { return launch_adj_interp<T>(io, tab, c->d_grids, c->stream); }),
          "interpolation transpose");
  if (wbar != 0.0 && gas) {
    for (int l = 0; l < nl; ++l) {
      if (!gas[l]) continue;
      const LevelDesc& L = P.levels[l];
      HIP_TRY(timed(c, "adj_gas_seed", [&] {
                return launch_adj_gas_seed<T>(c->d_grids, c->d_owner_map, (int32_t)P.levels.size(),
                                              L.first, L.count, c->d_act_begin[l],
                                              c->act_blocks[l], (const T*)gas[l], io.fld[l],
                                              wbar, io.fbar[l], fs, io.gas_bar[l], c->stream);
              }), "gas energy seeds");
    }
  }
  for (int l = nl - 1; l >= 1; --l) {
    const LevelDesc& L = P.levels[l];
    HIP_TRY(timed(c, "adj_restrict", [&] {
              return launch_adj_restrict(c->d_grids, L.first, L.count, c->d_foot_begin[l],
                                         c->foot_blocks[l], io.fbar[l], io.fbar[l - 1], fs,
                                         c->stream);
            }), "composition transpose");
  }
  // transposed convolution of every grid of every level
  const std::vector<int> set = grid_set(c, -1);
  APM_TRY(prepare_tables<T>(c, set));
  APM_TRY(ensure(c, c->spec, c->spec_elems * sizeof(C2<T>), "spectrum buffer"));
  APM_TRY(ensure(c, c->zbuf, c->z_elems * sizeof(C2<T>), "z-pass output buffer"));
  APM_TRY(ensure(c, c->ybuf, c->y_elems * sizeof(C2<T>), "y-pass output buffer"));
  AdjPtrs<T> ap{};
  for (int l = 0; l < nl; ++l) {
    ap.gmf[l] = (T*)c->adj_gmf[di][l].p;
    ap.fbar[l] = io.fbar[l];
  }
  APM_TRY(adj_convolve_branches_t<T>(c, ap, pot_only));
  if (P.cfg.boundary == APM_BC_PERIODIC) {
    // the subgrids convolved GMF - rho_bar: rho_bar's cotangent is minus the sum of
    // their GMF cotangents (the root's kernel is zero at k = 0, so the root's sums to 0)
    double* mb_ = (double*)c->meanbuf.p;
    double* rb = mb_ + kMaxParts + 1;
    HIP_TRY(launch_fill_f64(rb, 1, 0.0, c->stream), "mean cotangent clear");
    for (int l = 1; l < nl; ++l)
      HIP_TRY(timed(c, "adj_mean", [&] {
                return launch_sum_scaled<T>((const T*)c->adj_gmf[di][l].p, P.levels[l].gmf_elems,
                                            -1.0, mb_, rb, c->stream);
              }), "mean cotangent");
    io.rbar = rb;
  }
  HIP_TRY(timed(c, "adj_deposit_grid", [&] { return launch_adj_deposit_grid<T>(io, tab, c->stream); }),
          "deposit transpose (grids)");
  if (io.rbar && io.gas_bar[0]) {
    const double vol = P.levels[0].dx * P.levels[0].dx * P.levels[0].dx;
    HIP_TRY(launch_add_scalar(io.gas_bar[0], P.levels[0].gas_elems, io.rbar, vol, c->stream),
            "root gas: mean cotangent");
  }
  HIP_TRY(timed(c, "adj_deposit_particles", [&] {
            return launch_adj_deposit_particles<T>(io, tab, c->stream);
          }), "deposit transpose (particles)");
  HIP_TRY(timed(c, "adj_finish", [&] {
            return launch_adj_finish<T>(io, tab, (const int32_t*)c->owner.p, pot, xb, yb, zb, mb,
                                        c->stream);
          }), "adjoint outputs");
  if (gas_bar) {
    for (int l = 0; l < nl; ++l) {
      if (!gas_bar[l]) continue;
      if (!io.gas_bar[l])
        return fail(APM_ERR_INVALID, "apm_solve_adjoint: gas_bar given for a level without gas");
      HIP_TRY(launch_to_t<T>(io.gas_bar[l], (T*)gas_bar[l], P.levels[l].gas_elems, c->stream),
              "gas cotangent output");
    }
  }
  return APM_OK;
}

// Layout of the totals scratch (doubles): [0] W_gas accumulator, [kTotOut ..) the
// synchronous entry points' results, [kTotPart ..) reduction partials.
constexpr int64_t kTotOut = 8, kTotPart = 64;

// Launch arguments of the totals: GMF sums of every level and the particle sums,
// partials at `part` ((nlev + 4) kMaxParts doubles), results at out_dev.
template <typename T>
apm_status totals_io_t(apm_ctx c, const void* const* gmf, const T* m, const int32_t* owner,
                       int64_t npart, const T* ax, const T* ay, const T* az, const T* pot,
                       double* part, double* out_dev, TotalsIO<T>* out) {
  const Plan& P = c->plan;
  const int nl = (int)P.levels.size();
  TotalsIO<T>& io = *out;
  io.nlev = nl;
  for (int l = 0; l < nl; ++l) {
    if (!gmf[l]) return fail(APM_ERR_INVALID, "totals: NULL gmf pointer");
    io.gmf[l] = (const T*)gmf[l];
    io.gmf_n[l] = P.levels[l].gmf_elems;
    io.vol[l] = P.levels[l].dx * P.levels[l].dx * P.levels[l].dx;
  }
  io.m = m; io.owner = owner; io.npart = npart;
  io.ax = ax; io.ay = ay; io.az = az; io.pot = pot;
  io.gas_w = nullptr;
  io.part = part;
  io.out = out_dev;
  return APM_OK;
}

// A9 totals on the stream into out_dev (nlev + 5 doubles, device): two launches, plus
// the gas-energy passes when gas is given (they read the composed fields of the last
// solve of this dtype).
template <typename T>
apm_status totals_t(apm_ctx c, apm_dtype dt, const void* const* gmf, const T* m,
                    const int32_t* owner, int64_t npart, const T* ax, const T* ay, const T* az,
                    const T* pot, const void* const* gas, double* out_dev) {
  const Plan& P = c->plan;
  const int nl = (int)P.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(kTotPart + (kMaxLevels + 4) * kMaxParts) * 8, "totals"));
  double* d = (double*)c->totals.p;
  TotalsIO<T> io{};
  APM_TRY(totals_io_t<T>(c, gmf, m, owner, npart, ax, ay, az, pot, d + kTotPart, out_dev, &io));
  bool any_gas = false;
  for (int l = 0; gas && l < nl; ++l) any_gas = any_gas || gas[l];
  if (any_gas) {
    HIP_TRY(launch_fill_f64(d, 1, 0.0, c->stream), "gas energy fill");
    std::vector<const V4<T>*> f(nl);
    for (int l = 0; l < nl; ++l) f[l] = (const V4<T>*)c->fld[(int)dt][l].p;
    APM_TRY(gas_energy_levels_t<T>(c, gas, f.data(), d));
    io.gas_w = d;
  }
  HIP_TRY(launch_totals<T>(io, c->stream), "totals");
  return APM_OK;
}

apm_status totals_any(apm_ctx c, apm_dtype dt, const void* const* gmf, const void* m,
                      const int32_t* owner, int64_t npart, const void* ax, const void* ay,
                      const void* az, const void* pot, const void* const* gas, double* out_dev) {
  if (dt == APM_F32)
    return totals_t<float>(c, dt, gmf, (const float*)m, owner, npart, (const float*)ax,
                           (const float*)ay, (const float*)az, (const float*)pot, gas, out_dev);
  return totals_t<double>(c, dt, gmf, (const double*)m, owner, npart, (const double*)ax,
                          (const double*)ay, (const double*)az, (const double*)pot, gas, out_dev);
}

// Number and mass of the particles outside the box or NaN (stream-ordered, then read).
template <typename T>
apm_status dropped_t(apm_ctx c, const T* x, const T* y, const T* z, const T* m, int64_t n,
                     int64_t* count, double* mass) {
  const int nl = (int)c->plan.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(kTotPart + (kMaxLevels + 4) * kMaxParts) * 8, "totals"));
  (void)nl;
  double* d = (double*)c->totals.p;
  double h[2] = {0.0, 0.0};
  if (n > 0) {
    HIP_TRY(launch_fill_f64(d, 2, 0.0, c->stream), "dropped clear");
    HIP_TRY(launch_dropped<T>(x, y, z, m, n, d + kTotPart, d, c->stream), "dropped particles");
    HIP_TRY(hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, c->stream), "dropped copy");
  }
  HIP_TRY(hipStreamSynchronize(c->stream), "dropped sync");
  if (count) *count = (int64_t)h[0];
  if (mass) *mass = h[1];
  return APM_OK;
}

apm_status dropped_any(apm_ctx c, apm_dtype dt, const void* x, const void* y, const void* z,
                       const void* m, int64_t n, int64_t* count, double* mass) {
  if (dt == APM_F32)
    return dropped_t<float>(c, (const float*)x, (const float*)y, (const float*)z, (const float*)m,
                            n, count, mass);
  return dropped_t<double>(c, (const double*)x, (const double*)y, (const double*)z,
                           (const double*)m, n, count, mass);
}

// Strict mode: APM_ERR_RANGE (after the call's work) if any particle was left out.
apm_status strict_check(apm_ctx c, apm_dtype dt, const void* x, const void* y, const void* z,
                        const void* m, int64_t n, const char* where) {
  if (!c->plan.cfg.strict || n <= 0) return APM_OK;
  int64_t cnt = 0;
  double mass = 0.0;
  APM_TRY(dropped_any(c, dt, x, y, z, m, n, &cnt, &mass));
  if (cnt == 0) return APM_OK;
  std::ostringstream e;
  e << where << ": strict mode: " << cnt << " particle(s) outside [0,1)^3 or NaN, mass " << mass
    << " left out";
  return fail(APM_ERR_RANGE, e.str());
}

extern "C" {

apm_status apm_dropped(apm_ctx c, apm_dtype dt, const void* x, const void* y, const void* z,
                       const void* m, int64_t npart, int64_t* count, double* mass) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_dropped: npart < 0");
  if (!count || !mass || (npart > 0 && (!x || !y || !z || !m)))
    return fail(APM_ERR_INVALID, "apm_dropped: NULL argument");
  return dropped_any(c, dt, x, y, z, m, npart, count, mass);
}

apm_status apm_create(apm_plan plan, int32_t device, void* stream, apm_ctx* out) {
  if (!plan || !out) return fail(APM_ERR_INVALID, "apm_create: NULL argument");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(APM_ERR_DEVICE, "apm_create: no HIP device visible");
  }
  if (device < 0 || device >= n) return fail(APM_ERR_DEVICE, "apm_create: device index out of range");
  HIP_TRY(hipSetDevice(device), "apm_create: hipSetDevice");
  apm_ctx c = new (std::nothrow) apm_ctx_s;
  if (!c) return fail(APM_ERR_OOM, "apm_create: host allocation failed");
  c->plan = plan->plan;
  c->device = device;
  c->stream = (hipStream_t)stream;
  {
    // once per process and device, with the device current, before any launch or
    // capture: transform kernels may use up to the device's LDS per workgroup, and the
    // device address of the fixed totals scratch is taken
    std::lock_guard<std::mutex> lock(device_setup_mutex());
    if (std::find(setup_done().begin(), setup_done().end(), device) == setup_done().end()) {
      hipError_t e = allow_lds_forward();
      if (e == hipSuccess) e = allow_lds_adjoint();
      if (e != hipSuccess) {
        apm_destroy(c);
        return hip_fail(e, "apm_create: LDS limit");
      }
      void* sp = nullptr;
      e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !sp) {
        apm_destroy(c);
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                        "apm_create: address of the fixed totals scratch");
      }
      scratch_ptrs()[device] = (double*)sp;
      setup_done().push_back(device);
    }
  }
  const Plan& P = c->plan;
  apm_status st = upload(c, (void**)&c->d_grids, P.grids.data(), sizeof(GridDesc) * P.grids.size(),
                         "grid table");
  if (st == APM_OK && P.cfg.boundary == APM_BC_PERIODIC)
    st = ensure(c, c->meanbuf, (size_t)(kMaxParts + 2) * 8, "average density");
  if (st != APM_OK) { apm_destroy(c); return st; }
  for (const LevelDesc& L : P.levels) {
    std::vector<int64_t> dep(L.count + 1), cmp(L.count + 1), act(L.count + 1), foot(L.count + 1);
    dep[0] = cmp[0] = act[0] = foot[0] = 0;
    for (int i = 0; i < L.count; ++i) {
      const GridDesc& g = P.grids[L.first + i];
      const int64_t gc = (int64_t)g.gmf_n[0] * g.gmf_n[1] * g.gmf_n[2];
      const int64_t fc = (int64_t)g.fld_n[0] * g.fld_n[1] * g.fld_n[2];
      const int64_t ac = (int64_t)g.n[0] * g.n[1] * g.n[2];
      dep[i + 1] = dep[i] + (gc + kBlock * kGmfPer - 1) / (kBlock * kGmfPer);
      cmp[i + 1] = cmp[i] + (fc + kBlock - 1) / kBlock;
      act[i + 1] = act[i] + (ac + kBlock - 1) / kBlock;
      int64_t fc2 = 0;                               // parent field cells under g's stencils
      if (g.parent >= 0) {
        fc2 = 1;
        for (int a = 0; a < 3; ++a) {
          const int l0 = std::max((g.fld_lo[a] >> 1) - 1, g.parent_fld_lo[a]);
          const int h0 = std::min(((g.fld_lo[a] + g.fld_n[a] - 1) >> 1) + 1,
                                  g.parent_fld_lo[a] + g.parent_fld_n[a] - 1);
          fc2 *= std::max(h0 - l0 + 1, 0);
        }
      }
      foot[i + 1] = foot[i] + (fc2 + kBlock - 1) / kBlock;
      const int64_t W = (g.M[0] / 2 + 1 + kRowAlign - 1) / kRowAlign * kRowAlign;   // row pitch
      c->spec_off.push_back((int64_t)c->spec_elems);
      c->z_off.push_back((int64_t)c->z_elems);
      c->y_off.push_back((int64_t)c->y_elems);
      c->spec_elems += (size_t)(g.gmf_n[2] * (int64_t)g.M[1] * W);
      c->z_elems += (size_t)(3 * (int64_t)g.fld_n[2] * g.M[1] * W);
      c->y_elems += (size_t)(4 * (int64_t)g.fld_n[2] * g.fld_n[1] * W);
    }
    void *d1 = nullptr, *d2 = nullptr, *d3 = nullptr, *d4 = nullptr;
    st = upload(c, &d1, dep.data(), dep.size() * 8, "deposit block table");
    if (st == APM_OK) st = upload(c, &d2, cmp.data(), cmp.size() * 8, "compose block table");
    if (st == APM_OK) st = upload(c, &d3, act.data(), act.size() * 8, "active cell block table");
    if (st == APM_OK) st = upload(c, &d4, foot.data(), foot.size() * 8, "restriction block table");
    if (st != APM_OK) { apm_destroy(c); return st; }
    c->d_foot_begin.push_back((int64_t*)d4);
    c->foot_blocks.push_back(foot.back());
    c->d_dep_begin.push_back((int64_t*)d1);
    c->d_cmp_begin.push_back((int64_t*)d2);
    c->d_act_begin.push_back((int64_t*)d3);
    c->dep_blocks.push_back(dep.back());
    c->cmp_blocks.push_back(cmp.back());
    c->act_blocks.push_back(act.back());
  }
  // owner lookup: each level's single grid box, or a table of the lowest-index grid
  // per cell over the bounding box of the level's active boxes
  std::vector<OwnerLevel> om(P.levels.size());
  for (size_t l = 0; l < P.levels.size(); ++l) {
    const LevelDesc& L = P.levels[l];
    OwnerLevel& o = om[l];
    o.inv_dx = 1.0 / L.dx;
    o.table = nullptr;
    if (L.count == 1) {
      const GridDesc& g = P.grids[L.first];
      for (int a = 0; a < 3; ++a) { o.lo[a] = g.lo[a]; o.n[a] = g.n[a]; }
      o.single = L.first;
      continue;
    }
    o.single = -1;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = INT32_MAX; hi[a] = INT32_MIN; }
    for (int i = 0; i < L.count; ++i) {
      const GridDesc& g = P.grids[L.first + i];
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], g.lo[a]);
        hi[a] = std::max(hi[a], g.lo[a] + g.n[a]);
      }
    }
    for (int a = 0; a < 3; ++a) { o.lo[a] = lo[a]; o.n[a] = hi[a] - lo[a]; }
    std::vector<int32_t> tab((size_t)o.n[0] * o.n[1] * o.n[2], -1);
    for (int i = L.count - 1; i >= 0; --i) {          // lower indices overwrite
      const GridDesc& g = P.grids[L.first + i];
      for (int z = 0; z < g.n[2]; ++z)
        for (int y = 0; y < g.n[1]; ++y) {
          const size_t row = ((size_t)(g.lo[2] + z - lo[2]) * o.n[1] + (g.lo[1] + y - lo[1])) * o.n[0];
          for (int x = 0; x < g.n[0]; ++x) tab[row + g.lo[0] + x - lo[0]] = L.first + i;
        }
    }
    void* d = nullptr;
    st = upload(c, &d, tab.data(), tab.size() * 4, "owner table");
    if (st != APM_OK) { apm_destroy(c); return st; }
    o.table = (const int32_t*)d;
  }
  st = upload(c, (void**)&c->d_owner_map, om.data(), om.size() * sizeof(OwnerLevel), "owner map");
  if (st != APM_OK) { apm_destroy(c); return st; }
  *out = c;
  clear_error();
  return APM_OK;
}

apm_status apm_destroy(apm_ctx c) {
  if (!c) return APM_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  for (void* p : c->owned) (void)hipFree(p);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  DevBuf* bufs[] = {&c->spec, &c->zbuf, &c->ybuf, &c->pres, &c->owner, &c->totals,
                    &c->dep_tab, &c->gpart, &c->energy, &c->lf_pot, &c->meanbuf,
                    &c->skey[0], &c->skey[1], &c->sidx[0], &c->sidx[1], &c->sprec, &c->shist,
                    &c->shsum, &c->ssorted, &c->ssref, &c->sc_lev, &c->sc_pred, &c->sc_acc};
  for (auto& B : c->lvb)
    for (DevBuf* b : {&B.tbegin, &B.tend, &B.items, &B.work, &B.bsum, &B.accum})
      if (b->p) (void)hipFree(b->p);
  for (auto* v : {&c->adj_fbar, &c->adj_gas, &c->adj_gmf[0], &c->adj_gmf[1], &c->adj_gmf[2]})
    for (auto& b : *v) if (b.p) (void)hipFree(b.p);
  if (c->adj_pacc.p) (void)hipFree(c->adj_pacc.p);
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (auto& v : c->gmf)
    for (auto& b : v) if (b.p) (void)hipFree(b.p);
  for (auto& v : c->fld)
    for (auto& b : v) if (b.p) (void)hipFree(b.p);
  for (auto& v : c->sc_fld)
    for (auto& b : v) if (b.p) (void)hipFree(b.p);
  delete c;
  return APM_OK;
}

apm_status apm_set_stream(apm_ctx c, void* stream) {
  APM_TRY(check_ctx(c));
  c->stream = (hipStream_t)stream;
  return APM_OK;
}

apm_status apm_owner(apm_ctx c, apm_dtype dt, const void* x, const void* y, const void* z,
                     int64_t npart, int32_t* owner) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0 || npart > INT32_MAX) return fail(APM_ERR_RANGE, "apm_owner: npart out of range");
  if (npart > 0 && (!x || !y || !z || !owner)) return fail(APM_ERR_INVALID, "apm_owner: NULL array");
  const Plan& P = c->plan;
  hipError_t e = dt == APM_F32
      ? launch_owner<float>(c->d_owner_map, (int32_t)P.levels.size(), (const float*)x,
                            (const float*)y, (const float*)z, npart, owner, nullptr, nullptr,
                            nullptr, nullptr, c->stream)
      : launch_owner<double>(c->d_owner_map, (int32_t)P.levels.size(), (const double*)x,
                             (const double*)y, (const double*)z, npart, owner, nullptr, nullptr,
                             nullptr, nullptr, c->stream);
  HIP_TRY(e, "apm_owner");
  return APM_OK;
}

apm_status apm_deposit(apm_ctx c, apm_dtype dt, int32_t level, const void* x, const void* y,
                       const void* z, const void* m, int64_t npart, const void* gas,
                       const void* parent_gas, void* gmf) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  APM_TRY(check_level(c, level));
  if (npart < 0 || npart > INT32_MAX) return fail(APM_ERR_RANGE, "apm_deposit: npart out of range");
  if (!gmf || (npart > 0 && (!x || !y || !z || !m)))
    return fail(APM_ERR_INVALID, "apm_deposit: NULL array");
  if (level == 0 && parent_gas) return fail(APM_ERR_INVALID, "apm_deposit: root has no parent gas");
  c->last_solve.clear();                             // the particle sort is replaced
  const bool mean = level == 0 && c->plan.cfg.boundary == APM_BC_PERIODIC;
  if (dt == APM_F32) {
    const float* g = (const float*)gas;
    const float* pg = (const float*)parent_gas;
    float* out = (float*)gmf;
    APM_TRY(deposit_levels_t<float>(c, level, 1, (const float*)x, (const float*)y, (const float*)z,
                                    (const float*)m, npart, nullptr, &g, &pg, &out));
    if (mean)
      APM_TRY(mean_density_t<float>(c, (const float*)x, (const float*)y, (const float*)z,
                                    (const float*)m, npart, g));
    return strict_check(c, dt, x, y, z, m, npart, "apm_deposit");
  }
  const double* g = (const double*)gas;
  const double* pg = (const double*)parent_gas;
  double* out = (double*)gmf;
  APM_TRY(deposit_levels_t<double>(c, level, 1, (const double*)x, (const double*)y,
                                   (const double*)z, (const double*)m, npart, nullptr, &g, &pg,
                                   &out));
  if (mean)
    APM_TRY(mean_density_t<double>(c, (const double*)x, (const double*)y, (const double*)z,
                                   (const double*)m, npart, g));
  return strict_check(c, dt, x, y, z, m, npart, "apm_deposit");
}

apm_status apm_solve_level(apm_ctx c, apm_dtype dt, int32_t level, const void* gmf, void* field) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  APM_TRY(check_level(c, level));
  if (!gmf || !field) return fail(APM_ERR_INVALID, "apm_solve_level: NULL array");
  if (dt == APM_F32) return solve_level_t<float>(c, level, (const float*)gmf, (float*)field);
  return solve_level_t<double>(c, level, (const double*)gmf, (double*)field);
}

apm_status apm_accel(apm_ctx c, apm_dtype dt, int32_t level, const void* own,
                     const void* parent_field, void* field) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  APM_TRY(check_level(c, level));
  if (!own || !field) return fail(APM_ERR_INVALID, "apm_accel: NULL array");
  if (level == 0 && parent_field) return fail(APM_ERR_INVALID, "apm_accel: root has no parent");
  if (level > 0 && !parent_field) return fail(APM_ERR_STATE, "apm_accel: parent field required");
  const LevelDesc& L = c->plan.levels[level];
  hipError_t e = dt == APM_F32
      ? launch_compose<float>(c->d_grids + L.first, c->d_cmp_begin[level], L.count,
                              (const float4*)own, (const float4*)parent_field, (float4*)field,
                              c->cmp_blocks[level], c->stream)
      : launch_compose<double>(c->d_grids + L.first, c->d_cmp_begin[level], L.count,
                               (const double4*)own, (const double4*)parent_field, (double4*)field,
                               c->cmp_blocks[level], c->stream);
  HIP_TRY(e, "apm_accel");
  return APM_OK;
}

apm_status apm_interp(apm_ctx c, apm_dtype dt, int32_t level, const void* field, const void* x,
                      const void* y, const void* z, const int32_t* owner, int64_t npart, void* ax,
                      void* ay, void* az, void* pot) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  APM_TRY(check_level(c, level));
  if (npart < 0 || npart > INT32_MAX) return fail(APM_ERR_RANGE, "apm_interp: npart out of range");
  if (npart > 0 && (!field || !x || !y || !z || !owner || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_interp: NULL array");
  hipError_t e = dt == APM_F32
      ? launch_interp<float>(c->d_grids, level, (const float4*)field, (const float*)x,
                             (const float*)y, (const float*)z, owner, npart, (float*)ax,
                             (float*)ay, (float*)az, (float*)pot, c->stream)
      : launch_interp<double>(c->d_grids, level, (const double4*)field, (const double*)x,
                              (const double*)y, (const double*)z, owner, npart, (double*)ax,
                              (double*)ay, (double*)az, (double*)pot, c->stream);
  HIP_TRY(e, "apm_interp");
  return APM_OK;
}

apm_status apm_totals(apm_ctx c, apm_dtype dt, const void* const* gmf, const void* m,
                      const int32_t* owner, int64_t npart, const void* ax, const void* ay,
                      const void* az, const void* pot, double* out) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (!out || !gmf) return fail(APM_ERR_INVALID, "apm_totals: NULL argument");
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_totals: npart < 0");
  if (npart > 0 && (!m || !owner || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_totals: NULL particle array");
  const int nl = (int)c->plan.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(kTotPart + (kMaxLevels + 4) * kMaxParts) * 8, "totals"));
  double* res = (double*)c->totals.p + kTotOut;
  APM_TRY(totals_any(c, dt, gmf, m, owner, npart, ax, ay, az, pot, nullptr, res));
  HIP_TRY(hipMemcpyAsync(out, res, (size_t)(nl + 4) * 8, hipMemcpyDeviceToHost, c->stream),
          "totals copy");
  HIP_TRY(hipStreamSynchronize(c->stream), "totals sync");
  return APM_OK;
}

apm_status apm_totals_noalloc(apm_ctx c, apm_dtype dt, const void* const* gmf, const void* m,
                              const int32_t* owner, int64_t npart, const void* ax, const void* ay,
                              const void* az, const void* pot, double* out_dev) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (!out_dev || !gmf) return fail(APM_ERR_INVALID, "apm_totals_noalloc: NULL argument");
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_totals_noalloc: npart < 0");
  if (npart > 0 && (!m || !owner || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_totals_noalloc: NULL particle array");
  const int nl = (int)c->plan.levels.size();
  if ((int64_t)(nl + 4) * kMaxParts > kNoAllocScratch)
    return fail(APM_ERR_RANGE, "apm_totals_noalloc: more levels than the fixed scratch holds");
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(device_setup_mutex());
    auto it = scratch_ptrs().find(c->device);
    if (it != scratch_ptrs().end()) part = it->second;
  }
  if (!part) return fail(APM_ERR_STATE, "apm_totals_noalloc: no fixed scratch on this device");
  // the same two launches as apm_totals, with the partials in the fixed scratch
  if (dt == APM_F32) {
    TotalsIO<float> io{};
    APM_TRY(totals_io_t<float>(c, gmf, (const float*)m, owner, npart, (const float*)ax,
                               (const float*)ay, (const float*)az, (const float*)pot, part,
                               out_dev, &io));
    HIP_TRY(launch_totals<float>(io, c->stream), "apm_totals_noalloc");
  } else {
    TotalsIO<double> io{};
    APM_TRY(totals_io_t<double>(c, gmf, (const double*)m, owner, npart, (const double*)ax,
                                (const double*)ay, (const double*)az, (const double*)pot, part,
                                out_dev, &io));
    HIP_TRY(launch_totals<double>(io, c->stream), "apm_totals_noalloc");
  }
  return APM_OK;
}

apm_status apm_solve(apm_ctx c, apm_dtype dt, const void* x, const void* y, const void* z,
                     const void* m, int64_t npart, const void* const* gas, void* ax, void* ay,
                     void* az, void* pot) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0 || npart > INT32_MAX) return fail(APM_ERR_RANGE, "apm_solve: npart out of range");
  if (npart > 0 && (!x || !y || !z || !m || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_solve: NULL array");
  if (dt == APM_F32)
    APM_TRY(solve_t<float>(c, dt, (const float*)x, (const float*)y, (const float*)z,
                           (const float*)m, npart, gas, (float*)ax, (float*)ay, (float*)az,
                           (float*)pot));
  else
    APM_TRY(solve_t<double>(c, dt, (const double*)x, (const double*)y, (const double*)z,
                            (const double*)m, npart, gas, (double*)ax, (double*)ay, (double*)az,
                            (double*)pot));
  return strict_check(c, dt, x, y, z, m, npart, "apm_solve");
}

static apm_status solve_totals_check(apm_ctx c, apm_dtype dt, const void* m, int64_t npart,
                                     const void* ax, const void* ay, const void* az) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  const int nl = (int)c->plan.levels.size();
  const int di = (int)dt;
  if ((int)c->gmf[di].size() != nl || (int)c->fld[di].size() != nl || !c->owner.p ||
      c->owner.bytes < (size_t)std::max<int64_t>(npart, 1) * 4)
    return fail(APM_ERR_STATE, "apm_solve_totals: no apm_solve of this dtype/size yet");
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_solve_totals: npart < 0");
  if (npart > 0 && (!m || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_solve_totals: NULL particle array");
  return APM_OK;
}

// The gas term reads the composed level fields: they must be those of the last
// apm_solve of this dtype (apm_autotune and apm_deposit invalidate them).
static apm_status solve_totals_gas_check(apm_ctx c, apm_dtype dt, const void* const* gas) {
  bool any = false;
  for (size_t l = 0; gas && l < c->plan.levels.size(); ++l) any = any || gas[l];
  if (any && (c->last_solve.empty() || c->last_solve[0] != (uintptr_t)dt))
    return fail(APM_ERR_STATE, "apm_solve_totals: the level fields are not those of an apm_solve "
                               "of this dtype (apm_autotune or apm_deposit ran since)");
  return APM_OK;
}

static apm_status solve_totals_into(apm_ctx c, apm_dtype dt, const void* m, int64_t npart,
                                    const void* const* gas, const void* ax, const void* ay,
                                    const void* az, const void* pot, double* out_dev) {
  const int nl = (int)c->plan.levels.size();
  std::vector<const void*> g(nl);
  for (int l = 0; l < nl; ++l) g[l] = c->gmf[(int)dt][l].p;
  return totals_any(c, dt, g.data(), m, (const int32_t*)c->owner.p, npart, ax, ay, az, pot, gas,
                    out_dev);
}

apm_status apm_solve_totals(apm_ctx c, apm_dtype dt, const void* m, int64_t npart,
                            const void* const* gas, const void* ax, const void* ay,
                            const void* az, const void* pot, double* out) {
  APM_TRY(solve_totals_check(c, dt, m, npart, ax, ay, az));
  APM_TRY(solve_totals_gas_check(c, dt, gas));
  if (!out) return fail(APM_ERR_INVALID, "apm_solve_totals: NULL out");
  const int nl = (int)c->plan.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(kTotPart + (kMaxLevels + 4) * kMaxParts) * 8, "totals"));
  double* res = (double*)c->totals.p + kTotOut;
  APM_TRY(solve_totals_into(c, dt, m, npart, gas, ax, ay, az, pot, res));
  HIP_TRY(hipMemcpyAsync(out, res, (size_t)(nl + 5) * 8, hipMemcpyDeviceToHost, c->stream),
          "totals copy");
  HIP_TRY(hipStreamSynchronize(c->stream), "totals sync");
  return APM_OK;
}

apm_status apm_solve_totals_async(apm_ctx c, apm_dtype dt, const void* m, int64_t npart,
                                  const void* const* gas, const void* ax, const void* ay,
                                  const void* az, const void* pot, double* out_dev) {
  APM_TRY(solve_totals_check(c, dt, m, npart, ax, ay, az));
  APM_TRY(solve_totals_gas_check(c, dt, gas));
  if (!out_dev) return fail(APM_ERR_INVALID, "apm_solve_totals_async: NULL out");
  return solve_totals_into(c, dt, m, npart, gas, ax, ay, az, pot, out_dev);
}

apm_status apm_gas_energy(apm_ctx c, apm_dtype dt, int32_t level, const void* gas,
                          const void* field, double* out) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  APM_TRY(check_level(c, level));
  if (!gas || !field || !out) return fail(APM_ERR_INVALID, "apm_gas_energy: NULL argument");
  const int nl = (int)c->plan.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(nl + 4 + 4 * kMaxParts) * 8, "totals"));
  double* d = (double*)c->totals.p;
  HIP_TRY(launch_fill_f64(d, 1, 0.0, c->stream), "gas energy fill");
  std::vector<const void*> g(nl, nullptr);
  g[level] = gas;
  if (dt == APM_F32) {
    std::vector<const V4<float>*> f(nl, nullptr);
    f[level] = (const V4<float>*)field;
    APM_TRY(gas_energy_levels_t<float>(c, g.data(), f.data(), d));
  } else {
    std::vector<const V4<double>*> f(nl, nullptr);
    f[level] = (const V4<double>*)field;
    APM_TRY(gas_energy_levels_t<double>(c, g.data(), f.data(), d));
  }
  HIP_TRY(hipMemcpyAsync(out, d, 8, hipMemcpyDeviceToHost, c->stream), "gas energy copy");
  HIP_TRY(hipStreamSynchronize(c->stream), "gas energy sync");
  return APM_OK;
}

apm_status apm_kick(apm_ctx c, apm_dtype dt, int64_t npart, void* vx, void* vy, void* vz,
                    const void* ax, const void* ay, const void* az, double h) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_kick: npart < 0");
  if (npart > 0 && (!vx || !vy || !vz || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_kick: NULL array");
  hipError_t e = dt == APM_F32
      ? launch_kick_drift<float>(npart, nullptr, nullptr, nullptr, (float*)vx, (float*)vy,
                                 (float*)vz, (const float*)ax, (const float*)ay, (const float*)az,
                                 h, 0.0, 0, c->stream)
      : launch_kick_drift<double>(npart, nullptr, nullptr, nullptr, (double*)vx, (double*)vy,
                                  (double*)vz, (const double*)ax, (const double*)ay,
                                  (const double*)az, h, 0.0, 0, c->stream);
  HIP_TRY(e, "apm_kick");
  return APM_OK;
}

apm_status apm_drift(apm_ctx c, apm_dtype dt, int64_t npart, void* x, void* y, void* z,
                     const void* vx, const void* vy, const void* vz, double h) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_drift: npart < 0");
  if (npart > 0 && (!x || !y || !z || !vx || !vy || !vz))
    return fail(APM_ERR_INVALID, "apm_drift: NULL array");
  const int wrap = c->plan.cfg.boundary == APM_BC_PERIODIC;
  hipError_t e = dt == APM_F32
      ? launch_kick_drift<float>(npart, (float*)x, (float*)y, (float*)z, (float*)vx, (float*)vy,
                                 (float*)vz, nullptr, nullptr, nullptr, 0.0, h, wrap, c->stream)
      : launch_kick_drift<double>(npart, (double*)x, (double*)y, (double*)z, (double*)vx,
                                  (double*)vy, (double*)vz, nullptr, nullptr, nullptr, 0.0, h, wrap,
                                  c->stream);
  HIP_TRY(e, "apm_drift");
  return APM_OK;
}

apm_status apm_kinetic_energy(apm_ctx c, apm_dtype dt, const void* m, const void* vx,
                              const void* vy, const void* vz, int64_t npart, double* out) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (!out) return fail(APM_ERR_INVALID, "apm_kinetic_energy: NULL out");
  if (npart < 0) return fail(APM_ERR_RANGE, "apm_kinetic_energy: npart < 0");
  if (npart > 0 && (!m || !vx || !vy || !vz))
    return fail(APM_ERR_INVALID, "apm_kinetic_energy: NULL array");
  const int nl = (int)c->plan.levels.size();
  APM_TRY(ensure(c, c->totals, (size_t)(nl + 4 + 4 * kMaxParts) * 8, "totals"));
  double* d = (double*)c->totals.p;
  HIP_TRY(launch_fill_f64(d, 1, 0.0, c->stream), "kinetic fill");
  hipError_t e = dt == APM_F32
      ? launch_kinetic<float>((const float*)m, (const float*)vx, (const float*)vy,
                              (const float*)vz, npart, d + nl + 4, d, c->stream)
      : launch_kinetic<double>((const double*)m, (const double*)vx, (const double*)vy,
                               (const double*)vz, npart, d + nl + 4, d, c->stream);
  HIP_TRY(e, "kinetic energy");
  HIP_TRY(hipMemcpyAsync(out, d, 8, hipMemcpyDeviceToHost, c->stream), "kinetic copy");
  HIP_TRY(hipStreamSynchronize(c->stream), "kinetic sync");
  return APM_OK;
}

apm_status apm_leapfrog(apm_ctx c, apm_dtype dt, void* x, void* y, void* z, void* vx, void* vy,
                        void* vz, const void* m, int64_t npart, const void* const* gas, double h,
                        int32_t nsteps, void* ax, void* ay, void* az, void* pot, double* energy) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0 || npart > INT32_MAX) return fail(APM_ERR_RANGE, "apm_leapfrog: npart out of range");
  if (nsteps < 0) return fail(APM_ERR_RANGE, "apm_leapfrog: nsteps < 0");
  if (npart > 0 && (!x || !y || !z || !vx || !vy || !vz || !m || !ax || !ay || !az))
    return fail(APM_ERR_INVALID, "apm_leapfrog: NULL array");
  if (dt == APM_F32)
    return leapfrog_t<float>(c, dt, (float*)x, (float*)y, (float*)z, (float*)vx, (float*)vy,
                             (float*)vz, (const float*)m, npart, gas, h, nsteps, (float*)ax,
                             (float*)ay, (float*)az, (float*)pot, energy);
  return leapfrog_t<double>(c, dt, (double*)x, (double*)y, (double*)z, (double*)vx, (double*)vy,
                            (double*)vz, (const double*)m, npart, gas, h, nsteps, (double*)ax,
                            (double*)ay, (double*)az, (double*)pot, energy);
}

apm_status apm_evolve_subcycled(apm_ctx c, apm_dtype dt, void* x, void* y, void* z, void* vx,
                                void* vy, void* vz, const void* m, int64_t npart,
                                const void* const* gas, double h0, int32_t nroot,
                                double* energy) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0 || npart > INT32_MAX)
    return fail(APM_ERR_RANGE, "apm_evolve_subcycled: npart out of range");
  if (nroot < 0) return fail(APM_ERR_RANGE, "apm_evolve_subcycled: nroot < 0");
  if (!(h0 > 0.0)) return fail(APM_ERR_INVALID, "apm_evolve_subcycled: h0 must be positive");
  if (npart > 0 && (!x || !y || !z || !vx || !vy || !vz || !m))
    return fail(APM_ERR_INVALID, "apm_evolve_subcycled: NULL array");
  c->last_solve.clear();                             // the particle sort is replaced
  if (dt == APM_F32)
    return evolve_subcycled_t<float>(c, dt, (float*)x, (float*)y, (float*)z, (float*)vx,
                                     (float*)vy, (float*)vz, (const float*)m, npart, gas, h0,
                                     nroot, energy);
  return evolve_subcycled_t<double>(c, dt, (double*)x, (double*)y, (double*)z, (double*)vx,
                                    (double*)vy, (double*)vz, (const double*)m, npart, gas, h0,
                                    nroot, energy);
}

const void* apm_field_ptr(apm_ctx c, apm_dtype dt, int32_t level) {
  if (!c || (dt != APM_F32 && dt != APM_F64) || level < 0 ||
      level >= (int32_t)c->fld[(int)dt].size())
    return nullptr;
  return c->fld[(int)dt][level].p;
}

apm_status apm_autotune(apm_ctx c, apm_dtype dt, int32_t reps, char* report, int32_t cap) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (reps < 1) reps = 5;
  APM_TRY(dt == APM_F32 ? autotune_t<float>(c, dt, reps) : autotune_t<double>(c, dt, reps));
  if (report && cap > 0) std::snprintf(report, (size_t)cap, "%s", c->tune_report.c_str());
  return APM_OK;
}

apm_status apm_set_graph(apm_ctx c, int32_t enable) {
  APM_TRY(check_ctx(c));
  c->use_graph = enable != 0;
  drop_graph(c);
  c->gkey.clear();
  return APM_OK;
}

apm_status apm_profile(apm_ctx c, int32_t enable) {
  APM_TRY(check_ctx(c));
  if (enable) {
    APM_TRY(prof_collect(c));
    c->prof_acc.clear();
    c->prof_names.clear();
    c->prof_on = true;
  } else {
    c->prof_on = false;
    APM_TRY(prof_collect(c));
  }
  return APM_OK;
}

int32_t apm_profile_count(apm_ctx c) {
  if (!c || check_ctx(c) != APM_OK || prof_collect(c) != APM_OK) return -1;
  return (int32_t)c->prof_names.size();
}

apm_status apm_profile_entry(apm_ctx c, int32_t i, char* name, int32_t cap, double* total_ms,
                             int64_t* launches) {
  APM_TRY(check_ctx(c));
  APM_TRY(prof_collect(c));
  if (i < 0 || i >= (int32_t)c->prof_names.size() || !name || cap < 1)
    return fail(APM_ERR_INVALID, "apm_profile_entry: bad index or buffer");
  const std::string& n = c->prof_names[i];
  std::snprintf(name, (size_t)cap, "%s", n.c_str());
  const auto& a = c->prof_acc[n];
  if (total_ms) *total_ms = a.first;
  if (launches) *launches = a.second;
  return APM_OK;
}

const void* apm_gmf_ptr(apm_ctx c, apm_dtype dt, int32_t level) {
  if (!c || (dt != APM_F32 && dt != APM_F64) || level < 0 ||
      level >= (int32_t)c->gmf[(int)dt].size())
    return nullptr;
  return c->gmf[(int)dt][level].p;
}


apm_status apm_solve_adjoint(apm_ctx c, apm_dtype dt, const void* x, const void* y, const void* z,
                             const void* m, int64_t npart, const void* const* gas,
                             const void* pot, const void* abar_x, const void* abar_y,
                             const void* abar_z, const void* phibar, double wbar, void* xbar,
                             void* ybar, void* zbar, void* mbar, void* const* gas_bar) {
  APM_TRY(check_ctx(c));
  APM_TRY(check_dtype(dt));
  if (npart < 0 || npart > INT32_MAX) return fail(APM_ERR_RANGE, "apm_solve_adjoint: npart out of range");
  if (npart > 0 && (!x || !y || !z || !m))
    return fail(APM_ERR_INVALID, "apm_solve_adjoint: NULL particle array");
  if (wbar != 0.0 && npart > 0 && !pot)
    return fail(APM_ERR_INVALID, "apm_solve_adjoint: wbar != 0 needs the solve's potentials");
  if (dt == APM_F32)
    return adjoint_t<float>(c, dt, (const float*)x, (const float*)y, (const float*)z,
                            (const float*)m, npart, gas, (const float*)pot, (const float*)abar_x,
                            (const float*)abar_y, (const float*)abar_z, (const float*)phibar, wbar,
                            (float*)xbar, (float*)ybar, (float*)zbar, (float*)mbar, gas_bar);
  return adjoint_t<double>(c, dt, (const double*)x, (const double*)y, (const double*)z,
                           (const double*)m, npart, gas, (const double*)pot, (const double*)abar_x,
                           (const double*)abar_y, (const double*)abar_z, (const double*)phibar,
                           wbar, (double*)xbar, (double*)ybar, (double*)zbar, (double*)mbar,
                           gas_bar);
}

}  // extern "C"
