// Host-side planning: validation of a static nested hierarchy and the layout of
// every per-level buffer (no device needed).
//
// Geometry rules (Sec. 2 and 2.2 of the paper, and the readings recorded in the
// design notes):
//  * level-l cell size dx_l = 1 / (root_n 2^l), refinement factor 2;
//  * GMF box: the root's active box (its mass is confined to the domain); a
//    subgrid's active box grown by `ghost` cells, filled from its parent;
//  * field box (where accelerations and potential are produced): the root's active
//    box; a subgrid's active box grown by one cell (TSC interpolation stencil);
//  * FFT box: root 2 root_n per axis (James doubling for the isolated boundary) or
//    root_n (periodic boundary, Sec. 2.1: no padding needed); subgrid: the power of
//    two >= GMF extent + p, p = ceil(pad_factor 2 a_cells)
//    (the 0.65 R a/dx cells of zero padding, Sec. 2.2).
#include <cmath>
#include <cstring>
#include <sstream>

#include "apm_internal.hpp"

namespace apm {

static thread_local std::string g_err;

apm_status fail(apm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

static int32_t next_pow2(int32_t v) {
  int32_t m = 1;
  while (m < v) m <<= 1;
  return m;
}

apm_status build_plan(const apm_config& cfg, const apm_grid* grids, int32_t ngrids, Plan& P) {
  std::ostringstream e;
  if (!grids || ngrids < 1) return fail(APM_ERR_INVALID, "apm_plan_create: no grids");
  if (!(cfg.G > 0.0) || !std::isfinite(cfg.G)) return fail(APM_ERR_INVALID, "G must be > 0");
  if (cfg.boundary != APM_BC_ISOLATED && cfg.boundary != APM_BC_PERIODIC)
    return fail(APM_ERR_INVALID, "unknown boundary");
  const bool periodic = cfg.boundary == APM_BC_PERIODIC;
  if (!is_pow2(cfg.root_n) || cfg.root_n < 8)
    return fail(APM_ERR_INVALID, "root_n must be a power of two >= 8");
  if ((periodic ? 1 : 2) * (int64_t)cfg.root_n > kMaxFFT)
    return fail(APM_ERR_RANGE, periodic ? "root_n > 1024: root FFT longer than 1024"
                                        : "root_n > 512: doubled root FFT longer than 1024");
  if (!(cfg.a_cells > 0.0) || !(cfg.pad_factor >= 0.0))
    return fail(APM_ERR_INVALID, "a_cells must be > 0 and pad_factor >= 0");
  if (cfg.ghost < 2) return fail(APM_ERR_INVALID, "ghost must be >= 2");
  if (cfg.brillouin < 0 || cfg.brillouin > 3) return fail(APM_ERR_INVALID, "brillouin in [0,3]");
  if (cfg.gradient != APM_GRAD_SPECTRAL && cfg.gradient != APM_GRAD_FD2)
    return fail(APM_ERR_INVALID, "unknown gradient");
  if (cfg.workspace_limit < 0) return fail(APM_ERR_INVALID, "workspace_limit < 0");
  if (cfg.strict != 0 && cfg.strict != 1) return fail(APM_ERR_INVALID, "strict must be 0 or 1");
  if (cfg.deposit_accum != APM_ACC_F64 && cfg.deposit_accum != APM_ACC_F32_COMP)
    return fail(APM_ERR_INVALID, "unknown deposit_accum");

  P.cfg = cfg;
  P.pad = (int32_t)std::ceil(cfg.pad_factor * 2.0 * cfg.a_cells - 1e-12);
  P.grids.clear();
  P.levels.clear();
  const int32_t N = cfg.root_n;
  const apm_grid& r = grids[0];
  if (r.level != 0 || r.parent != -1 || r.lo[0] || r.lo[1] || r.lo[2] || r.n[0] != N ||
      r.n[1] != N || r.n[2] != N)
    return fail(APM_ERR_INVALID, "grid 0 must be the root: level 0, parent -1, lo 0, n root_n");

  int32_t maxlev = 0;
  for (int32_t i = 0; i < ngrids; ++i) {
    const apm_grid& g = grids[i];
    GridDesc d{};
    d.level = g.level;
    d.parent = g.parent;
    d.index = i;
    for (int a = 0; a < 3; ++a) { d.lo[a] = g.lo[a]; d.n[a] = g.n[a]; }
    if (i > 0) {
      if (g.level < 1 || g.level > 20) { e << "grid " << i << ": level must be in [1,20]"; return fail(APM_ERR_INVALID, e.str()); }  // 21 levels at most
      if (g.level < grids[i - 1].level) { e << "grid " << i << ": grids must be sorted by level"; return fail(APM_ERR_INVALID, e.str()); }
      if (g.parent < 0 || g.parent >= i || grids[g.parent].level != g.level - 1) {
        e << "grid " << i << ": parent must be an earlier grid one level up";
        return fail(APM_ERR_INVALID, e.str());
      }
      for (int a = 0; a < 3; ++a) {
        if (g.n[a] < 2 || (g.n[a] & 1) || (g.lo[a] & 1)) {
          e << "grid " << i << ": lo and n must be even, n >= 2";
          return fail(APM_ERR_INVALID, e.str());
        }
      }
      // nesting: the parent cells under the GMF box (ghost gas is copied from them)
      // and under the interpolation stencil of the field box lie inside the
      // parent's active box: [floor((lo-b)/2), floor((lo+n+b-1)/2)], b >= 2.
      const apm_grid& p = grids[g.parent];
      for (int a = 0; a < 3; ++a) {
        const int64_t b = cfg.ghost;
        int64_t c0 = ((int64_t)g.lo[a] - b) >> 1, c1 = ((int64_t)g.lo[a] + g.n[a] + b - 1) >> 1;
        if (c0 < p.lo[a] || c1 > (int64_t)p.lo[a] + p.n[a] - 1) {
          e << "grid " << i << ": its ghost zone must lie inside its parent's active box (axis " << a << ")";
          return fail(APM_ERR_INVALID, e.str());
        }
      }
    }
    maxlev = std::max(maxlev, g.level);
    d.dx = 1.0 / ((double)N * std::ldexp(1.0, g.level));
    if (i == 0) {
      for (int a = 0; a < 3; ++a) {
        d.gmf_lo[a] = 0; d.gmf_n[a] = N;
        d.fld_lo[a] = 0; d.fld_n[a] = N;
        d.M[a] = periodic ? N : 2 * N;
      }
      d.wrap = periodic ? N : 0;
    } else {
      for (int a = 0; a < 3; ++a) {
        d.gmf_lo[a] = g.lo[a] - cfg.ghost;
        d.gmf_n[a] = g.n[a] + 2 * cfg.ghost;
        d.fld_lo[a] = g.lo[a] - 1;
        d.fld_n[a] = g.n[a] + 2;
        int64_t need = (int64_t)d.gmf_n[a] + P.pad;
        if (need > kMaxFFT) {
          e << "grid " << i << ": padded FFT length " << need << " > " << kMaxFFT;
          return fail(APM_ERR_RANGE, e.str());
        }
        d.M[a] = std::max(next_pow2((int32_t)need), 8);
      }
    }
    P.grids.push_back(d);
  }
  // the particle sort keys a particle by its 8^3-cell tile on the finest level, 21
  // bits per axis in a 64-bit Morton code
  if (((int64_t)N << maxlev) > ((int64_t)1 << 24)) {
    e << "finest level has " << ((int64_t)N << maxlev) << " cells per axis (at most 2^24)";
    return fail(APM_ERR_RANGE, e.str());
  }
  // levels: grids are sorted, so each level is a contiguous range
  P.levels.resize(maxlev + 1);
  for (auto& L : P.levels) { L = LevelDesc{}; L.first = -1; }
  for (int32_t i = 0; i < ngrids; ++i) {
    GridDesc& d = P.grids[i];
    LevelDesc& L = P.levels[d.level];
    if (L.first < 0) L.first = i;
    L.count++;
    L.dx = d.dx;
    d.gmf_offset = L.gmf_elems;
    d.fld_offset = L.fld_cells;
    d.gas_offset = L.gas_elems;
    L.gmf_elems += (int64_t)d.gmf_n[0] * d.gmf_n[1] * d.gmf_n[2];
    L.fld_cells += (int64_t)d.fld_n[0] * d.fld_n[1] * d.fld_n[2];
    L.gas_elems += (int64_t)d.n[0] * d.n[1] * d.n[2];
  }
  for (size_t l = 0; l < P.levels.size(); ++l) {
    LevelDesc& L = P.levels[l];
    if (L.count == 0) {
      e << "level " << l << " has no grids";
      return fail(APM_ERR_INVALID, e.str());
    }
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = INT64_MAX; hi[a] = INT64_MIN; }
    for (int32_t i = L.first; i < L.first + L.count; ++i) {
      const GridDesc& d = P.grids[i];
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min<int64_t>(lo[a], d.gmf_lo[a] - 1);
        hi[a] = std::max<int64_t>(hi[a], (int64_t)d.gmf_lo[a] + d.gmf_n[a] + 1);
      }
    }
    L.key_cells = 1;
    for (int a = 0; a < 3; ++a) {
      L.key_lo[a] = (int32_t)lo[a];
      L.key_n[a] = (int32_t)(hi[a] - lo[a]);
      L.key_cells *= L.key_n[a];
    }
    if (L.key_cells >= (int64_t)1 << 31) {
      e << "level " << l << ": binning box of " << L.key_cells << " cells exceeds int32";
      return fail(APM_ERR_RANGE, e.str());
    }
  }
  for (auto& d : P.grids) {
    if (d.parent >= 0) {
      const GridDesc& p = P.grids[d.parent];
      d.parent_fld_offset = p.fld_offset;
      d.parent_gas_offset = p.gas_offset;
      for (int a = 0; a < 3; ++a) {
        d.parent_lo[a] = p.lo[a]; d.parent_n[a] = p.n[a];
        d.parent_fld_lo[a] = p.fld_lo[a]; d.parent_fld_n[a] = p.fld_n[a];
      }
    }
  }
  clear_error();
  return APM_OK;
}

}  // namespace apm

// ------------------------------------------------------------------ C ABI (host) --

extern "C" {

void apm_config_default(apm_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->G = 1.0;
  cfg->root_n = 0;
  cfg->a_cells = 3.4;
  cfg->pad_factor = 0.65;
  cfg->ghost = 3;
  cfg->brillouin = 1;
  cfg->gradient = APM_GRAD_SPECTRAL;
  cfg->workspace_limit = 0;
  cfg->boundary = APM_BC_ISOLATED;
  cfg->deposit_accum = APM_ACC_F64;
}

apm_status apm_plan_create(const apm_config* cfg, const apm_grid* grids, int32_t ngrids,
                           apm_plan* out) {
  if (!cfg || !out) return apm::fail(APM_ERR_INVALID, "apm_plan_create: NULL argument");
  *out = nullptr;
  apm_plan p = new (std::nothrow) apm_plan_s;
  if (!p) return apm::fail(APM_ERR_OOM, "apm_plan_create: host allocation failed");
  apm_status st = apm::build_plan(*cfg, grids, ngrids, p->plan);
  if (st != APM_OK) {
    delete p;
    return st;
  }
  *out = p;
  return APM_OK;
}

apm_status apm_plan_destroy(apm_plan plan) {
  delete plan;
  return APM_OK;
}

int32_t apm_plan_nlevels(apm_plan plan) {
  return plan ? (int32_t)plan->plan.levels.size() : -1;
}

int32_t apm_plan_ngrids(apm_plan plan) {
  return plan ? (int32_t)plan->plan.grids.size() : -1;
}

apm_status apm_plan_grid(apm_plan plan, int32_t grid, apm_grid_layout* out) {
  if (!plan || !out) return apm::fail(APM_ERR_INVALID, "apm_plan_grid: NULL argument");
  if (grid < 0 || grid >= (int32_t)plan->plan.grids.size())
    return apm::fail(APM_ERR_INVALID, "apm_plan_grid: grid index out of range");
  const apm::GridDesc& d = plan->plan.grids[grid];
  out->level = d.level;
  out->parent = d.parent;
  for (int a = 0; a < 3; ++a) {
    out->lo[a] = d.lo[a]; out->n[a] = d.n[a];
    out->gmf_lo[a] = d.gmf_lo[a]; out->gmf_n[a] = d.gmf_n[a];
    out->fld_lo[a] = d.fld_lo[a]; out->fld_n[a] = d.fld_n[a];
    out->fft_n[a] = d.M[a];
  }
  out->gmf_offset = d.gmf_offset;
  out->fld_offset = d.fld_offset;
  out->gas_offset = d.gas_offset;
  out->dx = d.dx;
  return APM_OK;
}

apm_status apm_plan_level(apm_plan plan, int32_t level, apm_level_layout* out) {
  if (!plan || !out) return apm::fail(APM_ERR_INVALID, "apm_plan_level: NULL argument");
  if (level < 0 || level >= (int32_t)plan->plan.levels.size())
    return apm::fail(APM_ERR_INVALID, "apm_plan_level: level out of range");
  const apm::LevelDesc& L = plan->plan.levels[level];
  out->ngrids = L.count;
  out->first_grid = L.first;
  out->gmf_elems = L.gmf_elems;
  out->fld_cells = L.fld_cells;
  out->gas_elems = L.gas_elems;
  out->dx = L.dx;
  return APM_OK;
}

const char* apm_last_error(void) { return apm::last_error(); }

}  // extern "C"
