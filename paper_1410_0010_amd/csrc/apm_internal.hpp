// Internal declarations shared by the host plan, the kernels and the ABI layer.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/apm.h"

namespace apm {

constexpr int kMaxFFT = 1024;

// Per-grid layout as the kernels see it (plain data, copied to the device).
struct GridDesc {
  int32_t level, parent, index;
  int32_t lo[3], n[3];
  int32_t gmf_lo[3], gmf_n[3];
  int32_t fld_lo[3], fld_n[3];
  int32_t M[3];
  int64_t gmf_offset, fld_offset, gas_offset;
  int64_t parent_fld_offset;       // parent's field-box offset in its level buffer
  int64_t parent_gas_offset;
  int32_t parent_lo[3], parent_n[3];          // parent active box
  int32_t parent_fld_lo[3], parent_fld_n[3];  // parent field box
  int32_t wrap;                    // periodic root: cells per axis (stencils wrap), else 0
  double dx;
};

struct LevelDesc {
  int32_t first, count;            // grid range
  int64_t gmf_elems, fld_cells, gas_elems;
  int32_t key_lo[3], key_n[3];     // union of GMF boxes grown by 1 (binning box)
  int64_t key_cells;
  double dx;
};

struct Plan {
  apm_config cfg;
  int32_t pad;                      // total zero padding per axis of subgrids
  std::vector<GridDesc> grids;
  std::vector<LevelDesc> levels;
};

// thread-local error message helpers
apm_status fail(apm_status st, const std::string& msg);
void clear_error();

apm_status build_plan(const apm_config& cfg, const apm_grid* grids, int32_t ngrids, Plan& out);

inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace apm

struct apm_plan_s {
  apm::Plan plan;
};

namespace apm {
const char* last_error();
}
