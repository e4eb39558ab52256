// Host-side driver for the sanitizer build of the plan code (AddressSanitizer and
// UndefinedBehaviorSanitizer): valid hierarchies shaped like the benchmark
// configurations and a set of invalid descriptors, every layout query, NULL
// arguments, and the thread-local error message.  Exits non-zero on an unexpected
// status; the sanitizers abort on any memory or undefined-behaviour error.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/apm.h"

static int failures = 0;

static void expect(apm_status got, apm_status want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want,
                 apm_last_error());
    ++failures;
  }
}

static apm_grid grid(int level, int parent, int lx, int ly, int lz, int nx, int ny, int nz) {
  apm_grid g;
  g.level = level; g.parent = parent;
  g.lo[0] = lx; g.lo[1] = ly; g.lo[2] = lz;
  g.n[0] = nx; g.n[1] = ny; g.n[2] = nz;
  return g;
}

static void exercise(int root_n, const std::vector<apm_grid>& gs, int boundary, apm_status want,
                     const char* what) {
  apm_config cfg;
  apm_config_default(&cfg);
  cfg.root_n = root_n;
  cfg.boundary = boundary;
  apm_plan p = nullptr;
  apm_status st = apm_plan_create(&cfg, gs.data(), (int32_t)gs.size(), &p);
  expect(st, want, what);
  if (st != APM_OK) return;
  const int ng = apm_plan_ngrids(p), nl = apm_plan_nlevels(p);
  for (int i = -1; i <= ng; ++i) {
    apm_grid_layout gl;
    expect(apm_plan_grid(p, i, &gl), (i >= 0 && i < ng) ? APM_OK : APM_ERR_INVALID, "grid query");
  }
  for (int l = -1; l <= nl; ++l) {
    apm_level_layout ll;
    expect(apm_plan_level(p, l, &ll), (l >= 0 && l < nl) ? APM_OK : APM_ERR_INVALID, "level query");
  }
  expect(apm_plan_grid(p, 0, nullptr), APM_ERR_INVALID, "NULL layout");
  expect(apm_plan_destroy(p), APM_OK, "destroy");
}

int main() {
  std::vector<apm_grid> g;
  // a single 32^3 root; root 128^3 + two centred 64^3 levels; root 512^3 + three 256^3
  exercise(32, {grid(0, -1, 0, 0, 0, 32, 32, 32)}, APM_BC_ISOLATED, APM_OK, "root 32");
  exercise(128, {grid(0, -1, 0, 0, 0, 128, 128, 128), grid(1, 0, 96, 96, 96, 64, 64, 64),
                 grid(2, 1, 224, 224, 224, 64, 64, 64)}, APM_BC_ISOLATED, APM_OK, "nested 128");
  exercise(512, {grid(0, -1, 0, 0, 0, 512, 512, 512), grid(1, 0, 384, 384, 384, 256, 256, 256),
                 grid(2, 1, 896, 896, 896, 256, 256, 256),
                 grid(3, 2, 1920, 1920, 1920, 256, 256, 256)}, APM_BC_ISOLATED, APM_OK,
           "nested 512");
  exercise(1024, {grid(0, -1, 0, 0, 0, 1024, 1024, 1024)}, APM_BC_PERIODIC, APM_OK,
           "periodic 1024");
  // many uneven grids on one level (overlaps allowed)
  g = {grid(0, -1, 0, 0, 0, 64, 64, 64)};
  for (int i = 0; i < 64; ++i)
    g.push_back(grid(1, 0, 8 + 2 * (i % 40), 8 + 2 * ((i * 7) % 40), 8 + 2 * ((i * 13) % 40),
                     8 + 2 * (i % 9), 8 + 2 * ((i * 3) % 7), 8 + 2 * ((i * 5) % 11)));
  exercise(64, g, APM_BC_ISOLATED, APM_OK, "uneven level");
  // invalid descriptors
  exercise(12, {grid(0, -1, 0, 0, 0, 12, 12, 12)}, APM_BC_ISOLATED, APM_ERR_INVALID, "root 12");
  exercise(1024, {grid(0, -1, 0, 0, 0, 1024, 1024, 1024)}, APM_BC_ISOLATED, APM_ERR_RANGE,
           "isolated 1024");
  exercise(16, {grid(0, -1, 0, 0, 0, 16, 16, 16), grid(1, 0, 3, 8, 8, 8, 8, 8)}, APM_BC_ISOLATED,
           APM_ERR_INVALID, "odd lo");
  exercise(16, {grid(0, -1, 0, 0, 0, 16, 16, 16), grid(1, 5, 8, 8, 8, 8, 8, 8)}, APM_BC_ISOLATED,
           APM_ERR_INVALID, "bad parent");
  exercise(16, {grid(0, -1, 0, 0, 0, 16, 16, 16), grid(1, 0, 8, 8, 8, 2000000000, 8, 8)},
           APM_BC_ISOLATED, APM_ERR_INVALID, "huge n");
  exercise(16, {grid(0, -1, 0, 0, 0, 16, 16, 16), grid(1, 0, -2147483000, 8, 8, 8, 8, 8)},
           APM_BC_ISOLATED, APM_ERR_INVALID, "huge negative lo");
  exercise(16, {grid(0, -1, 0, 0, 0, 16, 16, 16)}, 9, APM_ERR_INVALID, "bad boundary");
  apm_plan p = nullptr;
  expect(apm_plan_create(nullptr, nullptr, 0, &p), APM_ERR_INVALID, "NULL config");
  apm_config cfg;
  apm_config_default(&cfg);
  cfg.root_n = 16;
  expect(apm_plan_create(&cfg, nullptr, 1, &p), APM_ERR_INVALID, "NULL grids");
  expect(apm_plan_destroy(nullptr), APM_OK, "destroy NULL");
  if (apm_plan_nlevels(nullptr) != -1) ++failures;
  if (std::strlen(apm_last_error()) == 0) ++failures;
  std::printf("plan driver: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
