// Host-side exercise of the library's C ABI for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (no GPU calls are made): cluster
// selection on a centroid file, the plan's counts, and every argument check that
// returns before device work.  Prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "osv.h"

#define REQUIRE(c)                                               \
  do {                                                           \
    if (!(c)) {                                                  \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                  \
    }                                                            \
  } while (0)

int main(int argc, char **argv) {
  if (argc < 5) return 2;
  // centroid file: int32 nocc, then nocc x 3 doubles; expected n1b n2b n3b
  FILE *f = std::fopen(argv[1], "rb");
  REQUIRE(f);
  int nocc = 0;
  REQUIRE(std::fread(&nocc, 4, 1, f) == 1);
  std::vector<double> cen((size_t)nocc * 3);
  REQUIRE(std::fread(cen.data(), 8, cen.size(), f) == cen.size());
  std::fclose(f);
  const long long want[3] = {std::atoll(argv[2]), std::atoll(argv[3]), std::atoll(argv[4])};
  osv_select sel{OSV_SEL_DISTANCE, 15.0, 7.0, 1e-2, 0.2, 1e-8};
  osv_counts c{};
  REQUIRE(osv_plan_clusters(nocc, cen.data(), &sel, &c, nullptr, nullptr, 0) == OSV_OK);
  REQUIRE(c.n1b == want[0] && c.n2b == want[1] && c.n3b == want[2]);
  std::vector<int32_t> lmos((size_t)3 * c.n_clusters);
  std::vector<double> coef(c.n_clusters);
  REQUIRE(osv_plan_clusters(nocc, cen.data(), &sel, &c, lmos.data(), coef.data(), c.n_clusters) == OSV_OK);
  REQUIRE(osv_plan_clusters(nocc, cen.data(), &sel, &c, lmos.data(), coef.data(), c.n_clusters - 1) == OSV_E_ARG);
  // each selected pair (and LMO) is counted once by the coefficients
  double tot = 0.0;
  for (long long X = 0; X < c.n_clusters; X++) tot += coef[X];
  REQUIRE(tot > 0.0);
  osv_select full{OSV_SEL_FULL, 0, 0, 0, 0, 1e-8};
  REQUIRE(osv_plan_clusters(nocc, cen.data(), &full, &c, nullptr, nullptr, 0) == OSV_OK);
  REQUIRE(c.n_clusters == 1 && c.n_pair_blocks == (long long)nocc * (nocc + 1) / 2);
  osv_select bad{7, 0, 0, 0, 0, 1e-8};
  REQUIRE(osv_plan_clusters(nocc, cen.data(), &bad, &c, nullptr, nullptr, 0) == OSV_E_ARG);
  REQUIRE(osv_plan_clusters(nocc, nullptr, &sel, &c, nullptr, nullptr, 0) == OSV_E_ARG);
  // argument checks of the device entry points (return before any device work)
  osv_ctx *ctx = nullptr;
  std::vector<int32_t> r(2, 3);
  osv_system sys{};
  sys.nocc = 2; sys.nvir = 10; sys.naux = 5; sys.r = r.data();
  sys.Q = (const double *)16; sys.C = (const void *)16; sys.C_dtype = OSV_DT_F64;
  sys.eps_vir = (const double *)16; sys.F_occ = (const double *)16; sys.centroid = cen.data();
  REQUIRE(osv_build_pairs(nullptr, &sel, OSV_FP64, nullptr, &ctx) == OSV_E_ARG && !ctx);
  REQUIRE(osv_build_pairs(&sys, &sel, 9, nullptr, &ctx) == OSV_E_ARG);
  REQUIRE(osv_build_pairs(&sys, &sel, OSV_MIXED, nullptr, &ctx) == OSV_E_ARG);   // MIXED needs FP32 C
  r[1] = 200;
  REQUIRE(osv_build_pairs(&sys, &sel, OSV_FP64, nullptr, &ctx) == OSV_E_ARG);    // r_i > nvir
  REQUIRE(std::strlen(osv_last_error(nullptr)) > 0);
  int32_t rr[2];
  REQUIRE(osv_generate_osvs(2, 5000, 4, (const double *)16, (const double *)16, (const double *)16, 1e-4, 10,
                            nullptr, rr, nullptr, (double *)16, nullptr) == OSV_E_ARG);   // nvir too large
  REQUIRE(osv_generate_osvs(2, 10, 4, (const double *)16, (const double *)16, (const double *)16, 1e-4, 11,
                            nullptr, rr, nullptr, (double *)16, nullptr) == OSV_E_ARG);   // r_max > nvir
  double E = 0.0;
  REQUIRE(osv_solve_clusters(nullptr, 1e-10, 10, nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_energy(nullptr, nullptr, &E, nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_densities(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_weak_pairs(nullptr, nullptr, &E, nullptr, nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_weak_pairs_noalloc(nullptr, nullptr, &E, nullptr, nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_high_order_correction(nullptr, nullptr, &E, nullptr, nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_query(nullptr, nullptr) == OSV_E_ARG);
  REQUIRE(osv_release_cached_memory(-2) == OSV_E_ARG);
  for (int st = 0; st >= -8; st--) REQUIRE(osv_status_string(st) != nullptr);
  osv_destroy(nullptr);
  std::printf("ok\n");
  return 0;
}
