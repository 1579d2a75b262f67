// Runs the host-only surface of libsvdp (parameter defaults, workspace
// sizing of every op over edge shapes, the CANS / polynomial / Polar Express
// schedule tables, status strings, argument rejection before any launch)
// for AddressSanitizer / UndefinedBehaviorSanitizer builds of the library's
// host code (tests/test_host_sanitizers.py).  No GPU is needed: nothing here
// reaches a launch.  Prints "ok" or the first failed expectation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "svdp.h"

static int failures = 0;
#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::printf("failed: %s (line %d)\n", #cond, __LINE__);           \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

int main() {
  // workspace sizes of every op, over the workloads and the edges
  const int64_t shapes[][3] = {{1, 64, 64},      {256, 512, 512}, {16, 4096, 1024}, {1, 2048, 2048},
                               {2, 2048, 2048},  {1, 8192, 8192}, {64, 256, 256},   {0, 8, 8},
                               {1, 1, 1},        {3, 130, 100},   {1, 4096, 4096},  {5, 9000, 8}};
  for (const auto& sh : shapes)
    for (int prec = 0; prec < 2; ++prec)
      for (int poly = 0; poly < 4; ++poly)
        for (int op = 0; op < 8; ++op) {
          svdp_params p;
          svdp_default_params(&p, sh[0], sh[1], sh[2]);
          p.precision = prec;
          p.poly = poly;
          size_t bytes = 0;
          const svdp_status s = svdp_workspace_size(&p, op, &bytes);
          EXPECT(s == SVDP_OK || s == SVDP_ERR_SHAPE || s == SVDP_ERR_INVALID_ARG);
          if (s == SVDP_OK && sh[0] > 0) EXPECT(bytes > 0);
        }
  {
    svdp_params p;
    svdp_default_params(&p, 1, 4, 8);  // m < n
    size_t bytes = 0;
    EXPECT(svdp_workspace_size(&p, SVDP_OP_SVD_FWD, &bytes) == SVDP_ERR_SHAPE);
    EXPECT(svdp_last_error() != nullptr);
    svdp_default_params(&p, 1, 8, 8);
    EXPECT(svdp_workspace_size(&p, 99, &bytes) == SVDP_ERR_INVALID_ARG);
    EXPECT(svdp_workspace_size(&p, SVDP_OP_SVD_FWD, nullptr) == SVDP_ERR_INVALID_ARG);
    p.max_iters = 65;
    EXPECT(svdp_workspace_size(&p, SVDP_OP_SVD_FWD, &bytes) == SVDP_ERR_INVALID_ARG);
  }
  for (int s = -1; s < 8; ++s) EXPECT(svdp_status_string(s) != nullptr);
  // schedule tables
  {
    std::vector<double> tab(64 * 3);
    double t = 0.0;
    int32_t steps = 0;
    for (double delta : {0.9, 0.99, 0.999, 0.9999})
      for (int pre = 0; pre < 4; ++pre) {
        EXPECT(svdp_cans_table(0, delta, pre, 0.0, 64, tab.data(), &t) == SVDP_OK);
        for (int poly = 0; poly < 3; ++poly)
          EXPECT(svdp_poly_table(poly, delta, pre, 64, tab.data(), &t) == SVDP_OK);
      }
    for (double lo : {1e-7, 1e-3, 0.5, 0.99}) EXPECT(svdp_cans_table(1, 0.99, 2, lo, 64, tab.data(), &t) == SVDP_OK);
    EXPECT(svdp_cans_table(0, 0.99, 2, 0.0, 0, tab.data(), &t) == SVDP_OK);
    EXPECT(svdp_cans_table(0, 0.99, 2, 0.0, -1, tab.data(), &t) != SVDP_OK);
    EXPECT(svdp_cans_table(0, 1.5, 2, 0.0, 8, tab.data(), &t) != SVDP_OK);
    EXPECT(svdp_cans_table(1, 0.99, 2, 0.0, 8, tab.data(), &t) != SVDP_OK);
    EXPECT(svdp_cans_table(2, 0.99, 2, 0.0, 8, tab.data(), &t) != SVDP_OK);
    EXPECT(svdp_cans_table(0, 0.99, 2, 0.0, 8, nullptr, &t) != SVDP_OK);
    EXPECT(svdp_poly_table(7, 0.99, 2, 8, tab.data(), nullptr) != SVDP_OK);
    for (double lo : {8.2e-8, 1e-3, 0.5}) EXPECT(svdp_pe_table(lo, 64, tab.data(), &steps) == SVDP_OK);
    EXPECT(svdp_pe_table(1e-3, 2, tab.data(), &steps) != SVDP_OK);
    EXPECT(svdp_pe_table(0.0, 64, tab.data(), &steps) != SVDP_OK);
    EXPECT(svdp_pe_table(1.5, 64, tab.data(), &steps) != SVDP_OK);
  }
  // every device entry point rejects a null handle or bad sizes before a launch
  {
    svdp_params p;
    svdp_default_params(&p, 2, 16, 16);
    float dummy[4] = {0, 0, 0, 0};
    EXPECT(svd_polar_fwd(nullptr, &p, dummy, 16, 256, dummy, 16, 256, dummy, 16, dummy, 16, 256, nullptr,
                         dummy, 4, nullptr) != SVDP_OK);
    EXPECT(svdp_eigh(nullptr, &p, dummy, 16, 256, dummy, 16, dummy, 16, 256, nullptr, dummy, 4, nullptr) !=
           SVDP_OK);
    EXPECT(svdp_eigh_dc(nullptr, &p, dummy, 16, 256, dummy, 16, dummy, 16, 256, nullptr, dummy, 4, nullptr) !=
           SVDP_OK);
    EXPECT(svdp_spectral_features(dummy, dummy, 0, 16, dummy, dummy, dummy, nullptr) == SVDP_OK);
    EXPECT(svdp_spectral_features(dummy, dummy, -1, 16, dummy, dummy, dummy, nullptr) != SVDP_OK);
    EXPECT(svdp_training_targets(dummy, dummy, -1, 16, dummy, nullptr) != SVDP_OK);
    EXPECT(svdp_feature_stats(dummy, -1, dummy, dummy, nullptr) != SVDP_OK);
  }
  EXPECT(svdp_host_syncs() == 0);
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
