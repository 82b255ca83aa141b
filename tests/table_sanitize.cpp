// Test-only driver: runs the host table builders of libbf.so (bf_tables.cpp)
// over a sweep of parameters, including the edges the plan accepts, so that
// tests/test_host_sanitizers.py can build it with AddressSanitizer and
// UndefinedBehaviorSanitizer and check that no access or arithmetic is
// undefined.  Exit status 0 when every builder succeeded where it must.
#include <cstdio>
#include <string>
#include <vector>

#include "../paper_1203_5128_amd/csrc/bf_internal.h"

int main() {
  int failures = 0;
  std::string err;
  // raised-cosine order tables: 8-bit, 16-bit and float ranges, sigma_r from
  // tight to wide, eps from 1e-6 to 0.1, T caps from 0 up
  const double srs[] = {0.5, 3.0, 10.0, 40.0, 200.0, 800.0};
  const double epss[] = {1e-6, 1e-3, 0.05, 0.1};
  const struct { double range; int cap; } ranges[] = {{255.0, 255}, {65535.0, 4096}, {1.0, 1}, {255.0, 0}};
  for (double sr : srs)
    for (double eps : epss)
      for (const auto &r : ranges) {
        if (r.cap > 255 && sr < 200.0) continue;  // keeps the 16-bit tables small
        bfi::OrderTable t;
        if (bfi::build_order_table(sr, eps, r.range, r.cap, t, err)) {
          for (int T = 0; T <= r.cap; T++) {
            const bfi::OrderEntry &e = t.ent[t.idx_of_T[T]];
            if (e.K < 1 || e.off + e.K > (int)t.pm.size()) failures++;
          }
        }
        if (r.range == 255.0 && sr >= 10.0)  // non-local means: 8-bit input
          for (int p = 2; p <= 4; p++) {
            bfi::OrderTable nt;
            (void)bfi::build_nlm_table(sr, eps, r.range, r.cap, p, nt, err);
          }
      }
  // polynomial range kernel tables
  for (double sr : {5.0, 10.0, 30.0, 60.0})
    for (double eps : {1e-4, 1e-3, 1e-2}) {
      bfi::RpTable rt;
      if (!bfi::build_rp_table(sr, eps, 255.0, 255.0, rt, err)) failures++;
    }
  // recursive Gaussian constants over the accepted sigma range
  for (double s : {0.5, 0.7, 1.0, 2.5, 3.0, 10.0, 16.0, 40.0, 100.0}) {
    std::vector<float> v;
    if (!bfi::build_iir_consts(s, v, err) || (int)v.size() != bfi::kIirSize) failures++;
  }
  for (int R : {0, 1, 48, 120}) {
    std::vector<double> taps;
    bfi::build_fir_taps(3.0, R, taps);
    if ((int)taps.size() != 2 * R + 1) failures++;
  }
  std::printf("table sanitizer sweep: %d failures\n", failures);
  return failures ? 1 : 0;
}
