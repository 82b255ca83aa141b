// Test-only shim: exposes the host table code of libbf.so (bf_tables.cpp) to
// the CPU tests, which compare it with the FP64 oracle.  Built with g++ by
// tests/test_host_tables.py; not part of the library.
#include <cstring>
#include <string>

#include "../paper_1203_5128_amd/csrc/bf_internal.h"

extern "C" {
int shim_order_N(double T, double sigma_r) { return bfi::order_N(T, sigma_r); }
int shim_trunc_M(int N, double sigma_r8, double eps) { return bfi::trunc_M(N, sigma_r8, eps); }
// Fills N, M, K, qfix, alpha_turn for T and copies the pairs (m, c').
int shim_table_entry(double sigma_r, double eps, double range, int T_cap, int T, int *N, int *M, int *K,
                     unsigned long long *qfix, double *alpha_turn, int *pm, float *pc, int cap) {
  bfi::OrderTable t;
  std::string err;
  if (!bfi::build_order_table(sigma_r, eps, range, T_cap, t, err)) return -1;
  const bfi::OrderEntry &e = t.ent[t.idx_of_T[T]];
  *N = e.N; *M = e.M; *K = e.K; *qfix = e.qfix; *alpha_turn = e.alpha_turn;
  for (int k = 0; k < e.K && k < cap; k++) { pm[k] = t.pm[e.off + k]; pc[k] = t.pc[e.off + k]; }
  return t.K_max;
}
// Polynomial range kernel table: N, J, K, kappa and the per-slot basis values
// and coefficients ([K][256][2] floats each, at most cap floats copied).
int shim_rp_table(double sigma_r, double eps, double L, double T, int *N, int *J, int *K, double *kappa,
                  float *gen, float *comb, int cap) {
  bfi::RpTable t;
  std::string err;
  if (!bfi::build_rp_table(sigma_r, eps, L, T, t, err)) return -1;
  *N = t.N; *J = t.J; *K = t.K; *kappa = t.kappa;
  const int n = (int)t.gen.size() < cap ? (int)t.gen.size() : cap;
  std::memcpy(gen, t.gen.data(), sizeof(float) * n);
  std::memcpy(comb, t.comb.data(), sizeof(float) * n);
  return n;
}
int shim_iir_consts(double sigma, float *out, int n) {
  std::vector<float> v;
  std::string err;
  if (!bfi::build_iir_consts(sigma, v, err)) return -1;
  std::memcpy(out, v.data(), sizeof(float) * (n < (int)v.size() ? n : (int)v.size()));
  return (int)v.size();
}
int shim_layout(int c, int *o) {
  const int hb = c == bfi::kCSmall ? bfi::kIirHSmall : bfi::kIirHLarge;
  o[0] = bfi::kIirCoef; o[1] = bfi::kIirMts; o[2] = hb + bfi::iir_h_apow(c); o[3] = bfi::kIirSize;
  o[4] = c; o[5] = hb + bfi::iir_h_lane(c); o[6] = hb + bfi::iir_h_scan(c); o[7] = hb + bfi::iir_h_wave(c);
  return 0;
}
}
