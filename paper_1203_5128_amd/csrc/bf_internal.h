// Internal declarations shared by the host tables, the kernels and the plan
// runtime of libbf.so.  Not part of the public ABI (that is include/bf.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bf.h"

namespace bfi {

// ---------------------------------------------------------------- geometry
// Blocked recursive Gaussian: samples of a row (or column) owned by one
// thread (a per-plan choice between the two values below; each has its own
// block of scan constants).
constexpr int kCSmall = 16;
constexpr int kCLarge = 32;
// Threads per workgroup of both recursive passes.
constexpr int kHThreads = 256;
// Workgroups the horizontal pass aims for (rows x pair groups): two per CU.
// Short images split their pairs into groups to get there; taller ones keep
// one group (the partial sums and their reduction cost more than they gain).
constexpr int kHWorkgroups = 512;
// The same for each image of a batch: one pair group per image of 128 rows
// or more (64-image batch, horizontal stage at 64 / 128 / 256 / 512 per
// image: 1.14 / 1.14 / 1.15 / 1.17 ms).
constexpr int kHWorkgroupsBatch = 128;
// Workgroups the vertical pass aims for: one round of resident workgroups
// (two per CU); each takes several pairs of its columns one after another,
// so that its set-up (constants, input samples) is paid once.
constexpr int kVWorkgroups = 512;
// The same for each image of a batch, whose grouped launch the other images
// fill: more pairs per workgroup, whose set-up is then paid once for them
// (64-image batch, vertical stage at 64 / 96 / 128 / 192 / 256 / 512 / 1024
// per image: 1.10 / 1.06 / 1.04 / 1.03 / 1.05 / 1.10 / 1.16 ms).
constexpr int kVWorkgroupsBatch = 160;
// Largest supported width and height of the recursive path: one row (column)
// group of kHThreads threads.
constexpr int kMaxWidth = kCLarge * kHThreads;

// ------------------------------------------------------- order tables (a1)
// One entry per distinct order N reachable from T in [0, T_cap].
struct OrderEntry {
  int32_t N;         // order (Algorithm 2 step 3)
  int32_t M;         // terms dropped per tail (step 4)
  int32_t K;         // frequency pairs kept, the zero frequency included
  int32_t off;       // first pair in the pair arrays
  uint64_t qfix;     // frac(alpha / 2pi) * 2^64, alpha = 1 / (sqrt(N) sigma_r)
  double alpha_turn; // alpha / 2pi, turns per intensity unit per unit of m
};

struct OrderTable {
  int32_t T_cap = 0;
  std::vector<int32_t> idx_of_T;  // T -> entry
  std::vector<OrderEntry> ent;
  std::vector<int32_t> pm;        // per pair: m = 2n - N (<= 0)
  std::vector<float> pc;          // per pair: c' = 2^(1-N) C(N,n), or 2^-N C(N,N/2) for m = 0
  int32_t K_max = 0;
  int32_t N_max = 0;
};

int order_N(double T, double sigma_r);
// Non-local means: p patch samples share N and M; each pair is a folded
// multi-index (m_1..m_p) (first non-zero component negative, or all zero),
// packed as p signed bytes in pm, with weight 2 prod c (1 for all zero).
constexpr int kNlmMaxPatch = 4;
constexpr int kNlmMaxOffset = 2;
bool build_nlm_table(double sigma_r, double eps, double value_range, int32_t T_cap, int p, OrderTable &out,
                     std::string &err);
int trunc_M(int N, double sigma_r8, double eps);
bool build_order_table(double sigma_r, double eps, double value_range, int32_t T_cap,
                       OrderTable &out, std::string &err);

// ------------------------------------- polynomial range kernel (eq. (RP))
// Order N, highest kept Chebyshev order J, slots of two orders K = ceil((J+1)/2),
// and per slot k and 8-bit intensity v (float pairs, [k][v][2]): the basis
// values (T_2k, T_2k+1)(x(v)) and the coefficients (c_2k, c_2k+1)(v).
// kappa = max_v sum_j |c_j(v)|, the cancellation factor of the FP32 sums.
struct RpTable {
  int N = 0, J = 0, K = 0;
  double kappa = 0.0;
  std::vector<float> gen, comb;
};
bool build_rp_table(double sigma_r, double eps, double L, double T, RpTable &out, std::string &err);

// ------------------------------------------- recursive Gaussian constants
// State of one direction of the cascade after element n: (s[n], w[n], d[n])
// with s the first-order section, w the second-order section output and
// d[n] = (w[n] - w[n-1]) / g2.  Carrying the (scaled) increment instead of
// w[n-1] keeps the FP32 rounding of the second-order section from being fed
// back through its poles, which sit close to z = 1 for wide Gaussians.
// Rows and columns are padded with zeros to whole chunks and the
// zero-extension boundary is applied at the padded end: the causal outputs in
// the padding are exactly the continuation of the zero-extended signal, so the
// result is the same as at the true end and no chunk is ever short.
// Float layout of the constant block (offsets in floats):
constexpr int kIirCoef = 0;                      // 1-g1, g2, c2, g1
constexpr int kIirMts = 4;                       // 3x3: end boundary (zero extension)
// Block for a chunk of c samples per thread:
//   A^v, v = 0..c (9 each); A^(c l), l = 0..63; A^(c 2^k), k = 0..7; A^(64 c).
constexpr int iir_hblock_size(int c) { return 9 * (c + 1) + 9 * 64 + 9 * 8 + 9; }
constexpr int kIirHSmall = kIirMts + 9;
constexpr int kIirHLarge = kIirHSmall + iir_hblock_size(kCSmall);
constexpr int kIirSize = kIirHLarge + iir_hblock_size(kCLarge);
// offsets inside a block
constexpr int iir_h_apow(int) { return 0; }
constexpr int iir_h_lane(int c) { return 9 * (c + 1); }
constexpr int iir_h_scan(int c) { return 9 * (c + 1) + 9 * 64; }
constexpr int iir_h_wave(int c) { return 9 * (c + 1) + 9 * 64 + 9 * 8; }

bool yvv_cascade(double sigma, double &g1, double &g2, double &c1, double &c2, std::string &err);
bool build_iir_consts(double sigma_s, std::vector<float> &out, std::string &err);

// FIR taps exp(-j^2 / (2 sigma^2)), j = -R..R (FP64 on the host).
void build_fir_taps(double sigma_s, int R, std::vector<double> &taps);

}  // namespace bfi
