// Host-side FP64 tables of libbf.so: the order/truncation/coefficient table for
// every integer T a plan can meet, and the constants of the recursive Gaussian.
//
// Order and truncation follow Algorithm 2 of the paper: step 3 (N from T and
// sigma_r, rounded to the nearest integer, as Table 1 prints it), step 4 (M by
// the sigma_r band: none above 40, eq. (trunc) in (10, 40], eq. (Chernoff) at
// or below 10, sigma_r in 8-bit units), eq. (approx) for the kept terms and
// eq. (expansion) for their weights and frequencies.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "bf_internal.h"

namespace bfi {

int order_N(double T, double sigma_r) {
  double v = 0.405 * (T / sigma_r) * (T / sigma_r);
  double r = std::floor(v + 0.5);
  if (!(r >= 1.0)) return 1;
  if (r > 2147483647.0) return 2147483647;
  return (int)r;
}

// log of 2^-N C(N, n)
static double log_binom_weight(int N, int n) {
  return std::lgamma((double)N + 1.0) - std::lgamma((double)n + 1.0) -
         std::lgamma((double)(N - n) + 1.0) - (double)N * std::log(2.0);
}

// Eq. (trunc): the first m whose cumulative binomial mass exceeds eps/2; every
// term below it is dropped, so each tail loses at most eps/2.
static int trunc_exact(int N, double eps) {
  double s = 0.0;
  for (int m = 0; m <= N / 2; m++) {
    s += std::exp(log_binom_weight(N, m));
    if (s > 0.5 * eps) return m;
  }
  return N / 2;
}

// Eq. (Chernoff): M = (N - sqrt(4 N log(2/eps))) / 2, rounded down, >= 0.
static int trunc_chernoff(int N, double eps) {
  double v = 0.5 * ((double)N - std::sqrt(4.0 * (double)N * std::log(2.0 / eps)));
  if (!(v >= 0.0)) return 0;
  return (int)std::floor(v);
}

int trunc_M(int N, double sigma_r8, double eps) {
  int M;
  if (sigma_r8 > 40.0) M = 0;
  else if (sigma_r8 > 10.0) M = trunc_exact(N, eps);
  else M = trunc_chernoff(N, eps);
  if (M > N / 2) M = N / 2;
  return M;
}

bool build_order_table(double sigma_r, double eps, double value_range, int32_t T_cap,
                       OrderTable &out, std::string &err) {
  out = OrderTable();
  out.T_cap = T_cap;
  out.idx_of_T.resize((size_t)T_cap + 1);
  const double sigma_r8 = sigma_r * 255.0 / value_range;
  std::map<int, int> seen;
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int32_t T = 0; T <= T_cap; T++) {
    int N = order_N((double)T, sigma_r);
    auto it = seen.find(N);
    if (it != seen.end()) { out.idx_of_T[T] = it->second; continue; }
    if (N > (1 << 22)) { err = "order N above 4194304 (sigma_r too small for the value range)"; return false; }
    int M = trunc_M(N, sigma_r8, eps);
    OrderEntry e;
    e.N = N;
    e.M = M;
    e.off = (int32_t)out.pm.size();
    // kept n = M..N-M; fold n with N-n (same weight, opposite frequency)
    for (int n = M; 2 * n < N; n++) {
      out.pm.push_back(2 * n - N);
      out.pc.push_back((float)(2.0 * std::exp(log_binom_weight(N, n))));
    }
    if (N % 2 == 0) {
      out.pm.push_back(0);
      out.pc.push_back((float)std::exp(log_binom_weight(N, N / 2)));
    }
    e.K = (int32_t)out.pm.size() - e.off;
    if (out.pm.size() > (size_t)64 << 20) { err = "order table above 64M pairs"; return false; }
    // turns per unit of m * intensity, in 64-bit fixed point (long double keeps
    // the 64 fractional bits the integer phase reduction relies on)
    long double at = 1.0L / (two_pi * std::sqrt((long double)N) * (long double)sigma_r);
    long double fr = at - std::floor(at);
    long double sc = fr * 18446744073709551616.0L;
    e.qfix = sc >= 18446744073709551615.0L ? ~0ull : (uint64_t)sc;
    e.alpha_turn = (double)at;
    out.idx_of_T[T] = (int32_t)out.ent.size();
    seen[N] = (int32_t)out.ent.size();
    out.ent.push_back(e);
    if (e.K > out.K_max) out.K_max = e.K;
    if (N > out.N_max) out.N_max = N;
  }
  return true;
}

// ---------------------------------------------------- non-local means ---
// The product over the p patch samples of the truncated raised cosine of
// eq. (approx): prod_k sum_{n_k} c_{n_k} cos(m_k alpha s_k) with m = 2n - N,
// alpha = 1 / (sqrt(N) sigma_r).  Expanding the product of cosines gives one
// cosine of alpha sum_k m_k s_k per multi-index; m and -m give the same term,
// so each conjugate pair is kept once with twice the weight.
bool build_nlm_table(double sigma_r, double eps, double value_range, int32_t T_cap, int p, OrderTable &out,
                     std::string &err) {
  out = OrderTable();
  if (p < 2 || p > kNlmMaxPatch) { err = "patch size outside 2..4"; return false; }
  out.T_cap = T_cap;
  out.idx_of_T.resize((size_t)T_cap + 1);
  const double sigma_r8 = sigma_r * 255.0 / value_range;
  std::map<int, int> seen;
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int32_t T = 0; T <= T_cap; T++) {
    const int N = order_N((double)T, sigma_r);
    auto it = seen.find(N);
    if (it != seen.end()) { out.idx_of_T[T] = it->second; continue; }
    const int M = trunc_M(N, sigma_r8, eps);
    if (N - 2 * M > 127) { err = "non-local means: kept frequencies above 127 (sigma_r too small)"; return false; }
    const int L = N - 2 * M + 1;
    double total = 1.0;
    for (int k = 0; k < p; k++) total *= L;
    if (out.pm.size() + total / 2 + 1 > (double)(4 << 20)) {
      err = "non-local means: more than 4M frequency multi-indices (sigma_r too small for the patch size)";
      return false;
    }
    std::vector<double> w(L);
    for (int i = 0; i < L; i++) w[i] = std::exp(log_binom_weight(N, M + i));
    OrderEntry e;
    e.N = N;
    e.M = M;
    e.off = (int32_t)out.pm.size();
    std::vector<int> idx(p, 0);  // kept-term index per sample, sample 0 slowest
    for (;;) {
      int first = 0;  // first non-zero m
      double c = 1.0;
      uint32_t packed = 0;
      for (int k = 0; k < p; k++) {
        const int m = 2 * (M + idx[k]) - N;
        if (!first && m) first = m;
        c *= w[idx[k]];
        packed |= (uint32_t)(uint8_t)(int8_t)m << (8 * k);
      }
      if (first <= 0) {
        out.pm.push_back((int32_t)packed);
        out.pc.push_back((float)(first ? 2.0 * c : c));
      }
      int k = p - 1;
      while (k >= 0 && ++idx[k] == L) idx[k--] = 0;
      if (k < 0) break;
    }
    e.K = (int32_t)out.pm.size() - e.off;
    long double at = 1.0L / (two_pi * std::sqrt((long double)N) * (long double)sigma_r);
    long double fr = at - std::floor(at);
    long double sc = fr * 18446744073709551616.0L;
    e.qfix = sc >= 18446744073709551615.0L ? ~0ull : (uint64_t)sc;
    e.alpha_turn = (double)at;
    out.idx_of_T[T] = (int32_t)out.ent.size();
    seen[N] = (int32_t)out.ent.size();
    out.ent.push_back(e);
    if (e.K > out.K_max) out.K_max = e.K;
    if (N > out.N_max) out.N_max = N;
  }
  return true;
}

// ----------------------------------------------- polynomial range kernel ---
// Eq. (RPconv) of Section 1.3: phi(s) = (1 - s^2 / (2 N sigma_r^2))^N with the
// smallest N >= N0 = 0.5 (T/sigma_r)^2 (non-negative and monotone on
// [-T, T]).  As a polynomial of degree 2N in the neighbour's intensity a,
// phi(a - b) = sum_j c_j(b) T_j(x(a)) in the Chebyshev basis of
// x(a) = (a - L/2) / (L/2) on [0, L]: the shiftable form of Section 1.2 with
// basis functions T_j and coefficients c_j(b), one table row per integer
// intensity b.  Coefficients from the values at the 2N+1 Chebyshev points
// (the discrete cosine transform that is exact for degree <= 2N), long
// double.  Orders above J are dropped, J the smallest order with
// sum_{j > J} max_b |c_j(b)| <= eps, so that the kernel moves by at most eps
// anywhere on [0, L]^2 (|T_j| <= 1).
bool build_rp_table(double sigma_r, double eps, double L, double T, RpTable &out, std::string &err) {
  out = RpTable();
  const double n0 = 0.5 * (T / sigma_r) * (T / sigma_r);
  if (!(n0 <= 2048.0)) { err = "polynomial kernel order above 2048 (sigma_r too small for T)"; return false; }
  const int N = std::max(1, (int)std::ceil(n0));
  const int n = 2 * N + 1;  // nodes = coefficients
  const int nv = (int)L + 1;
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double K2 = 2.0L * N * (long double)sigma_r * (long double)sigma_r;
  const long double h = 0.5L * (long double)L;
  // cos(j theta_k), theta_k = pi (k + 1/2) / n, by k-major rows
  std::vector<long double> ct((size_t)n * n);
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++) ct[(size_t)k * n + j] = std::cos(pi * (long double)j * (k + 0.5L) / n);
  std::vector<double> c((size_t)nv * n);
  std::vector<long double> acc(n);
  for (int b = 0; b < nv; b++) {
    std::fill(acc.begin(), acc.end(), 0.0L);
    for (int k = 0; k < n; k++) {
      const long double a = h + h * ct[(size_t)k * n + 1];  // x_k = cos theta_k
      const long double d = a - (long double)b;
      const long double v = std::pow(1.0L - d * d / K2, (long double)N);
      const long double *row = &ct[(size_t)k * n];
      for (int j = 0; j < n; j++) acc[j] += v * row[j];
    }
    for (int j = 0; j < n; j++) c[(size_t)b * n + j] = (double)(acc[j] * (j ? 2.0L : 1.0L) / n);
  }
  std::vector<double> sup(n, 0.0);
  for (int b = 0; b < nv; b++)
    for (int j = 0; j < n; j++) sup[j] = std::max(sup[j], std::fabs(c[(size_t)b * n + j]));
  int J = n - 1;
  double tail = 0.0;
  while (J > 0 && tail + sup[J] <= eps) tail += sup[J--];
  out.N = N;
  out.J = J;
  out.K = (J + 2) / 2;  // slots of two orders: (2k, 2k+1)
  out.kappa = 0.0;
  for (int b = 0; b < nv; b++) {
    double sa = 0.0;
    for (int j = 0; j <= J; j++) sa += std::fabs(c[(size_t)b * n + j]);
    out.kappa = std::max(out.kappa, sa);
  }
  // per slot and intensity v (256 entries, v > L unused): the basis values
  // (T_2k, T_2k+1)(x(v)) and the coefficients (c_2k, c_2k+1)(v)
  out.gen.assign((size_t)out.K * 512, 0.f);
  out.comb.assign((size_t)out.K * 512, 0.f);
  for (int k = 0; k < out.K; k++)
    for (int v = 0; v < 256; v++) {
      const long double x = std::min(1.0L, std::max(-1.0L, ((long double)std::min(v, nv - 1) - h) / h));
      const long double th = std::acos(x);
      for (int u = 0; u < 2; u++) {
        const int j = 2 * k + u;
        const size_t o = ((size_t)k * 256 + v) * 2 + u;
        out.gen[o] = (float)std::cos((long double)j * th);
        out.comb[o] = (j <= J && v < nv) ? (float)c[(size_t)v * n + j] : 0.f;
      }
    }
  return true;
}

// ------------------------------------------------------------------ IIR ---
// Young & van Vliet (1995): q(sigma), then b0..b3; the denominator
// 1 - a1 z^-1 - a2 z^-2 - a3 z^-3 (a_i = b_i/b0) is factored into a real pole
// and a second-order section, which the kernels run in FP32.
bool yvv_cascade(double sigma, double &g1, double &g2, double &c1, double &c2, std::string &err) {
  if (!(sigma >= 0.5)) { err = "recursive Gaussian needs sigma_s >= 0.5"; return false; }
  double q = sigma >= 2.5 ? 0.98711 * sigma - 0.96330
                          : 3.97156 - 4.14554 * std::sqrt(1.0 - 0.26891 * sigma);
  double q2 = q * q, q3 = q2 * q;
  double b0 = 1.57825 + 2.44413 * q + 1.4281 * q2 + 0.422205 * q3;
  double a1 = (2.44413 * q + 2.85619 * q2 + 1.26661 * q3) / b0;
  double a2 = -(1.4281 * q2 + 1.26661 * q3) / b0;
  double a3 = (0.422205 * q3) / b0;
  // real root of z^3 - a1 z^2 - a2 z - a3 in (0, 1): bisection then Newton
  auto P = [&](double z) { return ((z - a1) * z - a2) * z - a3; };
  auto dP = [&](double z) { return (3.0 * z - 2.0 * a1) * z - a2; };
  double lo = 0.0, hi = 1.0;
  if (!(P(lo) < 0.0 && P(hi) > 0.0)) { err = "unexpected recursive filter poles"; return false; }
  for (int i = 0; i < 60; i++) {
    double mid = 0.5 * (lo + hi);
    (P(mid) < 0.0 ? lo : hi) = mid;
  }
  double p = 0.5 * (lo + hi);
  for (int i = 0; i < 4; i++) p -= P(p) / dP(p);
  c1 = a1 - p;
  c2 = p * c1 + a2;
  g1 = 1.0 - p;
  g2 = 1.0 - c1 - c2;
  if (std::fabs(p * c2 + a3) > 1e-9) { err = "recursive filter factorisation failed"; return false; }
  return true;
}

namespace {
struct M3 {
  double a[9];
};
M3 ident() { M3 m{}; m.a[0] = m.a[4] = m.a[8] = 1.0; return m; }
M3 mul(const M3 &x, const M3 &y) {
  M3 r{};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += x.a[i * 3 + k] * y.a[k * 3 + j];
      r.a[i * 3 + j] = s;
    }
  return r;
}
M3 mpow(const M3 &x, long e) {
  M3 r = ident(), b = x;
  while (e > 0) { if (e & 1) r = mul(r, b); b = mul(b, b); e >>= 1; }
  return r;
}
struct Casc {
  double g1, g2, c2;
  // one step of the cascade on state (s, w, d) with input x,
  // d = (w[n] - w[n-1]) / g2.  The first-order section runs without its input
  // gain g1 (s = (1-g1) s + x): each pass then scales its output by 1/g1, a
  // constant shared by every smoothed image that cancels in the ratio of
  // eqs. (f1), (f2).
  void step(double st[3], double x) const {
    double s = (1.0 - g1) * st[0] + x;
    double d = (s - st[1]) - c2 * st[2];
    st[1] = st[1] + g2 * d;
    st[2] = d;
    st[0] = s;
  }
};
void put(std::vector<float> &o, int off, const M3 &m) { for (int i = 0; i < 9; i++) o[off + i] = (float)m.a[i]; }

}  // namespace

bool build_iir_consts(double sigma_s, std::vector<float> &out, std::string &err) {
  double g1, g2, c1, c2;
  if (!yvv_cascade(sigma_s, g1, g2, c1, c2, err)) return false;
  Casc cs{g1, g2, c2};
  out.assign(kIirSize, 0.0f);
  out[kIirCoef + 0] = (float)(1.0 - g1);
  out[kIirCoef + 1] = (float)g2;
  out[kIirCoef + 2] = (float)c2;
  out[kIirCoef + 3] = (float)g1;  // the gain left out (not read by the kernels)
  // zero-input step of Casc as a matrix on (s, w, d)
  M3 A{};
  A.a[0] = 1.0 - g1;
  A.a[3] = g2 * (1.0 - g1); A.a[4] = 1.0 - g2; A.a[5] = -g2 * c2;
  A.a[6] = 1.0 - g1;        A.a[7] = -1.0;     A.a[8] = -c2;
  // zero-extension boundary: continue the causal recursion with zero input
  // past the end, run the anticausal recursion back from far away
  long L = (long)std::ceil(40.0 * sigma_s) + 64;
  std::vector<double> w(L);
  M3 mts{};
  for (int j = 0; j < 3; j++) {
    double st[3] = {0, 0, 0};
    st[j] = 1.0;
    for (long t = 0; t < L; t++) { cs.step(st, 0.0); w[t] = st[1]; }
    double q[3] = {0, 0, 0};
    for (long t = L - 1; t >= 0; t--) cs.step(q, w[t]);
    for (int r = 0; r < 3; r++) mts.a[r * 3 + j] = q[r];
  }
  put(out, kIirMts, mts);
  for (int c : {kCSmall, kCLarge}) {
    const int hb = c == kCSmall ? kIirHSmall : kIirHLarge;
    for (int v = 0; v <= c; v++) put(out, hb + iir_h_apow(c) + 9 * v, mpow(A, v));
    M3 Ac = mpow(A, c);
    for (int l = 0; l < 64; l++) put(out, hb + iir_h_lane(c) + 9 * l, mpow(Ac, l));
    for (int k = 0; k < 8; k++) put(out, hb + iir_h_scan(c) + 9 * k, mpow(Ac, 1L << k));
    put(out, hb + iir_h_wave(c), mpow(Ac, 64));
  }
  return true;
}

void build_fir_taps(double sigma_s, int R, std::vector<double> &taps) {
  taps.resize(2 * R + 1);
  for (int j = -R; j <= R; j++) taps[j + R] = std::exp(-(double)j * j / (2.0 * sigma_s * sigma_s));
}

}  // namespace bfi
