// Plan runtime and C ABI of libbf.so (declared in include/bf.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bf_device.h"
#include "bf_internal.h"

using namespace bfi;

namespace {

thread_local std::string g_detail;

bf_status fail(bf_status s, const std::string &why) {
  g_detail = why;
  return s;
}

bf_status dev_fail(hipError_t e, const char *what) {
  g_detail = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? BF_ERR_OUT_OF_MEMORY : BF_ERR_DEVICE;
}

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
};

// Everything one image needs on the device.
struct ImagePlan {
  bf_params p{};
  int R = 0;
  double range = 0.0;
  int32_t T_cap = 0;
  int32_t T_global = 0;    // GLOBAL mode: table index
  double T_global_raw = 0.0;
  Geom g{};
  OrderTable tab;
  int KC = 0;              // frequency pairs per launch of the blur passes
  int hpw = 0;             // term-group width knob of the recursive horizontal pass
  // workgroups the recursive vertical and horizontal passes aim for (pairs
  // per workgroup follow): kVWorkgroups / kHWorkgroups alone, the *Batch
  // values in a batch, whose grouped launches the other images fill
  int v_target = kVWorkgroups;
  int h_target = kHWorkgroups;
  int variant = BF_BLUR_IIR_F32;
  // device memory
  int32_t *d_idx = nullptr;
  OrderEntry *d_ent = nullptr;
  int32_t *d_pm = nullptr;
  float *d_pc = nullptr;
  float *d_iir = nullptr;
  float *d_taps = nullptr;  // Toeplitz path: FIR taps
  // polynomial range kernel: basis values and coefficients per pair slot and
  // intensity (NULL for the raised cosine)
  bool poly = false;
  float2 *d_rgen = nullptr, *d_rcomb = nullptr;
  // non-local means: patch samples per pixel (p >= 2), packed per pixel into
  // the workspace's patch image before the blur
  bool nlm = false;
  ToepCfg tc{};
  size_t z_per_pair = 0;    // workspace bytes of the smoothed images of one pair
  void *d_state = nullptr;  // T_used, flags, T_raw, q_nonpos
  // launch shape of bf_filter_noalloc, whose working memory is the fixed
  // static array: pairs per launch and offsets of the regions in it
  struct NoAlloc {
    bool ok = false;
    Geom g{};
    ToepCfg tc{};
    int KC = 0;
    size_t patch = 0, rowmax = 0, lut = 0, pq = 0, z = 0, end = 0;
  } na;
};

bool is_toeplitz(int v) { return v >= BF_BLUR_TOEPLITZ_F16 && v <= BF_BLUR_TOEPLITZ_BF16X2; }
bool is_split(int v) { return v == BF_BLUR_TOEPLITZ_F16X2 || v == BF_BLUR_TOEPLITZ_BF16X2; }

// Tile shape of the Toeplitz path for radius R: the tallest vertical tile
// (fewest recomputed halo rows) whose LDS leaves room for two workgroups per
// CU, else for one.  False when the band of 2R+1 taps does not fit.
bool toeplitz_shape(int variant, int R, int H, int lds_kb, ToepCfg &tc) {
  tc.R = R;
  tc.nks = (16 + 2 * R + 31) / 32;
  if (tc.nks > 8) return false;
  size_t pref = (size_t)kToepLdsMax / 2 - 2048;  // two workgroups per CU with their static tables
  if (const char *b = std::getenv("BF_TOEP_LDS_KB")) pref = (size_t)std::atoi(b) << 10;
  if (lds_kb > 0) pref = (size_t)lds_kb << 10;
  const int top = std::min(256, (H + 15) / 16 * 16);
  tc.rows = 0;
  for (size_t budget : {std::min(pref, (size_t)kToepDynMax), (size_t)kToepDynMax}) {
    for (int rows = top; rows >= 16 && !tc.rows; rows -= 16)
      if (toeplitz_v_lds(variant, rows, tc.nks) <= budget) tc.rows = rows;
    if (tc.rows) break;
  }
  if (tc.rows) {  // same tile count, least padding: spread the rows evenly over the tiles
    const int nty = (H + tc.rows - 1) / tc.rows;
    tc.rows = ((H + 15) / 16 + nty - 1) / nty * 16;
  }
  return tc.rows > 0 && toeplitz_h_lds(variant, tc.nks) <= (size_t)kToepDynMax;
}

size_t elem_size(bf_dtype d) { return d == BF_U8 ? 1 : (d == BF_U16 ? 2 : 4); }

// Largest sum of absolute Chebyshev coefficients (over the kept orders, worst
// intensity) a polynomial-kernel plan accepts: the FP32 sums of the smoothed
// images lose about that factor against their result.
constexpr double kRpKappaMax = 16.0;

// Size of the static working memory of bf_filter_noalloc (per device).
constexpr size_t kScratchBytes = (size_t)256 << 20;

}  // namespace

struct bf_plan_s {
  int device = 0;
  std::vector<ImagePlan> im;
  // workspace shared by the images of the plan (they run one after another)
  void *d_rowmax = nullptr;
  float4 *d_Z = nullptr;
  float2 *d_PQ = nullptr;
  float2 *d_lut = nullptr;  // cos/sin tables of the pairs in flight (8-bit inputs)
  void *d_patch = nullptr;  // non-local means: the patch image
  size_t rowmax_bytes = 0, Z_bytes = 0, PQ_bytes = 0, lut_bytes = 0, patch_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // stage timing (bf_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  hipEvent_t open_ev[BF_STAGE_COUNT] = {};
  double prof_ms[BF_STAGE_COUNT] = {};
  int64_t prof_n[BF_STAGE_COUNT] = {};
  StageRec rec;
  // graphs of the launch sequence, keyed by the image pointers they bake in
  struct GraphEntry { int img; const void *in; float *out; hipGraphExec_t exec; };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  bool use_graph = true;
  // batches: images on the Toeplitz path run as grouped launches (one launch
  // per stage for all of them), each in its own workspace region
  bool grouped = false;
  void *d_bws = nullptr;
  size_t bws_bytes = 0;
  std::vector<size_t> rowmax_off, z_off, pq_off, glut_off;
  struct BatchEntry {
    std::vector<const void *> in;
    std::vector<float *> out;
    hipGraphExec_t exec;
    void *d_args;
  };
  std::vector<BatchEntry> batches;
  void *d_eager_args = nullptr;  // argument arrays of batches launched directly
  size_t eager_args_bytes = 0;
};

namespace {

DevState state_at(void *d_state) {
  DevState st;
  char *b = (char *)d_state;
  st.T_used = (int32_t *)(b + 0);
  st.flags = (int32_t *)(b + 4);
  st.T_raw = (unsigned long long *)(b + 8);
  st.q_nonpos = (unsigned long long *)(b + 16);
  return st;
}
// d_state: the published state (24 bytes), then the range accumulators
// (top slot at 32, kRangeSubs slots from 48, then kRangeSubs lower bounds).
constexpr size_t kAccLbOff = 48 + kRangeSubs * sizeof(RangeAccSlot);
constexpr size_t kStateBytes = kAccLbOff + kRangeSubs * sizeof(unsigned long long);
RangeAcc acc_at(void *d_state) {
  char *b = (char *)d_state;
  return RangeAcc{(RangeAccSlot *)(b + 32), (RangeAccSlot *)(b + 48), (unsigned long long *)(b + kAccLbOff)};
}
DevState state_of(const ImagePlan &ip) { return state_at(ip.d_state); }
RangeAcc acc_of(const ImagePlan &ip) { return acc_at(ip.d_state); }

DevTables tables_of(const ImagePlan &ip) {
  DevTables t;
  t.idx_of_T = ip.d_idx;
  t.ent = ip.d_ent;
  t.pm = ip.d_pm;
  t.pc = ip.d_pc;
  t.T_cap = ip.T_cap;
  t.lut_gen = ip.d_rgen;
  t.lut_comb = ip.d_rcomb;
  return t;
}

bf_status check_params(const bf_params &p) {
  if (p.height < 1 || p.width < 1) return fail(BF_ERR_INVALID_ARG, "height and width must be >= 1");
  if (p.in_pitch < 0 || (p.in_pitch > 0 && p.in_pitch < p.width))
    return fail(BF_ERR_INVALID_ARG, "in_pitch must be 0 or >= width");
  if (p.out_pitch < 0 || (p.out_pitch > 0 && p.out_pitch < p.width))
    return fail(BF_ERR_INVALID_ARG, "out_pitch must be 0 or >= width");
  if (p.dtype != BF_U8 && p.dtype != BF_U16 && p.dtype != BF_F32)
    return fail(BF_ERR_INVALID_ARG, "unknown dtype");
  if (!(p.sigma_s > 0.0) || !std::isfinite(p.sigma_s)) return fail(BF_ERR_INVALID_ARG, "sigma_s must be > 0");
  if (!(p.sigma_r > 0.0) || !std::isfinite(p.sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be > 0");
  if (!(p.eps > 0.0 && p.eps < 1.0)) return fail(BF_ERR_INVALID_ARG, "eps must lie in (0, 1)");
  if (p.radius < 0) return fail(BF_ERR_INVALID_ARG, "radius must be >= 0");
  if (p.t_mode != BF_T_GLOBAL && p.t_mode != BF_T_LOCAL) return fail(BF_ERR_INVALID_ARG, "unknown t_mode");
  if (p.t_value < 0.0 || !std::isfinite(p.t_value)) return fail(BF_ERR_INVALID_ARG, "t_value must be >= 0");
  if (p.value_range < 0.0 || !std::isfinite(p.value_range))
    return fail(BF_ERR_INVALID_ARG, "value_range must be >= 0");
  if (p.blur < BF_BLUR_AUTO || p.blur > BF_BLUR_TOEPLITZ_BF16X2) return fail(BF_ERR_INVALID_ARG, "unknown blur");
  if (p.spatial != BF_SPATIAL_GAUSSIAN && p.spatial != BF_SPATIAL_BOX && p.spatial != BF_SPATIAL_GAUSSIAN_FIR)
    return fail(BF_ERR_INVALID_ARG, "unknown spatial kernel");
  if (p.range_kernel != BF_RANGE_RAISED_COSINE && p.range_kernel != BF_RANGE_POLYNOMIAL)
    return fail(BF_ERR_INVALID_ARG, "unknown range kernel");
  if (p.range_kernel == BF_RANGE_POLYNOMIAL && p.dtype != BF_U8)
    return fail(BF_ERR_UNSUPPORTED, "the polynomial range kernel takes 8-bit images");
  if (p.range_kernel == BF_RANGE_POLYNOMIAL && p.t_mode != BF_T_GLOBAL)
    return fail(BF_ERR_UNSUPPORTED, "the polynomial range kernel needs a global T");
  if (p.patch_size < 0 || p.patch_size > kNlmMaxPatch) return fail(BF_ERR_INVALID_ARG, "patch_size outside 0..4");
  if (p.patch_size >= 2) {
    if (p.patch_dy[0] != 0 || p.patch_dx[0] != 0)
      return fail(BF_ERR_INVALID_ARG, "the first patch sample must be the pixel itself (offset 0, 0)");
    for (int k = 1; k < p.patch_size; k++)
      if (std::abs(p.patch_dy[k]) > kNlmMaxOffset || std::abs(p.patch_dx[k]) > kNlmMaxOffset)
        return fail(BF_ERR_INVALID_ARG, "patch offsets must lie within +-2");
    if (p.dtype != BF_U8) return fail(BF_ERR_UNSUPPORTED, "non-local means takes 8-bit images");
    if (p.range_kernel != BF_RANGE_RAISED_COSINE)
      return fail(BF_ERR_UNSUPPORTED, "non-local means uses the raised-cosine range kernel");
    if (p.blur != BF_BLUR_TOEPLITZ_F16X2 && p.blur != BF_BLUR_TOEPLITZ_BF16X2)
      return fail(BF_ERR_UNSUPPORTED, "non-local means runs on the split Toeplitz blur variants");
  }
  if (p.spatial == BF_SPATIAL_BOX && p.blur == BF_BLUR_IIR_F32)
    return fail(BF_ERR_UNSUPPORTED, "the box spatial filter runs on the Toeplitz blur variants");
  if (p.spatial == BF_SPATIAL_GAUSSIAN_FIR && p.blur == BF_BLUR_IIR_F32)
    return fail(BF_ERR_UNSUPPORTED, "the sampled FIR Gaussian runs on the Toeplitz blur variants");
  return BF_OK;
}

// The discrete spatial operator an image is filtered with: the recursive
// Gaussian, or taps on the Toeplitz kernels (sampled Gaussian or box).  Fixed
// by the parameters alone; the autotuner only chooses among implementations
// of it.
bool fir_operator(const bf_params &p) {
  return p.spatial != BF_SPATIAL_GAUSSIAN || (p.blur != BF_BLUR_AUTO && p.blur != BF_BLUR_IIR_F32);
}

// Window radius R: the given radius, else ceil(3 sigma_s) for the Gaussian
// (Section 2) and round(sigma_s) for the box filter (whose sigma_s is its
// radius in Section 4).
int window_radius(const bf_params &p) {
  if (p.radius > 0) return p.radius;
  if (p.spatial == BF_SPATIAL_BOX) return std::max(1, (int)std::lround(p.sigma_s));
  return (int)std::ceil(3.0 * p.sigma_s);
}

// Every device allocation of a plan goes through here.  BF_FAIL_ALLOC set in
// the environment makes it fail before calling HIP (a test hook for the
// out-of-memory path).
bf_status dev_alloc(void **dst, size_t bytes, const char *what) {
  if (std::getenv("BF_FAIL_ALLOC")) {
    *dst = nullptr;
    return fail(BF_ERR_OUT_OF_MEMORY, std::string("allocation failure requested by BF_FAIL_ALLOC: ") + what);
  }
  hipError_t e = hipMalloc(dst, bytes);
  return e == hipSuccess ? BF_OK : dev_fail(e, what);
}

bf_status upload(void **dst, const void *src, size_t bytes) {
  bf_status st = dev_alloc(dst, bytes ? bytes : 16, "hipMalloc(table)");
  if (st) return st;
  hipError_t e;
  if (bytes) {
    e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return dev_fail(e, "hipMemcpy(table)");
  }
  return BF_OK;
}

// Per-image choices the autotuner makes (0 = default).
struct Knobs {
  int variant = 0;  // bf_blur other than AUTO
  int hchunk = 0;   // pixels per thread of the recursive horizontal pass (16 or 32)
  int lds_kb = 0;   // preferred LDS of a Toeplitz vertical tile
  int hpw = 0;      // term-group width of the recursive horizontal pass (pairs in
                    // flight per row): 0 the single-image rule, -1 the rule for a
                    // shared grouped launch, > 0 that width
};

// Launch shape of the blur passes for KC pairs per launch: the vertical
// pass's pairs per workgroup, the horizontal pass's pair groups (recursive
// path) or the Toeplitz pass's pair groups.
void set_chunk(ImagePlan &ip, int KC) {
  Geom &g = ip.g;
  ip.KC = KC;
  g.hgroups = 1;
  g.hkpg = KC;
  {
    // vertical pass: pairs per workgroup for about one round of workgroups
    const int ncb = (g.Spos + kHThreads / g.vS - 1) / (kHThreads / g.vS);
    const int gx = 8 * ((ncb + 7) / 8);
    int target = ip.v_target;
    if (const char *w = std::getenv("BF_V_WG")) target = std::max(1, std::atoi(w));
    const int groups = std::max(1, std::min(KC, (target + gx - 1) / gx));
    g.vppw = (KC + groups - 1) / groups;
  }
  g.hrows = 1;
  if (!is_toeplitz(ip.variant)) {
    // horizontal pass: a workgroup's NG = 256/S row groups take pw pairs at a
    // time on each of NG/pw rows (few pairs: several rows per workgroup
    // instead of idle groups).  The pairs of a launch are split over enough
    // groups of workgroups to fill the GPU (as many as with one row per
    // workgroup), each group a whole number of the pw pairs in flight.
    const int ng = kHThreads / g.S;
    int target = ip.h_target;
    if (const char *w = std::getenv("BF_H_WG")) target = std::max(1, std::atoi(w));
    const int groups = std::max(1, std::min((KC + ng - 1) / ng, (target + g.H - 1) / g.H));
    int pw = ng;
    if (ip.hpw > 0) {
      while (pw > ip.hpw) pw >>= 1;
    } else if (ip.hpw < 0) {
      // in a launch shared with other images, which fill the GPU: the
      // largest width whose last round leaves at most 1/8 of the slots idle
      while (pw > 1 && 8 * KC < 7 * ((KC + pw - 1) / pw * pw)) pw >>= 1;
    } else {
      // alone: the smallest rounds x waves of workgroups (resident: the
      // workgroups all CUs hold at once), so that fewer idle slots do not cost occupancy
      const int resident = 256 * (g.cC == kCSmall ? (ip.p.dtype == BF_F32 ? 2 : 3) : 1);
      long best = -1;
      for (int w = ng; w >= 1; w >>= 1) {
        const long nrb = (g.H + ng / w - 1) / (ng / w);
        const long rounds = (((KC + w - 1) / w) + groups - 1) / groups;
        const long t = rounds * ((nrb * groups + resident - 1) / resident);
        if (best < 0 || t < best) {
          best = t;
          pw = w;
        }
      }
    }
    g.hrows = ng / pw;
    const int slots = (KC + pw - 1) / pw;
    g.hkpg = (slots + groups - 1) / groups * pw;
    g.hgroups = (KC + g.hkpg - 1) / g.hkpg;
  } else {
    // split the pairs of a launch over enough horizontal workgroups to fill the GPU
    const int tiles = toeplitz_h_tiles(ip.variant, g.H, g.W);
    const int groups = std::max(1, std::min(KC, (2048 + tiles - 1) / tiles));
    ip.tc.kpg = (KC + groups - 1) / groups;
    ip.tc.groups = (KC + ip.tc.kpg - 1) / ip.tc.kpg;
  }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Device bytes of an image's range-stage workspace: the tile statistics of
// the one-launch kernel (one int2 per 32 x 32 tile), or the row maxima of the
// two passes (R > 48); none with a global T.
size_t range_ws_bytes(const ImagePlan &ip) {
  if (ip.p.t_mode != BF_T_LOCAL) return 0;
  if (range_tile_ok(ip.R, ip.p.dtype)) {
    const GroupGrid gt = range_tile_grid(ip.g);
    return (size_t)gt.gx * gt.gy * sizeof(int2);
  }
  return (size_t)ip.g.H * ip.g.W * elem_size(ip.p.dtype);
}

// Shape of bf_filter_noalloc for an image: the most pairs per launch whose
// working memory (device state, row maxima of the two-pass range stage,
// 8-bit cos/sin tables, partial sums, smoothed images) fits kScratchBytes.
// Leaves the plan's own launch shape as it was.
void noalloc_shape(ImagePlan &ip) {
  const Geom g0 = ip.g;
  const ToepCfg tc0 = ip.tc;
  const int KC0 = ip.KC;
  const size_t px = (size_t)g0.H * g0.W;
  const bool toep = is_toeplitz(ip.variant);
  const size_t state = align256(kStateBytes);
  const size_t rowmax = align256(range_ws_bytes(ip));
  const size_t patch = ip.nlm ? align256(px * sizeof(Patch8x4)) : 0;
  ImagePlan::NoAlloc na;
  auto fits = [&](int kc) {
    set_chunk(ip, kc);
    na.patch = state;
    na.rowmax = na.patch + patch;
    na.lut = na.rowmax + rowmax;
    na.pq = na.lut + (toep ? 0 : align256((size_t)kc * 256 * sizeof(float2)));
    na.z = na.pq + align256((size_t)(toep ? ip.tc.groups : ip.g.hgroups) * px * sizeof(float2));
    na.end = na.z + align256((size_t)kc * ip.z_per_pair);
    return na.end <= kScratchBytes;
  };
  const size_t fixed = state + patch + rowmax + align256(px * sizeof(float2));
  int kc = fixed >= kScratchBytes ? 1
                                  : (int)std::max<size_t>(1, std::min<size_t>((size_t)ip.tab.K_max,
                                                                              (kScratchBytes - fixed) / ip.z_per_pair));
  while (kc > 1 && !fits(kc)) kc = std::max(1, kc - std::max(1, kc / 8));
  na.ok = fits(kc);
  na.KC = kc;
  na.g = ip.g;
  na.tc = ip.tc;
  ip.na = na;
  ip.g = g0;
  ip.tc = tc0;
  ip.KC = KC0;
}

bf_status prepare_image(const bf_params &p, ImagePlan &ip, const Knobs &kn) {
  ip.p = p;
  ip.hpw = kn.hpw;
  const double full = p.dtype == BF_U16 ? 65535.0 : 255.0;
  ip.range = p.value_range > 0.0 ? p.value_range : full;
  if (p.dtype == BF_U8 && ip.range > 255.0) return fail(BF_ERR_INVALID_ARG, "value_range above 255 for u8");
  if (p.dtype == BF_U16 && ip.range > 65535.0) return fail(BF_ERR_INVALID_ARG, "value_range above 65535 for u16");
  const bool box = p.spatial == BF_SPATIAL_BOX;
  ip.R = window_radius(p);
  if (ip.R > 1024) return fail(BF_ERR_UNSUPPORTED, "radius above 1024");
  double Tg = p.t_value > 0.0 ? p.t_value : ip.range;
  double cap = std::ceil(ip.range);
  if (p.t_mode == BF_T_GLOBAL) cap = std::max(cap, std::ceil(Tg));
  if (cap > 4194304.0) return fail(BF_ERR_UNSUPPORTED, "value range above 2^22");
  ip.T_cap = (int32_t)cap;
  ip.T_global = (int32_t)std::ceil(Tg);
  ip.T_global_raw = Tg;
  const bool fir = fir_operator(p);
  int variant = kn.variant ? kn.variant
                           : (p.blur != BF_BLUR_AUTO ? p.blur : (fir ? BF_BLUR_TOEPLITZ_F16X2 : BF_BLUR_IIR_F32));
  ip.variant = variant;
  if (fir != is_toeplitz(variant))
    return fail(BF_ERR_UNSUPPORTED, "blur variant does not implement the requested spatial operator");
  if (!is_toeplitz(variant) && (p.width > kMaxWidth || p.height > kMaxWidth))
    return fail(BF_ERR_UNSUPPORTED, "width or height above 8192 for the recursive blur");
  if (is_toeplitz(variant) && !toeplitz_shape(variant, ip.R, p.height, kn.lds_kb, ip.tc))
    return fail(BF_ERR_UNSUPPORTED, "radius above 120 for the Toeplitz blur");
  std::string err;
  RpTable rt;
  ip.poly = p.range_kernel == BF_RANGE_POLYNOMIAL;
  if (ip.poly) {
    // one entry for the plan's global T: pair slots of two Chebyshev orders,
    // unit weights (the coefficients sit in the per-intensity table)
    if (!build_rp_table(p.sigma_r, p.eps, ip.range, Tg, rt, err)) return fail(BF_ERR_UNSUPPORTED, err);
    if (rt.kappa > kRpKappaMax)
      return fail(BF_ERR_UNSUPPORTED, "polynomial kernel: the Chebyshev coefficients sum to " +
                                          std::to_string(rt.kappa) + " (T far below value_range), FP32 sums would cancel");
    OrderTable &t = ip.tab;
    t = OrderTable();
    t.T_cap = ip.T_cap;
    t.idx_of_T.assign((size_t)ip.T_cap + 1, 0);
    OrderEntry oe{};
    oe.N = rt.N;
    oe.M = rt.J;
    oe.K = rt.K;
    oe.off = 0;
    t.ent.push_back(oe);
    t.pm.assign(rt.K, 0);
    t.pc.assign(rt.K, 1.0f);
    t.K_max = rt.K;
    t.N_max = rt.N;
  } else if (p.patch_size >= 2) {
    ip.nlm = true;
    if (!build_nlm_table(p.sigma_r, p.eps, ip.range, ip.T_cap, p.patch_size, ip.tab, err))
      return fail(BF_ERR_UNSUPPORTED, err);
  } else if (!build_order_table(p.sigma_r, p.eps, ip.range, ip.T_cap, ip.tab, err)) {
    return fail(BF_ERR_UNSUPPORTED, err);
  }
  std::vector<float> iir, taps;
  if (is_toeplitz(variant)) {
    std::vector<double> t;
    if (box) t.assign(2 * ip.R + 1, 1.0);  // the constant filter: unit taps
    else build_fir_taps(p.sigma_s, ip.R, t);
    taps.assign(t.begin(), t.end());
  } else if (!build_iir_consts(p.sigma_s, iir, err)) {
    return fail(BF_ERR_INVALID_ARG, err);
  }
  // geometry
  Geom &g = ip.g;
  g.H = p.height;
  g.W = p.width;
  g.pitch = p.in_pitch > 0 ? p.in_pitch : p.width;
  g.opitch = p.out_pitch > 0 ? p.out_pitch : p.width;
  // pixels per thread of the horizontal pass: the smaller chunk needs fewer
  // registers (more waves in flight) but twice the scan steps per pixel
  int cC = kCSmall;
  if (const char *c = std::getenv("BF_HCHUNK")) cC = std::atoi(c) == kCLarge ? kCLarge : kCSmall;
  if (kn.hchunk) cC = kn.hchunk == kCLarge ? kCLarge : kCSmall;
  if (g.W > kCSmall * kHThreads) cC = kCLarge;
  int S = 1, logS = 0;
  while (S * cC < g.W) { S <<= 1; logS++; }
  g.S = S;
  g.logS = logS;
  g.cC = cC;
  // positions: whole chunks only; the row group's remaining threads (a
  // power of two in all) hold no positions and smooth zeros, so neither the
  // vertical pass nor the smoothed images carry the padding of the group
  g.Seff = (g.W + cC - 1) / cC;
  g.Spos = g.Seff * cC;
  // vertical pass: one row group per column, kCLarge rows per thread; float
  // input (whose phases are computed per sample, not read from a table)
  // kCSmall up to 4096 rows: half the registers, three waves per SIMD
  // instead of two to hide the sine/cosine and scan latencies (4096² float:
  // 2.05 -> 1.40 ms; for 8- and 16-bit input the extra scan level costs more
  // than the waves gain: 512² 53 -> 58 µs, 2048² 3.79 -> 4.63 ms).
  // BF_VCHUNK=16/32 overrides.
  g.vC = (p.dtype == BF_F32 && g.H <= kCSmall * kHThreads) ? kCSmall : kCLarge;
  if (const char *c = std::getenv("BF_VCHUNK")) {
    if (std::atoi(c) == kCSmall && g.H <= kCSmall * kHThreads) g.vC = kCSmall;
    if (std::atoi(c) == kCLarge) g.vC = kCLarge;
  }
  g.vS = 1;
  while (g.vS * g.vC < g.H) g.vS <<= 1;
  // a vertical workgroup covers 256 / vS columns; the smoothed images are
  // stored in tiles whose row in a workgroup's columns holds
  // z_tile_words(vS) elements
  g.zlog = 0;
  while ((kHThreads / g.vS) << g.zlog < z_tile_words(g.vS)) g.zlog++;
  g.Hz = (g.H + (1 << g.zlog) - 1) >> g.zlog << g.zlog;
  g.center = (float)(0.5 * ip.range);
  if (!(g.center > 0.f)) return fail(BF_ERR_INVALID_ARG, "value_range too small");
  g.padl = ip.R & 7;
  g.zpitch = ((int64_t)g.W + g.padl + 7) / 8 * 8;
  // device tables
  bf_status st;
  if ((st = upload((void **)&ip.d_idx, ip.tab.idx_of_T.data(), ip.tab.idx_of_T.size() * 4))) return st;
  if ((st = upload((void **)&ip.d_ent, ip.tab.ent.data(), ip.tab.ent.size() * sizeof(OrderEntry)))) return st;
  if ((st = upload((void **)&ip.d_pm, ip.tab.pm.data(), ip.tab.pm.size() * 4))) return st;
  if ((st = upload((void **)&ip.d_pc, ip.tab.pc.data(), ip.tab.pc.size() * 4))) return st;
  if ((st = upload((void **)&ip.d_iir, iir.data(), iir.size() * 4))) return st;
  if ((st = upload((void **)&ip.d_taps, taps.data(), taps.size() * 4))) return st;
  if (ip.poly) {
    if ((st = upload((void **)&ip.d_rgen, rt.gen.data(), rt.gen.size() * 4))) return st;
    if ((st = upload((void **)&ip.d_rcomb, rt.comb.data(), rt.comb.size() * 4))) return st;
  }
  ip.tc.taps = ip.d_taps;
  {
    // the range accumulator and counter must start at zero
    const std::vector<unsigned char> zero(kStateBytes, 0);
    if ((st = upload(&ip.d_state, zero.data(), zero.size()))) return st;
  }
  // pairs per launch: bounded by a workspace budget for the smoothed images
  size_t per_pair = (size_t)g.Hz * g.Spos * sizeof(float4);
  if (is_toeplitz(variant)) per_pair = (size_t)4 * g.H * g.zpitch * (is_split(variant) ? 4 : 2);
  ip.z_per_pair = per_pair;
  size_t budget = (size_t)64 << 30;
  if (const char *b = std::getenv("BF_Z_BUDGET_MB")) budget = (size_t)std::atoll(b) << 20;
  size_t kc = budget / per_pair;
  if (kc < 1) kc = 1;
  set_chunk(ip, (int)std::min<size_t>(std::min<size_t>(kc, (size_t)ip.tab.K_max), 65535));
  noalloc_shape(ip);
  if (is_toeplitz(variant)) {
    hipError_t he = toeplitz_setup();
    if (he != hipSuccess) return dev_fail(he, "Toeplitz LDS attributes");
  }
  return BF_OK;
}

void free_image(ImagePlan &ip) {
  (void)hipFree(ip.d_idx);
  (void)hipFree(ip.d_ent);
  (void)hipFree(ip.d_pm);
  (void)hipFree(ip.d_pc);
  (void)hipFree(ip.d_iir);
  (void)hipFree(ip.d_taps);
  (void)hipFree(ip.d_rgen);
  (void)hipFree(ip.d_rcomb);
  (void)hipFree(ip.d_state);
}

bf_status ensure(void **ptr, size_t &have, size_t need) {
  if (need <= have) return BF_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  have = 0;
  bf_status st = dev_alloc(ptr, need, "hipMalloc(workspace)");
  if (st) return st;
  have = need;
  return BF_OK;
}

hipEvent_t take_event(bf_plan_s *pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void stage_mark(void *ctx, int stage, hipStream_t s, bool end) {
  bf_plan_s *pl = (bf_plan_s *)ctx;
  if (!end) {
    hipEvent_t e = take_event(pl);
    if (e && hipEventRecord(e, s) == hipSuccess) pl->open_ev[stage] = e;
    return;
  }
  hipEvent_t a = pl->open_ev[stage];
  pl->open_ev[stage] = nullptr;
  if (!a) return;
  hipEvent_t b = take_event(pl);
  if (!b || hipEventRecord(b, s) != hipSuccess) {
    pl->ev_pool.push_back(a);
    return;
  }
  pl->pending.push_back({stage, a, b});
}

// Working memory of one image's launch sequence: the row maxima of the
// two-pass range stage, the smoothed images of the pairs of a launch, the
// pair groups' partial sums and the 8-bit cos/sin tables of the pairs.
struct Workspace {
  void *rowmax;
  float4 *Z;
  float2 *PQ;
  float2 *lut;
  void *patch;  // non-local means: H x W packed patch samples
};
// Launch shape of one image: geometry, Toeplitz configuration, pairs per
// launch and the device state (T, flags, range accumulators) it runs with.
struct Shape {
  const Geom *g;
  const ToepCfg *tc;
  int KC;
  void *d_state;
};
bf_status run_image_ws(const Workspace &ws, const StageRec &rec, const ImagePlan &ip, const Shape &sh,
                       const void *d_in, float *d_out, hipStream_t s);
bf_status run_image(bf_plan_s *pl, ImagePlan &ip, const void *d_in, float *d_out, hipStream_t s) {
  return run_image_ws(Workspace{pl->d_rowmax, pl->d_Z, pl->d_PQ, pl->d_lut, pl->d_patch}, pl->rec, ip,
                      Shape{&ip.g, &ip.tc, ip.KC, ip.d_state}, d_in, d_out, s);
}

// Launch image img through a captured graph of its kernel sequence.  The
// graph is captured once per (image, input, output) on a private stream and
// replayed on the caller's stream; the sequence has kernels only.
bf_status run_image_graph(bf_plan_s *pl, int img, const void *d_in, float *d_out, hipStream_t s) {
  for (auto &g : pl->graphs)
    if (g.img == img && g.in == d_in && g.out == d_out) {
      hipError_t e = hipGraphLaunch(g.exec, s);
      return e == hipSuccess ? BF_OK : dev_fail(e, "hipGraphLaunch");
    }
  hipError_t e;
  if (!pl->cap_stream) {
    e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return dev_fail(e, "hipStreamCreate");
  }
  e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return dev_fail(e, "hipStreamBeginCapture");
  bf_status st = run_image(pl, pl->im[img], d_in, d_out, pl->cap_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(pl->cap_stream, &graph);
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return dev_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return dev_fail(e, "hipGraphInstantiate");
  if (pl->graphs.size() >= 16) {
    (void)hipGraphExecDestroy(pl->graphs.front().exec);
    pl->graphs.erase(pl->graphs.begin());
  }
  pl->graphs.push_back({img, d_in, d_out, exec});
  e = hipGraphLaunch(exec, s);
  return e == hipSuccess ? BF_OK : dev_fail(e, "hipGraphLaunch");
}

// Enqueue the whole of Algorithm 2 for one image.
bf_status run_image_ws(const Workspace &ws, const StageRec &rec, const ImagePlan &ip, const Shape &sh,
                       const void *d_in, float *d_out, hipStream_t s) {
  const Geom &g = *sh.g;
  const int KC = sh.KC;
  DevState st = state_at(sh.d_state);
  DevTables tab = tables_of(ip);
  hipError_t e;
  if (ip.p.t_mode == BF_T_LOCAL) {
    e = launch_range(s, ip.p.dtype, d_in, g, ip.R, ws.rowmax, st, acc_at(sh.d_state), ip.T_cap, rec);
    if (e != hipSuccess) return dev_fail(e, "dynamic range");
  } else {
    e = launch_reset(s, st, ip.T_global, ip.T_global_raw);
    if (e != hipSuccess) return dev_fail(e, "reset");
  }
  const int Kmax = ip.tab.K_max;
  if (ip.nlm) {
    // the patch samples of every pixel, then the blur of the multi-index
    // terms reads the packed words in place of the image
    PatchArgs pa{(const uint8_t *)d_in, g.pitch, g.H, g.W, ip.p.patch_size, {}, {}, (Patch8x4 *)ws.patch};
    for (int k = 0; k < kNlmMaxPatch; k++) {
      pa.dy[k] = k < ip.p.patch_size ? ip.p.patch_dy[k] : 0;
      pa.dx[k] = k < ip.p.patch_size ? ip.p.patch_dx[k] : 0;
    }
    e = launch_patch_pack(s, pa);
    if (e != hipSuccess) return dev_fail(e, "patch samples");
    Geom gp = g;
    gp.pitch = g.W;
    for (int k0 = 0; k0 < Kmax; k0 += KC) {
      const int kcount = std::min(KC, Kmax - k0);
      e = launch_toeplitz_chunk(s, kDtPatch, ip.variant, ws.patch, d_out, gp, tab, st, *sh.tc, k0, kcount, ws.Z,
                                ws.PQ, k0 == 0, k0 + KC >= Kmax, rec);
      if (e != hipSuccess) return dev_fail(e, "Toeplitz blur (non-local means)");
    }
    return BF_OK;
  }
  if (is_toeplitz(ip.variant)) {
    for (int k0 = 0; k0 < Kmax; k0 += KC) {
      const int kcount = std::min(KC, Kmax - k0);
      e = launch_toeplitz_chunk(s, ip.p.dtype, ip.variant, d_in, d_out, g, tab, st, *sh.tc, k0, kcount, ws.Z,
                                ws.PQ, k0 == 0, k0 + KC >= Kmax, rec);
      if (e != hipSuccess) return dev_fail(e, "Toeplitz blur");
    }
    return BF_OK;
  }
  for (int k0 = 0; k0 < Kmax; k0 += KC) {
    const int kcount = std::min(KC, Kmax - k0);
    e = launch_iir_chunk(s, ip.p.dtype, d_in, d_out, g, tab, st, ip.d_iir, k0, kcount, ws.Z, ws.PQ, k0 == 0,
                         k0 + KC >= Kmax, ws.lut, rec);
    if (e != hipSuccess) return dev_fail(e, "blur");
  }
  return BF_OK;
}

// Whether an image of the plan runs inside the grouped launches of a batch
// (all its pairs in one launch).
bool in_group(const bf_plan_s *pl, const ImagePlan &ip) { return pl->grouped && ip.KC == ip.tab.K_max && !ip.nlm; }

// Host image of the argument arrays of one batch, packed for one upload.
struct ArgPack {
  std::vector<unsigned char> buf;
  template <typename T>
  size_t add(const std::vector<T> &v) {
    const size_t off = (buf.size() + 255) / 256 * 256;
    buf.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

// Block starts of a grouped launch from the per-image block counts.
std::vector<int> starts_of(const std::vector<int> &blocks) {
  std::vector<int> st(blocks.size() + 1, 0);
  for (size_t i = 0; i < blocks.size(); i++) st[i + 1] = st[i] + blocks[i];
  return st;
}

// The grouped launches of a batch: offsets of their argument arrays in the
// packed buffer, block totals and LDS sizes.
struct GLaunch {
  int kind;  // 0 reset, 1 range, 2 Toeplitz stages, 3 recursive vertical, 4 recursive horizontal,
            // 5 one-launch range, 6 its tile statistics
  bf_dtype dt;
  int variant;
  int S, cC;
  int cnt;
  size_t o[10];
  int t[5];
  size_t lds[2];
};
struct BatchPlan {
  ArgPack pack;
  std::vector<GLaunch> launches;
};

// Host side of a batch over images [0, n): the Toeplitz images grouped by
// dtype and variant (their range stage by dtype and column-pass kind).
void build_batch(bf_plan_s *pl, int n, const void *const *d_in, float *const *d_out, BatchPlan &bp) {
  std::vector<int> gidx;
  for (int i = 0; i < n; i++)
    if (in_group(pl, pl->im[i])) gidx.push_back(i);
  if (gidx.empty()) return;
  {
    std::vector<ResetArgs> ra;
    std::vector<int> blocks;
    for (int i : gidx) {
      const ImagePlan &ip = pl->im[i];
      const bool loc = ip.p.t_mode == BF_T_LOCAL;
      if (loc && range_tile_ok(ip.R, ip.p.dtype)) continue;  // the tile kernel resets its own state
      ra.push_back(ResetArgs{GroupGrid{1, 1, 1}, state_of(ip), loc ? 0 : ip.T_global, loc ? 0.0 : ip.T_global_raw});
      blocks.push_back(1);
    }
    if (!ra.empty()) {
      const std::vector<int> st = starts_of(blocks);
      GLaunch L{};
      L.kind = 0;
      L.cnt = (int)ra.size();
      L.o[0] = bp.pack.add(ra);
      L.o[1] = bp.pack.add(st);
      L.t[0] = st.back();
      bp.launches.push_back(L);
    }
  }
  for (bf_dtype dt : {BF_U8, BF_U16, BF_F32}) {
    // the tile statistics of every tile-kernel image of this dtype (one
    // workgroup per strip of tiles), then one tile launch per staged-block size
    auto tile_args = [&](int kr, std::vector<RangeTileArgs> &ta) {
      for (int i : gidx) {
        const ImagePlan &ip = pl->im[i];
        if (ip.p.t_mode != BF_T_LOCAL || ip.p.dtype != dt || !range_tile_ok(ip.R, dt) ||
            (kr && range_tile_kr(ip.R) != kr))
          continue;
        ta.push_back(RangeTileArgs{range_tile_grid(ip.g), d_in[i], ip.g.pitch, ip.g.H, ip.g.W, ip.R, state_of(ip),
                                   acc_of(ip), ip.T_cap, (int2 *)((char *)pl->d_bws + pl->rowmax_off[i]), 0});
      }
    };
    std::vector<RangeTileArgs> sa;
    tile_args(0, sa);
    if (sa.empty()) continue;
    {
      std::vector<int> sb;
      for (const RangeTileArgs &t : sa) {
        const GroupGrid gs = range_stats_grid(t.gg);
        sb.push_back(gs.gx * gs.gy);
      }
      const std::vector<int> ss = starts_of(sb);
      GLaunch L{};
      L.kind = 6;
      L.dt = dt;
      L.cnt = (int)sa.size();
      L.o[0] = bp.pack.add(sa);
      L.o[1] = bp.pack.add(ss);
      L.t[0] = ss.back();
      bp.launches.push_back(L);
    }
    // 8- and 16-bit input: one tile launch for all of them, staged for the
    // largest block size among them (few tiles are computed once the
    // statistics let the rest be skipped, so the larger staging of the
    // R <= 32 images costs less than a second launch).  Float input: one
    // launch per block size (its R > 32 kernel reads the rows from memory
    // and assumes R > 32).
    int kr_all = 32;
    for (const RangeTileArgs &t : sa) kr_all = std::max(kr_all, range_tile_kr(t.R));
    for (int kr : {32, 48}) {
      if (dt != BF_F32 && kr != kr_all) continue;
      std::vector<RangeTileArgs> ta;
      tile_args(dt == BF_F32 ? kr : 0, ta);
      if (ta.empty()) continue;
      size_t lds = 0;
      for (const RangeTileArgs &t : ta) lds = std::max(lds, range_tile_lds(t.R, dt, kr));
      long long total = 0;
      for (const RangeTileArgs &t : ta) total += t.gg.gx * t.gg.gy;
      std::vector<int> wb;
      for (RangeTileArgs &t : ta) {
        t.nwg = range_tile_wgs(t.gg.gx * t.gg.gy, total);
        wb.push_back(t.nwg);
      }
      const std::vector<int> ws = starts_of(wb);
      GLaunch L{};
      L.kind = 5;
      L.dt = dt;
      L.S = kr;
      L.cnt = (int)ta.size();
      L.o[0] = bp.pack.add(ta);
      L.o[1] = bp.pack.add(ws);
      L.t[0] = ws.back();
      L.lds[0] = lds;
      bp.launches.push_back(L);
    }
  }
  for (bf_dtype dt : {BF_U8, BF_U16, BF_F32}) {
    std::vector<RowmaxArgs> ra;
    std::vector<ColmaxArgs> ca;
    std::vector<int> rb, cb;
    for (int i : gidx) {
      const ImagePlan &ip = pl->im[i];
      if (ip.p.t_mode != BF_T_LOCAL || ip.p.dtype != dt || range_tile_ok(ip.R, dt)) continue;
      void *rm = (char *)pl->d_bws + pl->rowmax_off[i];
      const GroupGrid gr = range_row_grid(ip.g), gc = range_col_grid(ip.g);
      ra.push_back(RowmaxArgs{gr, d_in[i], ip.g.pitch, ip.g.H, ip.g.W, ip.R, rm, state_of(ip)});
      ca.push_back(ColmaxArgs{gc, d_in[i], ip.g.pitch, rm, ip.g.H, ip.g.W, ip.R, state_of(ip), ip.T_cap});
      rb.push_back(gr.gx * gr.gy);
      cb.push_back(gc.gx * gc.gy);
    }
    if (ra.empty()) continue;
    const std::vector<int> rs = starts_of(rb), cs = starts_of(cb);
    GLaunch L{};
    L.kind = 1;
    L.dt = dt;
    L.cnt = (int)ra.size();
    L.o[0] = bp.pack.add(ra);
    L.o[1] = bp.pack.add(rs);
    L.o[2] = bp.pack.add(ca);
    L.o[3] = bp.pack.add(cs);
    L.t[0] = rs.back();
    L.t[1] = cs.back();
    bp.launches.push_back(L);
  }
  for (bf_dtype dt : {BF_U8, BF_U16, BF_F32})
    for (int v = BF_BLUR_TOEPLITZ_F16; v <= BF_BLUR_TOEPLITZ_BF16X2; v++) {
      std::vector<ToepVArgs> va;
      std::vector<ToepHArgs> ha;
      std::vector<FinishArgs> fa;
      std::vector<int> vb, hb, fb;
      size_t vl = 0, hl = 0;
      for (int i : gidx) {
        const ImagePlan &ip = pl->im[i];
        if (ip.p.dtype != dt || ip.variant != v) continue;
        ToepVArgs a;
        ToepHArgs b;
        FinishArgs c;
        toeplitz_args(v, d_in[i], d_out[i], ip.g, tables_of(ip), state_of(ip), ip.tc, 0, ip.tab.K_max,
                      (char *)pl->d_bws + pl->z_off[i], (float2 *)((char *)pl->d_bws + pl->pq_off[i]), true, true,
                      a, b, c);
        va.push_back(a);
        ha.push_back(b);
        fa.push_back(c);
        vb.push_back(a.gg.gx * a.gg.gy);
        hb.push_back(b.gg.gx * b.gg.gy);
        fb.push_back(b.finish ? 0 : c.gg.gx);
        vl = std::max(vl, toeplitz_v_lds(v, ip.tc.rows, ip.tc.nks));
        hl = std::max(hl, toeplitz_h_lds(v, ip.tc.nks));
      }
      if (va.empty()) continue;
      const std::vector<int> vs = starts_of(vb), hs = starts_of(hb), fs = starts_of(fb);
      GLaunch L{};
      L.kind = 2;
      L.dt = dt;
      L.variant = v;
      L.cnt = (int)va.size();
      L.o[0] = bp.pack.add(va);
      L.o[1] = bp.pack.add(vs);
      L.o[2] = bp.pack.add(ha);
      L.o[3] = bp.pack.add(hs);
      L.o[4] = bp.pack.add(fa);
      L.o[5] = bp.pack.add(fs);
      L.t[0] = vs.back();
      L.t[1] = hs.back();
      L.t[2] = fs.back();
      L.lds[0] = vl;
      L.lds[1] = hl;
      bp.launches.push_back(L);
    }
  // recursive images: every vertical pass (grouped by dtype, threads per column
  // and chunk), then every horizontal pass (by dtype, threads per row, chunk)
  for (int pass = 0; pass < 2; pass++)
    for (bf_dtype dt : {BF_U8, BF_U16, BF_F32})
      for (int cC : {kCSmall, kCLarge})
        for (int S = 1; S <= kHThreads; S <<= 1) {
          std::vector<IirArgs> ar;
          std::vector<FinishArgs> fa;
          std::vector<int> nb, fb;
          for (int i : gidx) {
            const ImagePlan &ip = pl->im[i];
            if (is_toeplitz(ip.variant) || ip.p.dtype != dt) continue;
            if (pass == 0 ? (ip.g.vC != cC || ip.g.vS != S) : (ip.g.cC != cC || ip.g.S != S)) continue;
            char *ws = (char *)pl->d_bws;
            IirArgs a[2];
            FinishArgs c;
            iir_args(d_in[i], d_out[i], ip.g, tables_of(ip), state_of(ip), ip.d_iir, 0, ip.tab.K_max,
                     (float4 *)(ws + pl->z_off[i]), (float2 *)(ws + pl->pq_off[i]), true, true,
                     (float2 *)(ws + pl->glut_off[i]), a, c);
            ar.push_back(a[pass]);
            nb.push_back(a[pass].gg.gx * a[pass].gg.gy * a[pass].gg.gz);
            fa.push_back(c);
            fb.push_back(pass == 1 && ip.g.hgroups > 1 ? c.gg.gx : 0);
          }
          if (ar.empty()) continue;
          GLaunch L{};
          L.kind = 3 + pass;
          L.dt = dt;
          L.S = S;
          L.cC = cC;
          L.cnt = (int)ar.size();
          const std::vector<int> st = starts_of(nb), fs = starts_of(fb);
          L.o[0] = bp.pack.add(ar);
          L.o[1] = bp.pack.add(st);
          L.t[0] = st.back();
          L.o[2] = bp.pack.add(fa);
          L.o[3] = bp.pack.add(fs);
          L.t[1] = fs.back();
          bp.launches.push_back(L);
        }
}

// Device side of a batch: the grouped launches (their arguments already in
// d_args) and then the launch sequences of the images outside the groups.
// Kernels only, so it may run under stream capture.
bf_status enqueue_batch(bf_plan_s *pl, int n, const void *const *d_in, float *const *d_out, const BatchPlan &bp,
                        const char *d_args, hipStream_t s) {
  for (const GLaunch &L : bp.launches) {
    hipError_t e;
    if (L.kind == 0) {
      e = launch_reset_group(s, (const ResetArgs *)(d_args + L.o[0]), (const int *)(d_args + L.o[1]), L.t[0], L.cnt);
    } else if (L.kind == 6) {
      pl->rec.begin(BF_STAGE_RANGE, s);
      e = launch_range_stats_group(s, L.dt, (const RangeTileArgs *)(d_args + L.o[0]), (const int *)(d_args + L.o[1]),
                                   L.t[0], L.cnt);
      pl->rec.end(BF_STAGE_RANGE, s);
    } else if (L.kind == 5) {
      pl->rec.begin(BF_STAGE_RANGE, s);
      e = launch_range_tile_group(s, L.dt, L.S, (const RangeTileArgs *)(d_args + L.o[0]),
                                  (const int *)(d_args + L.o[1]), L.t[0], L.cnt, L.lds[0]);
      pl->rec.end(BF_STAGE_RANGE, s);
    } else if (L.kind == 1) {
      pl->rec.begin(BF_STAGE_RANGE, s);
      e = launch_range_group(s, L.dt, (const RowmaxArgs *)(d_args + L.o[0]), (const int *)(d_args + L.o[1]),
                             L.t[0], (const ColmaxArgs *)(d_args + L.o[2]), (const int *)(d_args + L.o[3]), L.t[1],
                             L.cnt);
      pl->rec.end(BF_STAGE_RANGE, s);
    } else if (L.kind == 3) {
      e = launch_iir_v_group(s, L.dt, L.S, L.cC, (const IirArgs *)(d_args + L.o[0]), (const int *)(d_args + L.o[1]),
                             L.cnt, L.t[0], pl->rec);
    } else if (L.kind == 4) {
      e = launch_iir_h_group(s, L.dt, L.S, L.cC, (const IirArgs *)(d_args + L.o[0]), (const int *)(d_args + L.o[1]),
                             L.cnt, L.t[0], (const FinishArgs *)(d_args + L.o[2]), (const int *)(d_args + L.o[3]),
                             L.t[1], pl->rec);
    } else {
      const ToepGroup tg{L.cnt,
                         (const ToepVArgs *)(d_args + L.o[0]), (const int *)(d_args + L.o[1]), L.t[0], L.lds[0],
                         (const ToepHArgs *)(d_args + L.o[2]), (const int *)(d_args + L.o[3]), L.t[1], L.lds[1],
                         (const FinishArgs *)(d_args + L.o[4]), (const int *)(d_args + L.o[5]), L.t[2]};
      e = launch_toeplitz_group(s, L.dt, L.variant, tg, pl->rec);
    }
    if (e != hipSuccess) return dev_fail(e, "grouped launch");
  }
  for (int i = 0; i < n; i++) {
    if (in_group(pl, pl->im[i])) continue;
    bf_status st = run_image(pl, pl->im[i], d_in[i], d_out[i], s);
    if (st) return st;
  }
  return BF_OK;
}

// A batch launched directly: arguments go to the plan's buffer once the
// stream has finished with its previous contents.
bf_status run_batch_eager(bf_plan_s *pl, int n, const void *const *d_in, float *const *d_out, hipStream_t s) {
  BatchPlan bp;
  build_batch(pl, n, d_in, d_out, bp);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
  bf_status st = ensure(&pl->d_eager_args, pl->eager_args_bytes, std::max<size_t>(bp.pack.buf.size(), 256));
  if (st) return st;
  if (!bp.pack.buf.empty()) {
    e = hipMemcpy(pl->d_eager_args, bp.pack.buf.data(), bp.pack.buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return dev_fail(e, "hipMemcpy(batch arguments)");
  }
  return enqueue_batch(pl, n, d_in, d_out, bp, (const char *)pl->d_eager_args, s);
}

// The whole batch through one captured graph, cached per set of pointers;
// the graph owns a private copy of the argument arrays.
bf_status run_batch_graph(bf_plan_s *pl, int n, const void *const *d_in, float *const *d_out, hipStream_t s) {
  for (auto &b : pl->batches) {
    if ((int)b.in.size() != n) continue;
    bool same = true;
    for (int i = 0; i < n && same; i++) same = b.in[i] == d_in[i] && b.out[i] == d_out[i];
    if (!same) continue;
    hipError_t e = hipGraphLaunch(b.exec, s);
    return e == hipSuccess ? BF_OK : dev_fail(e, "hipGraphLaunch");
  }
  BatchPlan bp;
  build_batch(pl, n, d_in, d_out, bp);
  void *d_args = nullptr;
  bf_status ast = dev_alloc(&d_args, std::max<size_t>(bp.pack.buf.size(), 256), "hipMalloc(batch arguments)");
  if (ast) return ast;
  hipError_t e = hipSuccess;
  if (!bp.pack.buf.empty()) e = hipMemcpy(d_args, bp.pack.buf.data(), bp.pack.buf.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pl->cap_stream) e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipFree(d_args);
    return dev_fail(e, "batch capture setup");
  }
  bf_status st = enqueue_batch(pl, n, d_in, d_out, bp, (const char *)d_args, pl->cap_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(pl->cap_stream, &graph);
  hipGraphExec_t exec = nullptr;
  if (!st && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (st || e != hipSuccess) {
    (void)hipFree(d_args);
    return st ? st : dev_fail(e, "batch graph");
  }
  if (pl->batches.size() >= 4) {
    (void)hipGraphExecDestroy(pl->batches.front().exec);
    (void)hipFree(pl->batches.front().d_args);
    pl->batches.erase(pl->batches.begin());
  }
  pl->batches.push_back({std::vector<const void *>(d_in, d_in + n), std::vector<float *>(d_out, d_out + n), exec, d_args});
  e = hipGraphLaunch(exec, s);
  return e == hipSuccess ? BF_OK : dev_fail(e, "hipGraphLaunch");
}

bf_status fill_report(const ImagePlan &ip, const void *d_state, bf_report *rep, float ms) {
  unsigned char buf[24];
  hipError_t e = hipMemcpy(buf, d_state, 24, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_fail(e, "read report");
  int32_t Tu, flags;
  unsigned long long traw, qn;
  std::memcpy(&Tu, buf + 0, 4);
  std::memcpy(&flags, buf + 4, 4);
  std::memcpy(&traw, buf + 8, 8);
  std::memcpy(&qn, buf + 16, 8);
  double T;
  std::memcpy(&T, &traw, 8);
  int Tc = Tu < 0 ? 0 : (Tu > ip.T_cap ? ip.T_cap : Tu);
  const OrderEntry &oe = ip.tab.ent[ip.tab.idx_of_T[Tc]];
  rep->T = T;
  rep->T_used = Tu;
  rep->N = oe.N;
  rep->M = oe.M;
  rep->kept = ip.poly ? oe.M + 1 : oe.N - 2 * oe.M + 1;
  rep->pairs = oe.K;
  rep->variant = ip.variant;
  rep->flags = flags;
  rep->q_nonpos = (int64_t)qn;
  rep->ms = ms;
  if (flags & 1) return fail(BF_ERR_NOT_FINITE, "input holds NaN or Inf");
  if (flags & 2) return fail(BF_ERR_RANGE, "dynamic range above value_range");
  return BF_OK;
}

}  // namespace

extern "C" {

const char *bf_status_string(bf_status s) {
  switch (s) {
    case BF_OK: return "ok";
    case BF_ERR_INVALID_ARG: return "invalid argument";
    case BF_ERR_UNSUPPORTED: return "unsupported";
    case BF_ERR_OUT_OF_MEMORY: return "out of memory";
    case BF_ERR_DEVICE: return "device error";
    case BF_ERR_NOT_FINITE: return "non-finite input";
    case BF_ERR_RANGE: return "input outside value_range";
  }
  return "unknown status";
}

const char *bf_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"

namespace {
bf_status autotune(const bf_params &p, Knobs &kn);
void autotune_batch(const bf_params *params, int n, std::vector<Knobs> &kn);
}

// Plan creation with explicit per-image knobs (the autotuner's choices).
static bf_status create_plan(const bf_params *params, int32_t n_images, const Knobs *knobs, bf_plan_t *out) {
  bf_plan_s *pl = new bf_plan_s();
  (void)hipGetDevice(&pl->device);
  pl->im.resize(n_images);
  size_t rowmax = 0, Z = 0, PQ = 0, lut = 0, patch = 0;
  for (int i = 0; i < n_images; i++) {
    pl->im[i].v_target = n_images > 1 ? kVWorkgroupsBatch : kVWorkgroups;
    pl->im[i].h_target = n_images > 1 ? kHWorkgroupsBatch : kHWorkgroups;
    bf_status s = prepare_image(params[i], pl->im[i], knobs ? knobs[i] : Knobs());
    if (s) {
      bf_plan_destroy(pl);
      return s;
    }
    const ImagePlan &ip = pl->im[i];
    const Geom &g = ip.g;
    rowmax = std::max(rowmax, std::max<size_t>(range_ws_bytes(ip), 256));
    if (!is_toeplitz(ip.variant)) {
      lut = std::max(lut, (size_t)ip.KC * 256 * sizeof(float2));
    }
    Z = std::max(Z, (size_t)ip.KC * ip.z_per_pair);
    PQ = std::max(PQ, (size_t)(is_toeplitz(ip.variant) ? ip.tc.groups : g.hgroups) * g.H * g.W * sizeof(float2));
    if (ip.nlm) patch = std::max(patch, (size_t)g.H * g.W * sizeof(Patch8x4));
  }
  bf_status s;
  if ((s = ensure(&pl->d_rowmax, pl->rowmax_bytes, rowmax)) ||
      (s = ensure((void **)&pl->d_Z, pl->Z_bytes, Z)) || (s = ensure((void **)&pl->d_PQ, pl->PQ_bytes, PQ)) ||
      (s = ensure((void **)&pl->d_lut, pl->lut_bytes, lut)) ||
      (patch && (s = ensure(&pl->d_patch, pl->patch_bytes, patch)))) {
    bf_plan_destroy(pl);
    return s;
  }
  if (n_images > 1) {
    // per-image regions for the grouped launches (row maxima, smoothed
    // images of every pair, partial sums), within the workspace budget
    size_t off = 0, zsum = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) / 256 * 256;
      return o;
    };
    for (int i = 0; i < n_images; i++) {
      const ImagePlan &ip = pl->im[i];
      const Geom &g = ip.g;
      const bool t = is_toeplitz(ip.variant);
      const size_t K = (size_t)ip.tab.K_max;
      const size_t zb = K * ip.z_per_pair;
      zsum += zb;
      pl->rowmax_off.push_back(take(range_ws_bytes(ip)));
      pl->z_off.push_back(take(zb));
      pl->pq_off.push_back(take((size_t)(t ? ip.tc.groups : g.hgroups) * g.H * g.W * sizeof(float2)));
      pl->glut_off.push_back(take(t ? 0 : K * 256 * sizeof(float2)));
    }
    size_t budget = (size_t)64 << 30;
    if (const char *b = std::getenv("BF_Z_BUDGET_MB")) budget = (size_t)std::atoll(b) << 20;
    if (zsum <= budget) {
      if ((s = ensure(&pl->d_bws, pl->bws_bytes, off))) {
        bf_plan_destroy(pl);
        return s;
      }
      pl->grouped = true;
    }
  }
  if (const char *g = std::getenv("BF_GRAPH")) pl->use_graph = std::atoi(g) != 0;
  if (hipEventCreate(&pl->ev0) != hipSuccess || hipEventCreate(&pl->ev1) != hipSuccess) {
    bf_plan_destroy(pl);
    return fail(BF_ERR_DEVICE, "hipEventCreate");
  }
  *out = pl;
  return BF_OK;
}

extern "C" {

bf_status bf_plan(const bf_params *params, int32_t n_images, bf_plan_t *out) {
  if (!out) return fail(BF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!params || n_images < 1) return fail(BF_ERR_INVALID_ARG, "params NULL or n_images < 1");
  for (int i = 0; i < n_images; i++) {
    bf_status s = check_params(params[i]);
    if (s) return s;
  }
  std::vector<Knobs> kn(n_images);
  bool any_auto = false;
  for (int i = 0; i < n_images; i++)
    if (params[i].blur == BF_BLUR_AUTO) {
      any_auto = true;
      bf_status s = autotune(params[i], kn[i]);
      if (s) return s;
    }
  if (n_images > 1 && any_auto) autotune_batch(params, n_images, kn);
  return create_plan(params, n_images, kn.data(), out);
}

bf_status bf_profile(bf_plan_t pl, int32_t enable) {
  if (!pl) return fail(BF_ERR_INVALID_ARG, "NULL plan");
  pl->prof = enable != 0;
  pl->rec.mark = pl->prof ? stage_mark : nullptr;
  pl->rec.ctx = pl;
  return BF_OK;
}

bf_status bf_profile_read(bf_plan_t pl, double *ms, int64_t *launches) {
  if (!pl || !ms || !launches) return fail(BF_ERR_INVALID_ARG, "NULL argument");
  for (auto &p : pl->pending) {
    hipError_t e = hipEventSynchronize(p.b);
    if (e != hipSuccess) return dev_fail(e, "hipEventSynchronize");
    float t = 0.f;
    (void)hipEventElapsedTime(&t, p.a, p.b);
    pl->prof_ms[p.stage] += t;
    pl->prof_n[p.stage] += 1;
    pl->ev_pool.push_back(p.a);
    pl->ev_pool.push_back(p.b);
  }
  pl->pending.clear();
  for (int i = 0; i < BF_STAGE_COUNT; i++) {
    ms[i] = pl->prof_ms[i];
    launches[i] = pl->prof_n[i];
    pl->prof_ms[i] = 0.0;
    pl->prof_n[i] = 0;
  }
  return BF_OK;
}

void bf_plan_destroy(bf_plan_t pl) {
  if (!pl) return;
  for (auto &p : pl->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : pl->ev_pool) (void)hipEventDestroy(e);
  for (auto &g : pl->graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto &b : pl->batches) {
    (void)hipGraphExecDestroy(b.exec);
    (void)hipFree(b.d_args);
  }
  (void)hipFree(pl->d_bws);
  (void)hipFree(pl->d_eager_args);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  for (auto e : pl->open_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &ip : pl->im) free_image(ip);
  (void)hipFree(pl->d_rowmax);
  (void)hipFree(pl->d_Z);
  (void)hipFree(pl->d_PQ);
  (void)hipFree(pl->d_lut);
  (void)hipFree(pl->d_patch);
  if (pl->ev0) (void)hipEventDestroy(pl->ev0);
  if (pl->ev1) (void)hipEventDestroy(pl->ev1);
  delete pl;
}

bf_status bf_filter(bf_plan_t pl, const void *d_in, float *d_out, void *hip_stream, bf_report *rep) {
  if (!pl || !d_in || !d_out) return fail(BF_ERR_INVALID_ARG, "NULL plan or buffer");
  hipStream_t s = (hipStream_t)hip_stream;
  ImagePlan &ip = pl->im[0];
  if (rep) (void)hipEventRecord(pl->ev0, s);
  bf_status st = (pl->use_graph && !pl->prof) ? run_image_graph(pl, 0, d_in, d_out, s)
                                               : run_image(pl, ip, d_in, d_out, s);
  if (st) return st;
  if (!rep) return BF_OK;
  (void)hipEventRecord(pl->ev1, s);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, pl->ev0, pl->ev1);
  return fill_report(ip, ip.d_state, rep, ms);
}

}  // extern "C"

// ------------------------------------------ working memory without allocation
// bf_filter_noalloc runs the launch sequence of bf_filter with its working
// memory (device state, row maxima, cos/sin tables, partial sums, smoothed
// images) in this array instead of the plan's.  Each GPU the library runs on
// holds its own copy until the process ends.  Host code never uses the name
// as an address: the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

bf_status scratch_on(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BF_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return dev_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(BF_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = (unsigned char *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return BF_OK;
}
}  // namespace

extern "C" {

bf_status bf_filter_noalloc(bf_plan_t pl, const void *d_in, float *d_out, void *hip_stream, bf_report *rep) {
  if (!pl || !d_in || !d_out) return fail(BF_ERR_INVALID_ARG, "NULL plan or buffer");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_fail(e, "hipGetDevice");
  if (dev != pl->device) return fail(BF_ERR_INVALID_ARG, "the current device is not the plan's");
  ImagePlan &ip = pl->im[0];
  if (!ip.na.ok)
    return fail(BF_ERR_UNSUPPORTED, "image needs more than the " + std::to_string(kScratchBytes >> 20) +
                                        " MiB of static working memory for one frequency pair per launch");
  unsigned char *base = nullptr;
  bf_status st = scratch_on(dev, &base);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  if (rep) (void)hipEventRecord(pl->ev0, s);
  // the range accumulators and counters must start at zero; the array keeps
  // whatever the previous call on this device left in it
  e = launch_zero(s, base, align256(kStateBytes));
  if (e != hipSuccess) return dev_fail(e, "clear state");
  const ImagePlan::NoAlloc &na = ip.na;
  const Workspace ws{base + na.rowmax, (float4 *)(base + na.z), (float2 *)(base + na.pq), (float2 *)(base + na.lut),
                     base + na.patch};
  st = run_image_ws(ws, StageRec(), ip, Shape{&na.g, &na.tc, na.KC, base}, d_in, d_out, s);
  if (st) return st;
  if (!rep) return BF_OK;
  (void)hipEventRecord(pl->ev1, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, pl->ev0, pl->ev1);
  return fill_report(ip, base, rep, ms);
}

bf_status bf_filter_batch(bf_plan_t pl, int32_t n, const void *const *d_in, float *const *d_out, void *hip_stream,
                          bf_report *reps) {
  if (!pl || !d_in || !d_out) return fail(BF_ERR_INVALID_ARG, "NULL plan or pointer array");
  if (n < 1 || n > (int32_t)pl->im.size()) return fail(BF_ERR_INVALID_ARG, "n outside [1, n_images]");
  for (int i = 0; i < n; i++)
    if (!d_in[i] || !d_out[i]) return fail(BF_ERR_INVALID_ARG, "NULL image pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  if (reps) (void)hipEventRecord(pl->ev0, s);
  bf_status bst = (pl->use_graph && !pl->prof) ? run_batch_graph(pl, n, d_in, d_out, s)
                                               : run_batch_eager(pl, n, d_in, d_out, s);
  if (bst) return bst;
  if (!reps) return BF_OK;
  (void)hipEventRecord(pl->ev1, s);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, pl->ev0, pl->ev1);
  bf_status first = BF_OK;
  for (int i = 0; i < n; i++) {
    bf_status st = fill_report(pl->im[i], pl->im[i].d_state, &reps[i], ms);
    if (st && !first) first = st;
  }
  return first;
}

bf_status bf_dynamic_range(bf_plan_t pl, const void *d_in, void *hip_stream, double *T_out) {
  if (!pl || !d_in || !T_out) return fail(BF_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)hip_stream;
  ImagePlan &ip = pl->im[0];
  DevState st = state_of(ip);
  hipError_t e = launch_range(s, ip.p.dtype, d_in, ip.g, ip.R, pl->d_rowmax, st, acc_of(ip), ip.T_cap, pl->rec);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "dynamic range");
  unsigned long long traw;
  e = hipMemcpy(&traw, (char *)ip.d_state + 8, 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_fail(e, "read T");
  std::memcpy(T_out, &traw, 8);
  return BF_OK;
}

}  // extern "C"

// ------------------------------------------------------------- autotuner
// BF_BLUR_AUTO: among the implementations of the image's spatial operator
// whose worst error over the parity suite (adversarial noise included) stays
// within the 2e-3 target -- for the recursive Gaussian the FP32 recursive
// blur with either horizontal chunk width, for the FIR operators (sampled
// Gaussian, box) the split-FP16 Toeplitz blur with either LDS budget of its
// vertical tile -- take the fastest on this device at the image's shape and
// dtype with every pair kept (T at the full range).  The operator itself is
// never changed, so the output does not depend on the choice beyond rounding.
// Choices are cached in the process and, when BF_TUNE_CACHE names a file, in
// that file (one JSON object per line).
namespace {

std::mutex g_tune_mu;
std::map<std::string, Knobs> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const bf_params &p) {
  char arch[64] = "gfx";
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s|d%d|%dx%d|ss%.9g|sr%.9g|e%.9g|R%d|t%d|tv%.9g|vr%.9g|k%d", arch, (int)p.dtype,
                p.height, p.width, p.sigma_s, p.sigma_r, p.eps, p.radius, (int)p.t_mode, p.t_value, p.value_range,
                (int)p.spatial);
  return buf;
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("BF_TUNE_CACHE");
  if (!path) return;
  FILE *fp = std::fopen(path, "r");
  if (!fp) return;
  char line[1024];
  while (std::fgets(line, sizeof(line), fp)) {
    const char *k = std::strstr(line, "\"key\": \"");
    if (!k) continue;
    k += 8;
    const char *e = std::strchr(k, '"');
    if (!e) continue;
    Knobs kn;
    const char *v = std::strstr(e, "\"variant\": ");
    const char *h = std::strstr(e, "\"hchunk\": ");
    const char *l = std::strstr(e, "\"lds_kb\": ");
    if (!v || !h || !l) continue;
    kn.variant = std::atoi(v + 11);
    kn.hchunk = std::atoi(h + 10);
    kn.lds_kb = std::atoi(l + 10);
    if (kn.variant == BF_BLUR_IIR_F32 || kn.variant == BF_BLUR_TOEPLITZ_F16X2) g_tune[std::string(k, e)] = kn;
  }
  std::fclose(fp);
}

void tune_save(const std::string &key, const Knobs &kn, double ms) {
  const char *path = std::getenv("BF_TUNE_CACHE");
  if (!path) return;
  FILE *fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "{\"key\": \"%s\", \"variant\": %d, \"hchunk\": %d, \"lds_kb\": %d, \"ms\": %.6f}\n",
               key.c_str(), kn.variant, kn.hchunk, kn.lds_kb, ms);
  std::fclose(fp);
}

// Device time of one filter call of a candidate (median of 5 after warm-up), or
// a negative value when the candidate cannot run this image.
double time_candidate(const bf_params &p, const Knobs &kn, void *d_in, float *d_out, hipStream_t s, hipEvent_t a,
                      hipEvent_t b) {
  bf_params q = p;
  q.blur = (bf_blur)kn.variant;
  q.in_pitch = q.out_pitch = 0;
  if (q.t_mode == BF_T_LOCAL) {  // every pair kept: T at the full range
    q.t_mode = BF_T_GLOBAL;
    q.t_value = 0.0;
  }
  bf_plan_t pl = nullptr;
  if (create_plan(&q, 1, &kn, &pl) != BF_OK) return -1.0;
  std::vector<float> t;
  bool ok = true;
  for (int r = 0; r < 7 && ok; r++) {
    ok = hipEventRecord(a, s) == hipSuccess && run_image(pl, pl->im[0], d_in, d_out, s) == BF_OK &&
         hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
    float ms = 0.f;
    if (ok && hipEventElapsedTime(&ms, a, b) == hipSuccess && r >= 2) t.push_back(ms);
  }
  bf_plan_destroy(pl);
  if (!ok || t.empty()) return -1.0;
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

bf_status autotune(const bf_params &p, Knobs &best) {
  const std::string key = tune_key(p);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && is_toeplitz(it->second.variant) == fir_operator(p)) {
      best = it->second;
      return BF_OK;
    }
  }
  std::vector<Knobs> cand;
  const int R = window_radius(p);
  if (!fir_operator(p)) {
    if (p.width > kMaxWidth || p.height > kMaxWidth)
      return fail(BF_ERR_UNSUPPORTED, "width or height above 8192 for the recursive blur");
    cand.push_back(Knobs{BF_BLUR_IIR_F32, kCSmall, 0});
    if (p.width > kCSmall && p.width <= kCSmall * kHThreads) cand.push_back(Knobs{BF_BLUR_IIR_F32, kCLarge, 0});
  } else {
    if (R > 120) return fail(BF_ERR_UNSUPPORTED, "radius above 120 for the Toeplitz blur");
    cand.push_back(Knobs{BF_BLUR_TOEPLITZ_F16X2, 0, kToepLdsMax / 2048 - 2});
    cand.push_back(Knobs{BF_BLUR_TOEPLITZ_F16X2, 0, kToepDynMax / 1024});
  }
  if (cand.size() == 1) {
    best = cand[0];
    return BF_OK;
  }
  // a full-range input: alternating 0 and the top of the range
  const size_t px = (size_t)p.height * p.width;
  void *d_in = nullptr;
  float *d_out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc(&d_in, px * elem_size(p.dtype));
  if (e == hipSuccess) e = hipMalloc((void **)&d_out, px * sizeof(float));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  const double full = p.dtype == BF_U16 ? 65535.0 : 255.0;
  const double range = p.value_range > 0.0 ? p.value_range : full;
  if (e == hipSuccess) e = launch_fill_checker(s, p.dtype, d_in, p.height, p.width, range);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  double best_ms = -1.0;
  if (e == hipSuccess) {
    for (const Knobs &kn : cand) {
      const double ms = time_candidate(p, kn, d_in, d_out, s, a, b);
      if (ms > 0.0 && (best_ms < 0.0 || ms < best_ms)) {
        best_ms = ms;
        best = kn;
      }
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(d_in);
  (void)hipFree(d_out);
  if (e != hipSuccess) return dev_fail(e, "autotune");
  if (best_ms < 0.0) best = cand[0];
  if (std::getenv("BF_TUNE_LOG"))
    std::fprintf(stderr, "[bf tune] %s -> variant %d hchunk %d lds %d KB (%.3f ms)\n", key.c_str(), best.variant,
                 best.hchunk, best.lds_kb, best_ms);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
  tune_save(key, best, best_ms);
  return BF_OK;
}

// Batch-level choice: a batch runs one set of grouped launches per kernel
// instantiation, so a mix of tile choices can lose to giving every image of
// an operator the same one (fuller launches).  The per-image choice and the
// uniform default choice (each image keeps its operator) are timed on the
// whole batch (full-range checkerboards, every pair kept) and the faster kept.
double time_batch(const bf_params *params, int n, const std::vector<Knobs> &kn, std::vector<void *> &ins,
                  std::vector<float *> &outs, hipStream_t s, hipEvent_t a, hipEvent_t b) {
  std::vector<bf_params> q(params, params + n);
  for (auto &p : q) {
    p.in_pitch = p.out_pitch = 0;
    if (p.t_mode == BF_T_LOCAL) {
      p.t_mode = BF_T_GLOBAL;
      p.t_value = 0.0;
    }
  }
  bf_plan_t pl = nullptr;
  if (create_plan(q.data(), n, kn.data(), &pl) != BF_OK) return -1.0;
  BatchPlan bp;
  build_batch(pl, n, ins.data(), outs.data(), bp);
  void *d_args = nullptr;
  double best = -1.0;
  if (hipMalloc(&d_args, std::max<size_t>(bp.pack.buf.size(), 256)) == hipSuccess &&
      (bp.pack.buf.empty() ||
       hipMemcpy(d_args, bp.pack.buf.data(), bp.pack.buf.size(), hipMemcpyHostToDevice) == hipSuccess)) {
    std::vector<float> t;
    for (int r = 0; r < 5; r++) {
      bool ok = hipEventRecord(a, s) == hipSuccess &&
                enqueue_batch(pl, n, ins.data(), outs.data(), bp, (const char *)d_args, s) == BF_OK &&
                hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
      float ms = 0.f;
      if (!ok) break;
      if (hipEventElapsedTime(&ms, a, b) == hipSuccess && r >= 1) t.push_back(ms);
    }
    if (!t.empty()) {
      std::sort(t.begin(), t.end());
      best = t[t.size() / 2];
    }
  }
  (void)hipFree(d_args);
  bf_plan_destroy(pl);
  return best;
}

void autotune_batch(const bf_params *params, int n, std::vector<Knobs> &kn) {
  // The tuned recursive images take the term-group width for a launch they
  // share with the other images (which fill the GPU between them): fewer
  // idle pair slots rather than more workgroups.  (The proxy input keeps
  // every pair, so timing it could not tell the widths apart on real T.)
  for (int i = 0; i < n; i++)
    if (params[i].blur == BF_BLUR_AUTO && kn[i].variant == BF_BLUR_IIR_F32) kn[i].hpw = -1;
  // candidates: the per-image choice, and every tuned image on the default
  // implementation of its own operator (one set of grouped launches each)
  std::vector<std::vector<Knobs>> cand(1, kn);
  {
    std::vector<Knobs> alt = kn;
    bool differs = false;
    for (int i = 0; i < n; i++) {
      if (params[i].blur != BF_BLUR_AUTO) continue;
      const Knobs d = fir_operator(params[i]) ? Knobs{BF_BLUR_TOEPLITZ_F16X2, 0, kToepLdsMax / 2048 - 2}
                                              : Knobs{BF_BLUR_IIR_F32, kCSmall, 0, -1};
      if (d.variant != kn[i].variant || d.hchunk != kn[i].hchunk || d.lds_kb != kn[i].lds_kb) differs = true;
      alt[i] = d;
    }
    if (differs) cand.push_back(alt);
  }
  if (cand.size() == 1) return;
  std::vector<void *> ins(n, nullptr);
  std::vector<float *> outs(n, nullptr);
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  for (int i = 0; i < n && e == hipSuccess; i++) {
    const bf_params &p = params[i];
    const size_t px = (size_t)p.height * p.width;
    e = hipMalloc(&ins[i], px * elem_size(p.dtype));
    if (e == hipSuccess) e = hipMalloc((void **)&outs[i], px * sizeof(float));
    const double full = p.dtype == BF_U16 ? 65535.0 : 255.0;
    if (e == hipSuccess)
      e = launch_fill_checker(s, p.dtype, ins[i], p.height, p.width, p.value_range > 0.0 ? p.value_range : full);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    double best = -1.0;
    size_t pick = 0;
    for (size_t c = 0; c < cand.size(); c++) {
      const double t = time_batch(params, n, cand[c], ins, outs, s, a, b);
      if (std::getenv("BF_TUNE_LOG"))
        std::fprintf(stderr, "[bf tune] batch of %d, assignment %zu: %.3f ms\n", n, c, t);
      if (t > 0.0 && (best < 0.0 || t < best)) {
        best = t;
        pick = c;
      }
    }
    kn = cand[pick];
  }
  for (int i = 0; i < n; i++) {
    (void)hipFree(ins[i]);
    (void)hipFree(outs[i]);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (s) (void)hipStreamDestroy(s);
}

}  // namespace
