// gfx950 kernels of libbf.so: dynamic range (Algorithm 1), phase generation,
// the blocked recursive Gaussian (Young-van Vliet cascade) and the fused
// accumulate-and-normalise of eqs. (f1), (f2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "bf_device.h"
#include "bf_phase.h"

namespace bfi {


// ------------------------------------------------------------ small helpers
__device__ __forceinline__ float4 f4(float a) { return make_float4(a, a, a, a); }
__device__ __forceinline__ float4 add4(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float4 sub4(float4 a, float4 b) {
  return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
// acc + k * v
__device__ __forceinline__ float4 fma4(float k, float4 v, float4 acc) {
  return make_float4(fmaf(k, v.x, acc.x), fmaf(k, v.y, acc.y), fmaf(k, v.z, acc.z),
                     fmaf(k, v.w, acc.w));
}
// r = M v for a row-major 3x3 M acting on three float4 (four planes at once)
__device__ __forceinline__ void matvec3(const float *__restrict__ M, const float4 v[3], float4 r[3]) {
#pragma unroll
  for (int i = 0; i < 3; i++) {
    float4 a = f4(0.0f);
    a = fma4(M[3 * i + 0], v[0], a);
    a = fma4(M[3 * i + 1], v[1], a);
    a = fma4(M[3 * i + 2], v[2], a);
    r[i] = a;
  }
}
// M u for M a power of the cascade's zero-input state matrix
// A, whose first row is (m00, 0, 0): the first-order section does not see the
// second-order state (the tables hold those zeros exactly).
__device__ __forceinline__ void apow_acc(const float *__restrict__ M, const float4 u[3], float4 v[3]) {
  v[0] = fma4(M[0], u[0], v[0]);
#pragma unroll
  for (int i = 1; i < 3; i++) {
    v[i] = fma4(M[3 * i + 0], u[0], v[i]);
    v[i] = fma4(M[3 * i + 1], u[1], v[i]);
    v[i] = fma4(M[3 * i + 2], u[2], v[i]);
  }
}
__device__ __forceinline__ void apow_mul(const float *__restrict__ M, const float4 u[3], float4 r[3]) {
  r[0] = make_float4(M[0] * u[0].x, M[0] * u[0].y, M[0] * u[0].z, M[0] * u[0].w);
#pragma unroll
  for (int i = 1; i < 3; i++) {
    float4 a = make_float4(M[3 * i] * u[0].x, M[3 * i] * u[0].y, M[3 * i] * u[0].z, M[3 * i] * u[0].w);
    a = fma4(M[3 * i + 1], u[1], a);
    r[i] = fma4(M[3 * i + 2], u[2], a);
  }
}

// One step of the recursive Gaussian cascade on the state (s, w, d):
// first-order section s = a1 s + x (a1 = 1 - g1; the input gain g1 is left
// out, a constant factor per pass common to all smoothed images, which
// cancels in P / Q), then the second-order section carried as
// d[n] = (s - w[n-1]) - c2 d[n-1], w[n] = w[n-1] + g2 d[n] (d is the
// increment of w divided by g2): four operations per sample and image.
__device__ __forceinline__ void casc_step(float a1, float g2, float c2, float4 x, float4 &s, float4 &w,
                                          float4 &d) {
  s = fma4(a1, s, x);
  d = fma4(-c2, d, sub4(s, w));
  w = fma4(g2, d, w);
}

// ---- segmented running maxima across a wave (Appendix MAX-FILTER) --------
// Lane l holds element e = e0 + l.  Partitions of the running maxima start at
// segs (scan up) or end at sege (scan down).  Within each 16-lane row the
// scan uses DPP row shifts (VALU only); rows are then chained through
// v_readlane of the last lane of the previous row.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(-INFINITY), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ float seg_max_up(float v, int e, int segs, int lane) {
  const int lr = lane & 15;
  float o;
  o = dpp_mov<0x111>(v);  // row_shr:1
  if (lr >= 1 && e - 1 >= segs) v = fmaxf(v, o);
  o = dpp_mov<0x112>(v);  // row_shr:2
  if (lr >= 2 && e - 2 >= segs) v = fmaxf(v, o);
  o = dpp_mov<0x114>(v);  // row_shr:4
  if (lr >= 4 && e - 4 >= segs) v = fmaxf(v, o);
  o = dpp_mov<0x118>(v);  // row_shr:8
  if (lr >= 8 && e - 8 >= segs) v = fmaxf(v, o);
  const int e0 = e - lane;
  float t = lane_value(v, 15);
  if ((lane >> 4) == 1 && e0 + 15 >= segs) v = fmaxf(v, t);
  t = lane_value(v, 31);
  if ((lane >> 4) == 2 && e0 + 31 >= segs) v = fmaxf(v, t);
  t = lane_value(v, 47);
  if ((lane >> 4) == 3 && e0 + 47 >= segs) v = fmaxf(v, t);
  return v;
}
__device__ __forceinline__ float seg_max_down(float v, int e, int sege, int lane) {
  const int lr = lane & 15;
  float o;
  o = dpp_mov<0x101>(v);  // row_shl:1
  if (lr <= 14 && e + 1 <= sege) v = fmaxf(v, o);
  o = dpp_mov<0x102>(v);  // row_shl:2
  if (lr <= 13 && e + 2 <= sege) v = fmaxf(v, o);
  o = dpp_mov<0x104>(v);  // row_shl:4
  if (lr <= 11 && e + 4 <= sege) v = fmaxf(v, o);
  o = dpp_mov<0x108>(v);  // row_shl:8
  if (lr <= 7 && e + 8 <= sege) v = fmaxf(v, o);
  const int e0 = e - lane;
  float t = lane_value(v, 48);
  if ((lane >> 4) == 2 && e0 + 48 <= sege) v = fmaxf(v, t);
  t = lane_value(v, 32);
  if ((lane >> 4) == 1 && e0 + 32 <= sege) v = fmaxf(v, t);
  t = lane_value(v, 16);
  if ((lane >> 4) == 0 && e0 + 16 <= sege) v = fmaxf(v, t);
  return v;
}

// Publish a non-negative dynamic-range candidate.  Many workgroups race for
// the same two words, so an atomic is issued only when a relaxed read shows
// that the candidate is larger than the current value.
__device__ __forceinline__ void publish_T(const DevState &st, double t, int32_t T_cap) {
  const double tc = ceil(t);
  const int ti = tc > 2147483647.0 ? 2147483647 : (int)tc;
  const unsigned long long tb = (unsigned long long)__double_as_longlong(t);
  if (ti > __hip_atomic_load(st.T_used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(st.T_used, ti);
  if (tb > __hip_atomic_load(st.T_raw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(st.T_raw, tb);
  if (ti > T_cap) atomicOr(st.flags, 2);
}

// ------------------------------------------------------------------- reset
__device__ __forceinline__ void reset_body(const ResetArgs &a, const Blk b) {
  const DevState st = a.st;
  const int32_t T_used = a.T_used;
  const double T_raw = a.T_raw;

  if (threadIdx.x == 0 && b.x == 0) {
    *st.T_used = T_used;
    *st.T_raw = (unsigned long long)__double_as_longlong(T_raw);
    *st.flags = 0;
    *st.q_nonpos = 0ull;
  }
}
__global__ void k_reset(ResetArgs a) { reset_body(a, Blk{(int)blockIdx.x, 0, 0}); }
__global__ void k_reset_grp(const ResetArgs *__restrict__ a, const int *__restrict__ start, int n) {
  const int i = group_find(start, n, blockIdx.x);
  reset_body(a[i], group_blk(a[i].gg, blockIdx.x - start[i]));
}

// ------------------------------------------------- Algorithm 1, row pass
// MAX-FILTER (Appendix) along rows.  One wave per segment of kRowSeg outputs.
// The segment's input [xs-R, xs+n+R) is indexed by e; partitions of length
// 2R+1 start at e = 0.  Left running maxima l (reset at each partition start)
// and right running maxima r (reset at each partition end) are segmented
// scans done with wave shuffles, carried tile to tile; then
// out(x) = max(r[e], l[e+2R]) with e = x - xs.
// e mod Wd for 0 <= e < 2^22 without an integer division
__device__ __forceinline__ int mod_small(int e, int Wd, float inv) {
  int q = (int)((float)e * inv);
  int r = e - q * Wd;
  r = r < 0 ? r + Wd : r;
  r = r >= Wd ? r - Wd : r;
  return r;
}

constexpr int kRowSeg = 256;
constexpr int kMaxR = 1024;

template <typename Tin>
__device__ __forceinline__ void rowmax_body(const RowmaxArgs &a, const Blk b) {
  const Tin *__restrict__ f = (const Tin *)a.f;
  const int64_t pitch = a.pitch;
  const int W = a.W, R = a.R;
  Tin *__restrict__ rowmax = (Tin *)a.rowmax;
  const DevState st = a.st;

  __shared__ float sv[kRowSeg + 2 * kMaxR + 64];
  __shared__ float sl[kRowSeg + 2 * kMaxR + 64];
  const int y = b.y;
  const int xs = b.x * kRowSeg;
  if (xs >= W) return;
  const int n_out = min(kRowSeg, W - xs);
  const int L = n_out + 2 * R;
  const int Wd = 2 * R + 1;
  const float inv = 1.0f / (float)Wd;
  const int lane = threadIdx.x;
  const Tin *frow = f + (int64_t)y * pitch;
  bool bad = false;
  // stage the segment and its halo, 8 loads per lane in flight at a time
  for (int e0 = 0; e0 < L; e0 += 8 * 64) {
    float vb[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int e = e0 + u * 64 + lane;
      const int x = xs - R + e;
      const float raw = fval(frow[min(max(x, 0), W - 1)]);  // clamped: no branch around the load
      vb[u] = (e < L && x >= 0 && x < W) ? raw : -INFINITY;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int e = e0 + u * 64 + lane;
      if (e < L) {
        const int x = xs - R + e;
        const float v = vb[u];
        if (x >= 0 && x < W && !isfinite(v)) bad = true;  // NaN or Inf in the image
        sv[e] = isfinite(v) ? v : -INFINITY;
      }
    }
  }
  __syncthreads();
  float carry = -INFINITY;
  for (int e0 = 0; e0 < L; e0 += 64) {
    const int e = e0 + lane;
    float v = e < L ? sv[e] : -INFINITY;
    const int segs = e - mod_small(e, Wd, inv);
    v = seg_max_up(v, e, segs, lane);
    if (e0 > 0 && e0 - 1 >= segs) v = fmaxf(v, carry);
    carry = lane_value(v, 63);
    if (e < L) sl[e] = v;
  }
  carry = -INFINITY;
  for (int e0 = ((L - 1) / 64) * 64; e0 >= 0; e0 -= 64) {
    const int e = e0 + lane;
    float v = e < L ? sv[e] : -INFINITY;
    const int sege = e - mod_small(e, Wd, inv) + Wd - 1;
    v = seg_max_down(v, e, sege, lane);
    if (e0 + 64 <= sege) v = fmaxf(v, carry);
    carry = lane_value(v, 0);
    // r[e] is final here; out(x) = max(r[x - xs], l[x - xs + 2R])
    if (e < n_out) sv[e] = v;  // sv[e] no longer needed as input for e' <= e
  }
  __syncthreads();
  Tin *orow = rowmax + (int64_t)y * W + xs;
  for (int i = lane; i < n_out; i += 64) orow[i] = (Tin)fmaxf(sv[i], sl[i + 2 * R]);
  if (__any(bad) && lane == 0) atomicOr(st.flags, 1);
}
template <typename Tin>
__global__ __launch_bounds__(64) void k_rowmax(RowmaxArgs a) {
  rowmax_body<Tin>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin>
__global__ __launch_bounds__(64) void k_rowmax_grp(const RowmaxArgs *__restrict__ a,
                                                   const int *__restrict__ start, int n) {
  const int i = group_find(start, n, blockIdx.x);
  rowmax_body<Tin>(a[i], group_blk(a[i].gg, blockIdx.x - start[i]));
}

// ---------------------------------------- Algorithm 1, column pass and T
// (R > 48; smaller windows take the one-launch kernel below).  One lane per
// column walks a band of kColBandSeq output rows (plus the R halo) of the row
// maxima bottom-up for the right running maxima and top-down for the left
// ones, loading 16 rows ahead; T = max (out - f) (Prop. 2.1, sign read from
// its proof) is reduced over the wave.
constexpr int kColBandSeq = 128;

template <typename Tin>
__device__ __forceinline__ void colmax_T_seq_body(const ColmaxArgs &a, const Blk b) {
  const Tin *__restrict__ f = (const Tin *)a.f;
  const int64_t pitch = a.pitch;
  const Tin *__restrict__ rowmax = (const Tin *)a.rowmax;
  const int H = a.H, W = a.W, R = a.R;
  const DevState st = a.st;
  const int32_t T_cap = a.T_cap;

  __shared__ float srb[kColBandSeq][64];
  const int lane = threadIdx.x;
  const int x = b.x * 64 + lane;
  const int y0 = b.y * kColBandSeq;
  const int nb = min(kColBandSeq, H - y0);
  const int L = nb + 2 * R;
  const int Wd = 2 * R + 1;
  double tmax = 0.0;
  if (x < W) {
    float r = -INFINITY;
    int ph = (L - 1) % Wd;
    for (int eb = L - 1; eb >= 0; eb -= 16) {
      float vb[16];
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const int y = y0 - R + eb - u;
        const float raw = fval(rowmax[(int64_t)min(max(y, 0), H - 1) * W + x]);
        vb[u] = (eb - u >= 0 && y >= 0 && y < H) ? raw : -INFINITY;
      }
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const int e = eb - u;
        if (e < 0) break;
        r = (ph == Wd - 1) ? vb[u] : fmaxf(r, vb[u]);
        if (e < nb) srb[e][lane] = r;
        ph = ph == 0 ? Wd - 1 : ph - 1;
      }
    }
    float l = -INFINITY;
    ph = 0;
    for (int eb = 0; eb < L; eb += 16) {
      float vb[16], fv[16];
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const int y = y0 - R + eb + u;
        const float raw = fval(rowmax[(int64_t)min(max(y, 0), H - 1) * W + x]);
        vb[u] = (eb + u < L && y >= 0 && y < H) ? raw : -INFINITY;
        // f at output row e - 2R (clamped into the band; used only for e >= 2R)
        fv[u] = fval(f[(int64_t)(y0 + min(max(eb + u - 2 * R, 0), nb - 1)) * pitch + x]);
      }
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const int e = eb + u;
        if (e >= L) break;
        l = (ph == 0) ? vb[u] : fmaxf(l, vb[u]);
        ph = ph == Wd - 1 ? 0 : ph + 1;
        if (e >= 2 * R) {
          const int i = e - 2 * R;
          const float mx = fmaxf(srb[i][lane], l);
          const double d = (double)mx - (double)fv[u];
          tmax = d > tmax ? d : tmax;
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(tmax, off, 64);
    tmax = o > tmax ? o : tmax;
  }
  if (lane == 0) publish_T(st, tmax, T_cap);
}
template <typename Tin>
__global__ __launch_bounds__(64) void k_colmax_T_seq(ColmaxArgs a) {
  colmax_T_seq_body<Tin>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin>
__global__ __launch_bounds__(64) void k_colmax_T_seq_grp(const ColmaxArgs *__restrict__ a,
                                                         const int *__restrict__ start, int n) {
  const int i = group_find(start, n, blockIdx.x);
  colmax_T_seq_body<Tin>(a[i], group_blk(a[i].gg, blockIdx.x - start[i]));
}

// ------------------------------------------- Algorithm 1 in one launch
// A workgroup (8 waves) takes a 32 x 32 block of output pixels.  The block
// and its R-pixel halo are staged in LDS, one staged row per wave step with
// the lanes along the row.  Samples are kept as integer keys that order like
// them: the 8- or 16-bit value itself (out-of-image samples 0: every window
// holds its in-image centre, which is >= 0), or for float input the bit
// pattern sign-folded (non-finite samples and out-of-image ones -inf).
// With a window 2R+1 >= 32 the MAX-FILTER of the Appendix over a line of
// 32 + 2R samples x has, for output j in [0, 32), the window [j, j+2R] =
// [j, 30] u [31, 2R] u [2R+1, 2R+j]: a suffix maximum over the first 31
// samples, one maximum common to the whole line, and a prefix maximum over
// the last 31 samples (van Herk's forward and backward running maxima with
// the segment boundary placed at the line's 31st sample).  A half-wave
// takes one line, lane j holding output j; the common maximum enters the
// suffix scan as lane 31's sample.  Samples x[31] and x[2R] lie in every
// window of the line, so lanes whose piece is empty read one of them instead
// of a masked value; each scan step is one DPP max.  With a narrower window
// (R < 16) each output takes the maximum of its 2R+1 <= 31 samples directly.
// The row pass filters every staged row into the row maxima; the column pass
// filters every output column of those, and T = max (out - f) (Prop. 2.1)
// over the block is merged in two levels: into one of kRangeSubs
// sub-accumulators (block index mod kRangeSubs), whose last arrival merges
// it into the top accumulator, whose last arrival publishes T, the flags and
// a zero non-positive-denominator count and clears both levels for the next
// call.  So no reset launch precedes it, and no address takes more than a
// few dozen atomics.  KR is the largest R an instantiation stages (32, or
// 48 for 8- and 16-bit input, whose narrow keys keep that block in LDS).
constexpr int kTileW = 32;
constexpr int kTileH = 32;
constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / 64;
constexpr int kTileMS = kTileW + 1;  // row-maxima and centre strides (words)

template <typename Tin> struct TileKey { using T = int; };
template <> struct TileKey<uint8_t> { using T = uint8_t; };
template <> struct TileKey<uint16_t> { using T = uint16_t; };

// staged row stride in keys: the two half-waves of a row pass read rows e
// and e+1 at the same offsets, which this stride puts in disjoint banks
template <int KR> constexpr int tile_rs() { return KR <= 32 ? 96 : 160; }

// Float input with 32 < R <= 48: four-byte keys of the whole staged block
// would take ~100 KB of LDS, so the row pass reads its samples from global
// memory instead (coalesced 128-byte pieces, mostly cache hits) and only the
// row maxima and the centre samples live in LDS.
template <typename Tin, int KR>
__host__ __device__ constexpr bool tile_global_rows() { return std::is_same<Tin, float>::value && KR > 32; }

// LDS bytes: staged keys (L x RS, padded to a word; none when the row pass
// reads global memory), row-maxima keys (L x kTileMS words), raw centre
// samples (kTileH x kTileMS floats).
template <typename Tin, int KR>
__host__ __device__ constexpr size_t tile_lds_bytes(int R) {
  return (tile_global_rows<Tin, KR>()
              ? 0
              : ((size_t)(kTileH + 2 * R) * tile_rs<KR>() * sizeof(typename TileKey<Tin>::T) + 3) / 4 * 4) +
         (size_t)(kTileH + 2 * R) * kTileMS * 4 + (size_t)kTileH * kTileMS * 4;
}

template <typename Tin>
__device__ __forceinline__ int tile_key(float v) {
  if constexpr (std::is_same<Tin, float>::value) {
    const int bits = __float_as_int(isfinite(v) ? v : -INFINITY);
    return bits ^ ((bits >> 31) & 0x7FFFFFFF);
  }
  return (int)v;
}
template <typename Tin>
__device__ __forceinline__ float tile_unkey(int k) {
  if constexpr (std::is_same<Tin, float>::value) return __int_as_float(k ^ ((k >> 31) & 0x7FFFFFFF));
  return (float)k;
}

// Max scans over each 32-lane half of the wave (lanes 0-31 and 32-63 hold
// independent lines); lanes without a source take INT_MIN, max's identity.
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dpp_max(int v) {
  return max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, CTRL, RM, 0xF, false));
}
__device__ __forceinline__ int half_prefix_max(int v) {
  v = dpp_max<0x111>(v);          // row_shr:1
  v = dpp_max<0x112>(v);          // row_shr:2
  v = dpp_max<0x114>(v);          // row_shr:4
  v = dpp_max<0x118>(v);          // row_shr:8
  return dpp_max<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
}
__device__ __forceinline__ int half_suffix_max(int v) {
  v = dpp_max<0x101>(v);  // row_shl:1
  v = dpp_max<0x102>(v);  // row_shl:2
  v = dpp_max<0x104>(v);  // row_shl:4
  v = dpp_max<0x108>(v);  // row_shl:8
  const int t16 = __builtin_amdgcn_readlane(v, 16), t48 = __builtin_amdgcn_readlane(v, 48);
  return (threadIdx.x & 16) ? v : max(v, (threadIdx.x & 32) ? t48 : t16);
}
// Maximum over the half, complete in its upper row (lanes 16-31, 48-63).
__device__ __forceinline__ int half_upper_max(int v) {
  v = dpp_max<0x128>(v);          // row_ror:8
  v = dpp_max<0x124>(v);          // row_ror:4
  v = dpp_max<0x122>(v);          // row_ror:2
  v = dpp_max<0x121>(v);          // row_ror:1
  return dpp_max<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
}
// Window maxima of one line: lane j holds a = x[j], b = x[2R + j] and c = a
// sample of [31, 2R]; returns the key of max x[j .. j + 2R].
__device__ __forceinline__ int line_max(int a, int b, int c) {
  const int C = half_upper_max(c);
  const int S = half_suffix_max((threadIdx.x & 31) == 31 ? C : a);
  return max(S, half_prefix_max(b));
}

// Merge the candidate t and flags fl into accumulator slot c; true for the
// n-th (last) arrival, which then holds the merged values and has cleared
// the slot.  Each step waits for the previous atomic's return value, so an
// arrival's maximum and flags are performed before its count increment, and
// the last arrival reads the slot (by exchange) only after its own increment
// returned: every merged value is seen without L2 writeback fences.
__device__ __forceinline__ bool acc_merge(RangeAccSlot *c, unsigned long long &t, int32_t &fl, uint32_t n) {
  // (zero is both merges' identity: an arrival with nothing to merge only counts)
  const unsigned long long om = t ? atomicMax(&c->T, t) : 0ull;
  const int32_t of = fl ? atomicOr(&c->flags, fl) : 0;
  uint32_t one = 1u;
  asm volatile("" : "+v"(one) : "v"(om), "v"(of));
  const uint32_t done = atomicAdd(&c->count, one);
  if (done != n - 1) return false;
  unsigned long long z = 0ull;
  int32_t zf = 0;
  asm volatile("" : "+v"(z), "+v"(zf) : "v"(done));
  t = atomicExch(&c->T, z);
  fl = atomicExch(&c->flags, zf);
  atomicExch(&c->count, 0u);
  return true;
}

// Tile statistics.  T = max over x of (max of f over the window of x) -
// f(x) is a maximum over the pixels, so the tile kernel may skip a block of
// outputs none of which can exceed a value T is known to reach; the result
// is unchanged.  Per 32 x 32 output tile this pass records the maximum and
// the minimum of f (as keys), and a lower bound of T: the largest
// (maximum - minimum) over the b x b sub-blocks of the tiles, b the largest
// power of two <= min(R + 1, 32) -- two samples of such a sub-block lie in
// each other's window, so T reaches their difference.  Tiles of a strip with
// a non-finite sample record (INT_MAX, INT_MIN), which no bound lets skip.
// One workgroup of 256 threads per strip of kStatTiles tiles down a column
// of tiles (all loads issued at once); thread (g, c) holds rows 4g..4g+3 of
// column c of each tile.
constexpr int kStatThreads = 256;
template <typename Tin>
__device__ __forceinline__ double key_diff(int mx, int mn) {
  return mx >= mn ? (double)tile_unkey<Tin>(mx) - (double)tile_unkey<Tin>(mn) : 0.0;
}
template <typename Tin>
__device__ __forceinline__ void range_stats_body(const RangeTileArgs &a, const Blk b) {
  constexpr int NT = kStatTiles;
  __shared__ int smx[NT][8][kTileW], smn[NT][8][kTileW];
  __shared__ double wlb[kStatThreads / 64];
  const Tin *__restrict__ f = (const Tin *)a.f;
  const int tid = threadIdx.x, c = tid & 31, g = tid >> 5, lane = tid & 63;
  const int x = b.x * kTileW + c, xc = min(x, a.W - 1);
  const int by0 = b.y * NT;
  float v[NT][4];
#pragma unroll
  for (int k = 0; k < NT; k++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int y = (by0 + k) * kTileH + 4 * g + i;
      v[k][i] = fval(f[(int64_t)min(y, a.H - 1) * a.pitch + xc]);
    }
  // sub-block size: a power of two <= min(R + 1, 32)
  int sb = 1;
  while (2 * sb <= min(a.R + 1, kTileW)) sb *= 2;
  bool bad = false;
  double lb = 0.0;
#pragma unroll
  for (int k = 0; k < NT; k++) {
    int kx[4], kn[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int y = (by0 + k) * kTileH + 4 * g + i;
      const bool in = x < a.W && y < a.H;
      const bool fin = isfinite(v[k][i]);
      if (in && !fin) bad = true;
      kx[i] = (in && fin) ? tile_key<Tin>(v[k][i]) : INT_MIN;
      kn[i] = (in && fin) ? tile_key<Tin>(v[k][i]) : INT_MAX;
    }
    if (sb == 2 || sb == 4) {  // sub-blocks inside the thread's four rows
      int m0 = sb == 2 ? max(kx[0], kx[1]) : max(max(kx[0], kx[1]), max(kx[2], kx[3]));
      int n0 = sb == 2 ? min(kn[0], kn[1]) : min(min(kn[0], kn[1]), min(kn[2], kn[3]));
      int m1 = sb == 2 ? max(kx[2], kx[3]) : INT_MIN;
      int n1 = sb == 2 ? min(kn[2], kn[3]) : INT_MAX;
      for (int o = 1; o < sb; o <<= 1) {
        m0 = max(m0, __shfl_xor(m0, o, 64));
        n0 = min(n0, __shfl_xor(n0, o, 64));
        m1 = max(m1, __shfl_xor(m1, o, 64));
        n1 = min(n1, __shfl_xor(n1, o, 64));
      }
      lb = fmax(lb, fmax(key_diff<Tin>(m0, n0), key_diff<Tin>(m1, n1)));
    }
    smx[k][g][c] = max(max(kx[0], kx[1]), max(kx[2], kx[3]));
    smn[k][g][c] = min(min(kn[0], kn[1]), min(kn[2], kn[3]));
  }
  bad = __syncthreads_or(bad) != 0;
  if (sb >= 8) {  // sub-blocks of sb / 4 row groups: segment g mod (32 / sb)
    const int rows = sb / 4, seg = g % (kTileW / sb);
#pragma unroll
    for (int k = 0; k < NT; k++) {
      int m = INT_MIN, n = INT_MAX;
      for (int r = 0; r < rows; r++) {
        m = max(m, smx[k][seg * rows + r][c]);
        n = min(n, smn[k][seg * rows + r][c]);
      }
      for (int o = 1; o < sb; o <<= 1) {
        m = max(m, __shfl_xor(m, o, 64));
        n = min(n, __shfl_xor(n, o, 64));
      }
      lb = fmax(lb, key_diff<Tin>(m, n));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lb = fmax(lb, __shfl_xor(lb, o, 64));
  if (lane == 0) wlb[tid >> 6] = lb;
  // tile k's maximum and minimum: wave k, one column per lane
  const int k = tid >> 6;
  if (k < NT && by0 + k < a.gg.gy) {
    int m = INT_MIN, n = INT_MAX;
#pragma unroll
    for (int r = 0; r < 8; r++) {
      m = max(m, smx[k][r][c]);
      n = min(n, smn[k][r][c]);
    }
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      m = max(m, __shfl_xor(m, o, 64));
      n = min(n, __shfl_xor(n, o, 64));
    }
    if (lane == 0) a.tstats[(by0 + k) * a.gg.gx + b.x] = bad ? make_int2(INT_MAX, INT_MIN) : make_int2(m, n);
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int w = 1; w < kStatThreads / 64; w++) lb = fmax(lb, wlb[w]);
    const int bl = b.y * a.gg.gx + b.x;
    if (!bad && lb > 0.0)
      atomicMax(a.acc.lb + bl % kRangeSubs, (unsigned long long)__double_as_longlong(lb));
  }
}
template <typename Tin>
__global__ __launch_bounds__(kStatThreads) void k_range_stats(RangeTileArgs a) {
  range_stats_body<Tin>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin>
__global__ __launch_bounds__(kStatThreads) void k_range_stats_grp(const RangeTileArgs *__restrict__ a,
                                                                   const int *__restrict__ start, int n) {
  const int i = group_find(start, n, blockIdx.x);
  range_stats_body<Tin>(a[i], group_blk(range_stats_grid(a[i].gg), blockIdx.x - start[i]));
}

// The largest lower bound of T merged by the statistics pass (0 without
// one), in every lane.
__device__ __forceinline__ double tile_lower_bound(const RangeTileArgs &a, int lane) {
  double l = (a.tstats && lane < kRangeSubs) ? __longlong_as_double((long long)a.acc.lb[lane]) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l = fmax(l, __shfl_xor(l, o, 64));
  return l;
}
// Tiles c0 + j nwg (j < 64) of the image that must be computed, as a lane
// mask: those inside the image whose bound -- the largest maximum of the
// tiles the windows of its outputs reach (R <= 48: at most two tiles away)
// minus its own minimum -- exceeds the lower bound lb.  Without statistics
// every tile inside the image.
template <typename Tin>
__device__ __forceinline__ unsigned long long tiles_to_compute(const RangeTileArgs &a, int c0, int nwg, int ntiles,
                                                               int lane, double lb) {
  const int t = c0 + lane * nwg;
  bool keep = t < ntiles;
  if (a.tstats) {
    const int gx = a.gg.gx, gy = a.gg.gy, tc = min(t, ntiles - 1);
    const int by = tc / gx, bx = tc - by * gx;
    const int rt = (a.R + kTileW - 1) / kTileW;
    int nmax = INT_MIN;
#pragma unroll
    for (int dy = -2; dy <= 2; dy++)
#pragma unroll
      for (int dx = -2; dx <= 2; dx++) {
        const int ty = by + dy, tx = bx + dx;
        const bool in = abs(dy) <= rt && abs(dx) <= rt && ty >= 0 && ty < gy && tx >= 0 && tx < gx;
        const int v = a.tstats[min(max(ty, 0), gy - 1) * gx + min(max(tx, 0), gx - 1)].x;
        nmax = in ? max(nmax, v) : nmax;
      }
    const double ub = (double)tile_unkey<Tin>(nmax) - (double)tile_unkey<Tin>(a.tstats[tc].y);
    keep = keep && !(ub <= lb);
  }
  return __ballot(keep);
}

// One output tile (bx, by) of the tile kernel: stages, filters, and folds
// its outputs' (window maximum - f) into tmax and its non-finite samples
// into bad.  Starts with a barrier (the previous tile's readers of LDS).
template <typename Tin, int KR>
__device__ __forceinline__ void range_tile_one(const RangeTileArgs &a, int bx, int by, bool &bad_out,
                                               double &tmax) {
  using KeyT = typename TileKey<Tin>::T;
  constexpr int RS = tile_rs<KR>();
  constexpr bool kFloat = std::is_same<Tin, float>::value;
  extern __shared__ float tlds[];
  const Tin *__restrict__ f = (const Tin *)a.f;
  const int64_t pitch = a.pitch;
  const int H = a.H, W = a.W, R = a.R;
  const int L = kTileH + 2 * R;   // staged rows
  const int Lc = kTileW + 2 * R;  // staged columns
  const int nc = 2 * R - 30;      // samples [31, 2R] common to every window of a line
  constexpr bool kGlob = tile_global_rows<Tin, KR>();
  KeyT *reg = (KeyT *)tlds;
  int *rm = (int *)tlds + (kGlob ? 0 : ((size_t)L * RS * sizeof(KeyT) + 3) / 4);
  float *fc = (float *)(rm + L * kTileMS);
  const int tid = threadIdx.x, lane = tid & 63, j = lane & 31, half = lane >> 5;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x0 = bx * kTileW, y0 = by * kTileH;
  const float pad = kFloat ? -INFINITY : 0.f;
  bool bad = false;
  __syncthreads();

  // stage: staged row e = wv + kTileWaves k, columns lane and lane + 64; every
  // lane loads from a clamped in-image address (no branch around the load,
  // so all loads stay in flight) and masks afterwards
  if constexpr (kGlob) {
    // only the centre samples: rows tid / 32 and tid / 32 + 16, column tid % 32
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int ce = (tid >> 5) + 16 * h, cc = tid & 31, y = y0 + ce, x = x0 + cc;
      const bool in = y < H && x < W;
      const float v = fval(f[(int64_t)min(y, H - 1) * pitch + min(x, W - 1)]);
      fc[ce * kTileMS + cc] = v;
      if (in && !isfinite(v)) bad = true;
    }
  } else {
    constexpr int kRows = (kTileH + 2 * KR) / kTileWaves;
    float v[kRows][2];
    const int xa = x0 - R + lane, xb = xa + 64;
    const int xac = min(max(xa, 0), W - 1), xbc = min(max(xb, 0), W - 1);
    const bool ina = xa >= 0 && xa < W, inb = lane + 64 < Lc && xb >= 0 && xb < W;
#pragma unroll
    for (int k = 0; k < kRows; k++) {
      const int e = wv + kTileWaves * k, y = y0 - R + e;
      const bool rin = e < L && y >= 0 && y < H;
      const Tin *row = f + (int64_t)min(max(y, 0), H - 1) * pitch;
      const float ra = fval(row[xac]), rb = fval(row[xbc]);
      v[k][0] = (rin && ina) ? ra : pad;
      v[k][1] = (rin && inb) ? rb : pad;
      if ((rin && ina && !isfinite(ra)) || (rin && inb && !isfinite(rb))) bad = true;
    }
#pragma unroll
    for (int k = 0; k < kRows; k++) {
      const int e = wv + kTileWaves * k;
      if (e < L) {
        reg[e * RS + lane] = (KeyT)tile_key<Tin>(v[k][0]);
        if (lane + 64 < Lc) reg[e * RS + lane + 64] = (KeyT)tile_key<Tin>(v[k][1]);
        // centre columns [R, R + 32): from the first load, and past column 64
        // (R > 32) from the second
        const int ce = e - R, cc = lane - R, cc2 = lane + 64 - R;
        if (ce >= 0 && ce < kTileH && cc >= 0 && cc < kTileW) fc[ce * kTileMS + cc] = v[k][0];
        if (KR > 32 && ce >= 0 && ce < kTileH && cc2 < kTileW) fc[ce * kTileMS + cc2] = v[k][1];
      }
    }
  }
  bad = __syncthreads_or(bad) != 0;
  bad_out = bad_out || bad;

  // row pass: staged row e = 2 it + half, four row pairs per wave in flight
  const int n1 = nc - 1, n2 = nc - 33, n3 = nc - 65;
  constexpr int U = 4;
  if constexpr (kGlob) {
    // R > 32 here, so the common piece takes two or three loads
    for (int it0 = wv; 2 * it0 < L; it0 += kTileWaves * U) {
      int av[U], bv[U], cv[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int y = y0 - R + 2 * (it0 + kTileWaves * u) + half;
        const bool rin = y >= 0 && y < H;
        const float *row = (const float *)f + (int64_t)min(max(y, 0), H - 1) * pitch;
        // key of staged column s: clamped load, -inf outside the image
        const auto key_at = [&](int s) {
          const int x = x0 - R + s;
          const float v = row[min(max(x, 0), W - 1)];
          return tile_key<Tin>((rin && x >= 0 && x < W) ? v : -INFINITY);
        };
        av[u] = key_at(j);
        bv[u] = key_at(2 * R + j);
        cv[u] = max(key_at(31 + min(j, n1)), key_at(63 + min(j, n2)));
        if (nc > 64) cv[u] = max(cv[u], key_at(95 + min(j, n3)));
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int e = 2 * (it0 + kTileWaves * u) + half;
        const int m = line_max(av[u], bv[u], cv[u]);
        if (e < L) rm[e * kTileMS + j] = m;
      }
    }
  } else if (R >= 16) {
    for (int it0 = wv; 2 * it0 < L; it0 += kTileWaves * U) {
      int av[U], bv[U], cv[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const KeyT *xr = reg + min(2 * (it0 + kTileWaves * u) + half, L - 1) * RS;
        av[u] = xr[j];
        bv[u] = xr[2 * R + j];
        cv[u] = xr[31 + min(j, n1)];
        if (nc > 32) cv[u] = max(cv[u], (int)xr[63 + min(j, n2)]);
        if (KR > 32 && nc > 64) cv[u] = max(cv[u], (int)xr[95 + min(j, n3)]);
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int e = 2 * (it0 + kTileWaves * u) + half;
        const int m = line_max(av[u], bv[u], cv[u]);
        if (e < L) rm[e * kTileMS + j] = m;
      }
    }
  } else {
    for (int it = wv; 2 * it < L; it += kTileWaves) {
      const int e = 2 * it + half;
      const KeyT *xr = reg + min(e, L - 1) * RS + j;
      int m = xr[0];
#pragma unroll 8
      for (int k = 1; k <= 2 * R; k++) m = max(m, (int)xr[k]);
      if (e < L) rm[e * kTileMS + j] = m;
    }
  }
  __syncthreads();

  // column pass: output column cc = 2 it + half, it = wv + kTileWaves u
  {
    constexpr int UC = kTileW / 2 / kTileWaves;
    int mv[UC];
    if (R >= 16) {
      int av[UC], bv[UC], cv[UC];
#pragma unroll
      for (int u = 0; u < UC; u++) {
        const int *col = rm + 2 * (wv + kTileWaves * u) + half;
        av[u] = col[j * kTileMS];
        bv[u] = col[(2 * R + j) * kTileMS];
        cv[u] = col[(31 + min(j, n1)) * kTileMS];
        if (nc > 32) cv[u] = max(cv[u], col[(63 + min(j, n2)) * kTileMS]);
        if (KR > 32 && nc > 64) cv[u] = max(cv[u], col[(95 + min(j, n3)) * kTileMS]);
      }
#pragma unroll
      for (int u = 0; u < UC; u++) mv[u] = line_max(av[u], bv[u], cv[u]);
    } else {
#pragma unroll
      for (int u = 0; u < UC; u++) {
        const int *col = rm + 2 * (wv + kTileWaves * u) + half + j * kTileMS;
        int m = col[0];
#pragma unroll 8
        for (int k = 1; k <= 2 * R; k++) m = max(m, col[k * kTileMS]);
        mv[u] = m;
      }
    }
#pragma unroll
    for (int u = 0; u < UC; u++) {
      const int cc = 2 * (wv + kTileWaves * u) + half;
      const double d = (double)tile_unkey<Tin>(mv[u]) - (double)fc[j * kTileMS + cc];
      tmax = (y0 + j < H && x0 + cc < W && d > tmax) ? d : tmax;
    }
  }
}

// Workgroup wg of nwg takes the image's tiles wg, wg + nwg, ...: per round of
// 64 of them, wave 0 finds those that must be computed (the others cannot
// raise T above the statistics pass's lower bound lb), then the workgroup
// computes them one after another.  T = max(lb, the computed tiles'
// maxima), merged once per workgroup.
template <typename Tin, int KR>
__device__ __forceinline__ void range_tile_body(const RangeTileArgs &a, const int wg) {
  __shared__ double wmax[kTileWaves];
  __shared__ unsigned long long todo_s[2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nwg = a.nwg, ntiles = a.gg.gx * a.gg.gy;
  const double lb = tile_lower_bound(a, lane);
  bool bad = false;
  double tmax = 0.0;
  for (int c0 = wg, r = 0; c0 < ntiles; c0 += 64 * nwg, r ^= 1) {
    if (wv == 0) {
      const unsigned long long m = tiles_to_compute<Tin>(a, c0, nwg, ntiles, lane, lb);
      if (lane == 0) todo_s[r] = m;
    }
    __syncthreads();  // (double-buffered: wave 0 writes the other slot next round)
    unsigned long long todo = todo_s[r];
    todo = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(todo >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)todo);
    while (todo) {
      const int jt = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int t = c0 + jt * nwg, by = t / a.gg.gx;
      range_tile_one<Tin, KR>(a, t - by * a.gg.gx, by, bad, tmax);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(tmax, off, 64);
    tmax = o > tmax ? o : tmax;
  }
  if (lane == 0) wmax[wv] = tmax;
  // also orders every wave's read of the lower bounds before the arrival
  // below (the last arrival clears them)
  __syncthreads();

  if (tid == 0) {
    tmax = wmax[0];
#pragma unroll
    for (int w = 1; w < kTileWaves; w++) tmax = fmax(tmax, wmax[w]);
    const int sub = wg % kRangeSubs, nsub = min(nwg, kRangeSubs);
    // the computed tiles' maximum only (non-negative: the bit patterns order
    // as the values); the lower bound joins at the publication
    unsigned long long t = (unsigned long long)__double_as_longlong(tmax);
    int32_t fl = bad ? 1 : 0;
    if (acc_merge(a.acc.sub + sub, t, fl, (uint32_t)((nwg - sub + kRangeSubs - 1) / kRangeSubs)) &&
        acc_merge(a.acc.top, t, fl, (uint32_t)nsub)) {
      t = (unsigned long long)__double_as_longlong(fmax(__longlong_as_double((long long)t), lb));
      const double tc = ceil(__longlong_as_double((long long)t));
      const int32_t ti = tc > 2147483647.0 ? 2147483647 : (int32_t)tc;
      const DevState st = a.st;
      *st.T_raw = t;
      *st.T_used = ti;
      *st.flags = fl | (ti > a.T_cap ? 2 : 0);
      *st.q_nonpos = 0ull;
      if (a.tstats) {
#pragma unroll 4
        for (int k = 0; k < kRangeSubs; k++) atomicExch(a.acc.lb + k, 0ull);
      }
    }
  }
}
template <typename Tin, int KR>
__global__ __launch_bounds__(kTileThreads) void k_range_tile(RangeTileArgs a) {
  range_tile_body<Tin, KR>(a, (int)blockIdx.x);
}
template <typename Tin, int KR>
__global__ __launch_bounds__(kTileThreads) void k_range_tile_grp(const RangeTileArgs *__restrict__ a,
                                                                 const int *__restrict__ start, int n) {
  const int i = group_find(start, n, blockIdx.x);
  range_tile_body<Tin, KR>(a[i], __builtin_amdgcn_readfirstlane((int)blockIdx.x - start[i]));
}

// --------------------------------------------- blocked recursive Gaussian
// Both passes filter a padded line (a column in the vertical pass, a row in
// the horizontal one) with the causal and then the anticausal cascade.  The
// line is split over a row group of S threads, thread t owning the kC
// consecutive samples [t kC, t kC + kC): each thread runs its samples from
// rest, the chunk end states are scanned across the group (powers of A^kC),
// and each sample takes the correction w += (row 1 of A^i) . carry; the same
// for the anticausal direction, seeded at the padded end with the
// zero-extension boundary.
//
// Positions p index the padded row in an interleaved order: p -> column
// x = (p mod Seff) * c + p / Seff (Seff = ceil(W / c) threads of the row
// group hold positions), so that the horizontal pass, where thread t owns
// columns [t c, t c + c), reads consecutive addresses.

// Lane moves inside a wave through DPP (VALU only, no LDS round trip).  Lanes
// whose source falls outside the pattern, or whose row the row mask leaves
// out, read zero.
template <int CTRL, int ROWMASK = 0xF, bool BOUND0 = true>
__device__ __forceinline__ float4 dpp4(float4 v) {
  auto m = [](float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xF, BOUND0));
  };
  return make_float4(m(v.x), m(v.y), m(v.z), m(v.w));
}
__device__ __forceinline__ float4 keep4(bool k, float4 v) { return k ? v : f4(0.f); }
constexpr int kDppRowShl = 0x100, kDppRowShr = 0x110, kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138,
              kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// Inclusive scans of the chunk states across the SW lanes of a row group
// (SW a power of two, groups aligned within the wave): state(t) =
// sum_i A^{c |t - i|} x_i over i <= t (up) or i >= t (down).  sA holds A^{c m}
// for m = 0..64.  Inside each 16-lane row a Hillis-Steele scan with DPP row
// shifts; then the row totals are carried to the following rows with the
// lane's own power of A^c.
template <int D, int SW>
__device__ __forceinline__ void up_step(float4 v[3], const float *__restrict__ M, int ls) {
  float4 o[3];
#pragma unroll
  for (int r = 0; r < 3; r++) o[r] = keep4(SW >= 16 || ls >= D, dpp4<kDppRowShr + D>(v[r]));
  apow_acc(M, o, v);
}
template <int D, int SW>
__device__ __forceinline__ void down_step(float4 v[3], const float *__restrict__ M, int ls) {
  float4 o[3];
#pragma unroll
  for (int r = 0; r < 3; r++) o[r] = keep4(SW >= 16 || ls + D < SW, dpp4<kDppRowShl + D>(v[r]));
  apow_acc(M, o, v);
}
template <int SW>
__device__ __forceinline__ void scan_up(float4 v[3], const float *__restrict__ sA, int ls, int lane) {
  if constexpr (SW > 1) up_step<1, SW>(v, sA + 9 * 1, ls);
  if constexpr (SW > 2) up_step<2, SW>(v, sA + 9 * 2, ls);
  if constexpr (SW > 4) up_step<4, SW>(v, sA + 9 * 4, ls);
  if constexpr (SW > 8) up_step<8, SW>(v, sA + 9 * 8, ls);
  const int j = lane & 15;
  if constexpr (SW >= 32) {  // rows 1 and 3 take the totals of rows 0 and 2
    float4 o[3];
#pragma unroll
    for (int r = 0; r < 3; r++) o[r] = dpp4<kDppRowBcast15, 0xA, false>(v[r]);
    apow_acc(sA + 9 * (j + 1), o, v);
  }
  if constexpr (SW == 64) {  // rows 2 and 3 take the total of lanes 0..31
    float4 o[3];
#pragma unroll
    for (int r = 0; r < 3; r++) o[r] = dpp4<kDppRowBcast31, 0xC, false>(v[r]);
    apow_acc(sA + 9 * max(lane - 31, 0), o, v);
  }
}
template <int SW>
__device__ __forceinline__ void scan_down(float4 v[3], const float *__restrict__ sA, int ls, int lane) {
  if constexpr (SW > 1) down_step<1, SW>(v, sA + 9 * 1, ls);
  if constexpr (SW > 2) down_step<2, SW>(v, sA + 9 * 2, ls);
  if constexpr (SW > 4) down_step<4, SW>(v, sA + 9 * 4, ls);
  if constexpr (SW > 8) down_step<8, SW>(v, sA + 9 * 8, ls);
  const int j = lane & 15;
  if constexpr (SW >= 32) {  // rows 0 and 2 take the totals of rows 1 and 3 (from their first lane)
    const int src = (lane & 32) + 16;
    const bool even = ((lane >> 4) & 1) == 0;
    float4 o[3];
#pragma unroll
    for (int r = 0; r < 3; r++)
      o[r] = keep4(even, make_float4(__shfl(v[r].x, src, 64), __shfl(v[r].y, src, 64), __shfl(v[r].z, src, 64),
                                     __shfl(v[r].w, src, 64)));
    apow_acc(sA + 9 * (16 - j), o, v);
  }
  if constexpr (SW == 64) {  // rows 0 and 1 take the total of lanes 32..63
    const bool lo = lane < 32;
    float4 o[3];
#pragma unroll
    for (int r = 0; r < 3; r++)
      o[r] = keep4(lo, make_float4(lane_value(v[r].x, 32), lane_value(v[r].y, 32), lane_value(v[r].z, 32),
                                   lane_value(v[r].w, 32)));
    apow_acc(sA + 9 * max(32 - lane, 0), o, v);
  }
}
// z += row 1 of M times u (the w-component response to the state u)
// Read-only constants of a launch, addressed as constant memory: loads with
// a uniform address become scalar loads whatever the pointer's origin.
typedef const __attribute__((address_space(4))) float *cfloat_p;
__device__ __forceinline__ cfloat_p as_const(const float *p) { return (cfloat_p)p; }
// r = M u for M a power of A read from constant memory (first row (m00, 0, 0))
__device__ __forceinline__ void apow_mul_c(cfloat_p M, const float4 u[3], float4 r[3]) {
  r[0] = make_float4(M[0] * u[0].x, M[0] * u[0].y, M[0] * u[0].z, M[0] * u[0].w);
#pragma unroll
  for (int i = 1; i < 3; i++) {
    float4 a = make_float4(M[3 * i] * u[0].x, M[3 * i] * u[0].y, M[3 * i] * u[0].z, M[3 * i] * u[0].w);
    a = fma4(M[3 * i + 1], u[1], a);
    r[i] = fma4(M[3 * i + 2], u[2], a);
  }
}

__device__ __forceinline__ void row1_acc(cfloat_p M, const float4 u[3], float4 &z) {
  z = fma4(M[3], u[0], z);
  z = fma4(M[4], u[1], z);
  z = fma4(M[5], u[2], z);
}

// Constants of the blocked filter in LDS: A^{c m} for m = 0..64 and the end
// boundary (the scans read them in divergent code, where constants from
// memory would cost a round trip).
struct IirLds {
  float A[65 * 9];
  float Mts[9];
};
// Fetched into registers first and written to LDS later, so that loads
// issued in between (memory counters complete in order) need not be waited
// for before the tables are stored.
struct IirLdsRegs {
  float a[3], w, m;
};
template <int kC>
__device__ __forceinline__ IirLdsRegs fetch_iir_lds(const float *__restrict__ iir, int tid) {
  const float *hb = iir + (kC == kCSmall ? kIirHSmall : kIirHLarge);
  IirLdsRegs r;
#pragma unroll
  for (int j = 0; j < 3; j++) {
    const int i = tid + j * kHThreads;
    r.a[j] = i < 64 * 9 ? hb[iir_h_lane(kC) + i] : 0.f;
  }
  r.w = tid < 9 ? hb[iir_h_wave(kC) + tid] : 0.f;
  r.m = tid < 9 ? iir[kIirMts + tid] : 0.f;
  return r;
}
__device__ __forceinline__ void store_iir_lds(IirLds &L, const IirLdsRegs &r, int tid) {
#pragma unroll
  for (int j = 0; j < 3; j++) {
    const int i = tid + j * kHThreads;
    if (i < 64 * 9) L.A[i] = r.a[j];
  }
  if (tid < 9) {
    L.A[64 * 9 + tid] = r.w;
    L.Mts[tid] = r.m;
  }
}

// The causal and anticausal cascade over one line held by a row group of S
// threads (zv: this thread's kC samples, in place).  xw: this group's LDS
// slots for the wave carries (S > 64); every thread of the workgroup calls it
// (it holds barriers when S > 64).  The line ends with thread tlast's chunk:
// the zero extension starts there, and the threads after it (whatever their
// samples) pass nothing to the others and their outputs are not defined.
template <int S, int kC>
__device__ __forceinline__ void group_blur(float4 zv[kC], float a1, float g2, float c2, const IirLds &L,
                                           cfloat_p Apow, float4 (*xw)[3], int t, int lane, int tlast = S - 1) {
  constexpr int SW = S < 64 ? S : 64;
  constexpr int NW = S > 64 ? S / 64 : 1;
  const int ls = t % SW;
  const int wig = t / 64;
  const float *sA = L.A;
  const float *waveM = L.A + 9 * 64;
  // causal sweep from rest
  float4 s = f4(0.f), w = f4(0.f), d = f4(0.f);
#pragma unroll
  for (int i = 0; i < kC; i++) {
    casc_step(a1, g2, c2, zv[i], s, w, d);
    zv[i] = w;
  }
  float4 inc[3] = {s, w, d};
  scan_up<SW>(inc, sA, ls, lane);
  float4 exc[3];
#pragma unroll
  for (int r = 0; r < 3; r++) exc[r] = keep4(ls != 0, dpp4<kDppWaveShr1>(inc[r]));
  if constexpr (NW > 1) {
    if (ls == 63) {
#pragma unroll
      for (int r = 0; r < 3; r++) xw[wig][r] = inc[r];
    }
    __syncthreads();
    float4 Kc[3] = {f4(0.f), f4(0.f), f4(0.f)};
    for (int v = 0; v < wig; v++) {
      float4 tk[3];
      apow_mul(waveM, Kc, tk);
#pragma unroll
      for (int r = 0; r < 3; r++) Kc[r] = add4(xw[v][r], tk[r]);
    }
    __syncthreads();
    apow_acc(sA + 9 * ls, Kc, exc);
    // the line's last thread also needs its inclusive state: the carry
    // through its own chunk too (A^(c (ls + 1)); the wave matrix when it is
    // a wave's last lane)
    if (t == tlast) apow_acc(sA + 9 * (ls + 1), Kc, inc);
  }
  // true causal outputs.  In blocks of 16 samples: block b takes the carry
  // A^(16 b) exc, so that only the w rows of A^1..A^16 and A^16 itself are
  // needed (they stay in scalar registers)
  {
    float4 cb[3] = {exc[0], exc[1], exc[2]};
#pragma unroll
    for (int b0 = 0; b0 < kC; b0 += 16) {
      if (b0 > 0) {
        float4 nb[3];
        apow_mul_c(Apow + 9 * 16, cb, nb);
#pragma unroll
        for (int r = 0; r < 3; r++) cb[r] = nb[r];
      }
#pragma unroll
      for (int j = 0; j < (kC < 16 ? kC : 16); j++) row1_acc(Apow + 9 * (j + 1), cb, zv[b0 + j]);
    }
  }
  // zero extension beyond the line's end
  float4 Eb[3] = {f4(0.f), f4(0.f), f4(0.f)};
  if (t == tlast) matvec3(L.Mts, inc, Eb);
  // anticausal sweep from rest
  s = f4(0.f);
  w = f4(0.f);
  d = f4(0.f);
#pragma unroll
  for (int i = kC - 1; i >= 0; i--) {
    casc_step(a1, g2, c2, zv[i], s, w, d);
    zv[i] = w;
  }
  float4 hd[3] = {keep4(t <= tlast, s), keep4(t <= tlast, w), keep4(t <= tlast, d)};
  if (t == tlast) apow_acc(sA + 9, Eb, hd);  // A^c
  scan_down<SW>(hd, sA, ls, lane);
  float4 ein[3];
#pragma unroll
  for (int r = 0; r < 3; r++) ein[r] = keep4(ls != SW - 1, dpp4<kDppWaveShl1>(hd[r]));
  if constexpr (NW > 1) {
    if (ls == 0) {
#pragma unroll
      for (int r = 0; r < 3; r++) xw[wig][r] = hd[r];
    }
    __syncthreads();
    float4 Kc[3] = {f4(0.f), f4(0.f), f4(0.f)};
    for (int v = NW - 1; v > wig; v--) {
      float4 tk[3];
      apow_mul(waveM, Kc, tk);
#pragma unroll
      for (int r = 0; r < 3; r++) Kc[r] = add4(xw[v][r], tk[r]);
    }
    __syncthreads();
    apow_acc(sA + 9 * (63 - ls), Kc, ein);
  }
  if (t == tlast) {
#pragma unroll
    for (int r = 0; r < 3; r++) ein[r] = Eb[r];
  }
  // the anticausal corrections in the same blocks of 16, from the end
  {
    float4 cb[3] = {ein[0], ein[1], ein[2]};
#pragma unroll
    for (int b1 = kC; b1 > 0; b1 -= 16) {
      if (b1 < kC) {
        float4 nb[3];
        apow_mul_c(Apow + 9 * 16, cb, nb);
#pragma unroll
        for (int r = 0; r < 3; r++) cb[r] = nb[r];
      }
      constexpr int n = kC < 16 ? kC : 16;
#pragma unroll
      for (int j = 0; j < n; j++) row1_acc(Apow + 9 * (n - j), cb, zv[b1 - n + j]);
    }
  }
}

// ------------------------------------------------ vertical pass (a3, a4)
// One workgroup per (NG consecutive positions, pair); a row group of SV
// threads per column, thread t owning rows [t kC, t kC + kC).  The four
// images of the pair are generated from f at those rows (eq. (f1), (f2)
// integrands, a3), smoothed down the column and written once.  Padding
// columns (positions past the image width) are written as zeros.
template <typename Tin, int SV, int kC>
__device__ __forceinline__ void iir_v_impl(const Tin *__restrict__ f, const Geom &g, const DevTables &tab, const DevState &st, const float *__restrict__ iir, int k0, int kcount, float4 *__restrict__ Z, float2 *__restrict__ glut, const Blk b) {
  constexpr int NG = kHThreads / SV;
  constexpr int NW = SV > 64 ? SV / 64 : 1;
  constexpr bool kLut = PhaseLut<Tin>::kOn;
  // tile height of the smoothed images (2^ZL rows, the host's zlog for this
  // column group size)
  constexpr int ZL = NG >= 16 ? 0 : (NG == 8 ? 1 : 2);
  __shared__ float4 xw[NG][NW][3];
  __shared__ IirLds L;
  // 8-bit inputs: cos/sin per intensity and a zero entry for the samples
  // outside the image, double-buffered over the workgroup's pairs
  __shared__ float2 lut[kLut ? 2 * 257 : 1];
  // each thread's samples, kept for the workgroup's later pairs; 8-bit
  // inputs keep the table index instead (256, the zero entry, for samples
  // outside the image), so that no per-sample predicate stays live
  typedef typename std::conditional<kLut, uint16_t, Tin>::type Ts;
  constexpr int kQ = kC * (int)sizeof(Ts) / 16;  // 16-byte words per thread
  __shared__ uint4 fs[kHThreads * kQ];
  const int tid = threadIdx.x;
  const int t = tid % SV;
  const int grp = tid / SV;
  // column blocks in XCD order: the workgroups whose columns share the lines
  // of a Z row run on one XCD, whose L2 merges their partial-line writes
  const int ncb = (g.Spos + NG - 1) / NG;
  const int per = (ncb + 7) / 8;
  const int cbx = (b.x & 7) * per + (b.x >> 3);
  if (cbx >= ncb) return;  // the whole workgroup: past the last column block
  const UEntry e = uniform_entry(tab, st.T_used);
  // this workgroup's pairs: launch-local [kb, kend)
  const int kb = b.y * g.vppw;
  const int kend = min(min(kb + g.vppw, kcount), e.K - k0);
  if (kb >= kend) return;  // the whole workgroup: no pair kept for this image's T
  const int p = cbx * NG + grp;
  const bool inpos = p < g.Spos;
  const int x = inpos ? (p % g.Seff) * g.cC + p / g.Seff : 0;
  const bool col = inpos && x < g.W;  // a column of the image (else zeros)
  const int y0 = t * kC;
  const int xc = min(x, g.W - 1);
  int32_t m = const_load(tab.pm + e.off + k0 + kb);
  const IirLdsRegs tr = fetch_iir_lds<kC>(iir, tid);
  // this thread's samples, requested before the table set-up and kept in its
  // own LDS slot for all the workgroup's pairs
  {
    Tin fl[kC];
#pragma unroll
    for (int i = 0; i < kC; i++) fl[i] = f[(int64_t)min(y0 + i, g.H - 1) * g.pitch + xc];
    store_iir_lds(L, tr, tid);
    union { Ts v[kC]; uint4 q[kQ]; } u;
#pragma unroll
    for (int i = 0; i < kC; i++) {
      if constexpr (kLut) u.v[i] = (col && y0 + i < g.H) ? (Ts)fl[i] : (Ts)256;
      else u.v[i] = fl[i];
    }
#pragma unroll
    for (int j = 0; j < kQ; j++) fs[tid * kQ + j] = u.q[j];
  }
  const float a1 = iir[kIirCoef + 0], g2 = iir[kIirCoef + 1], c2 = iir[kIirCoef + 2];
  cfloat_p Apow = as_const(iir + (kC == kCSmall ? kIirHSmall : kIirHLarge) + iir_h_apow(kC));
  for (int kl = kb; kl < kend; kl++) {
    const int it = kl - kb;
    float2 *lt = lut + (it & 1) * 257;
    if constexpr (kLut) {
      // the other buffer was last read before the previous pair's barrier.
      // One workgroup per pair also leaves the table for the horizontal
      // pass, times the pair's weight (eqs. (f1), (f2)), which the
      // horizontal pass then need not apply per pixel
      if (tab.lut_gen) {
        // polynomial kernel: basis values per intensity from the table; the
        // horizontal pass combines with the coefficients instead
        const size_t row = (size_t)(e.off + k0 + kl) * 256 + tid;
        lt[tid] = tab.lut_gen[row];
        if (cbx == 0) {
          const float w = const_load(tab.pc + e.off + k0 + kl);
          const float2 cc = tab.lut_comb[row];
          glut[(size_t)kl * 256 + tid] = make_float2(w * cc.x, w * cc.y);
        }
      } else {
        build_lut(lt, m, e.qfix, e.alpha_turn, tid, kHThreads);
        if (cbx == 0) {
          const float w = const_load(tab.pc + e.off + k0 + kl);
          const float2 cs = lt[tid];
          glut[(size_t)kl * 256 + tid] = make_float2(w * cs.x, w * cs.y);
        }
      }
      if (tid == 0) lt[256] = make_float2(0.f, 0.f);
      __syncthreads();
    } else if (it == 0) {
      __syncthreads();  // the filter constants
    }
    const Freq fq = make_freq(m, e.qfix, e.alpha_turn);
    if (kl + 1 < kend) m = const_load(tab.pm + e.off + k0 + kl + 1);
    // samples of this thread inside the image: the tests below stay inside
    // the loop (the empty asm hides that nv does not change; hoisted, they
    // would hold 32 lane masks in scalar registers)
    int nv = col ? min(max(g.H - y0, 0), kC) : 0;
    if constexpr (!kLut) asm volatile("" : "+v"(nv));
    Ts fv[kC];
    {
      union { Ts v[kC]; uint4 q[kQ]; } u;
#pragma unroll
      for (int j = 0; j < kQ; j++) u.q[j] = fs[tid * kQ + j];
#pragma unroll
      for (int i = 0; i < kC; i++) fv[i] = u.v[i];
    }
    float4 zv[kC];
#pragma unroll
    for (int i = 0; i < kC; i++) {
      if constexpr (kLut) {
        // index 256 reads (0, 0): all four images vanish whatever d is
        const float2 cs = lt[fv[i]];
        const float d = (float)fv[i] - g.center;
        zv[i] = make_float4(d * cs.x, d * cs.y, cs.x, cs.y);
      } else {
        zv[i] = i < nv ? planes<Tin>(fv[i], fq, g.center) : f4(0.f);
      }
    }
    group_blur<SV, kC>(zv, a1, g2, c2, L, Apow, xw[grp], t, tid & 63);
    if (inpos) {
      // y0 is a multiple of the tile height: row y0 + i sits at the thread's
      // first row plus an offset that is the same in every lane
      // rows y0 .. y0+kC-1 by tiles of 2^ZL rows: consecutive elements
      // inside a tile, one pointer step of Spos 2^ZL elements between tiles
      float4 *q = Z + (size_t)kl * g.Hz * g.Spos + z_index(g, y0, p);
      const size_t step = (size_t)g.Spos << ZL;
      if (y0 + kC <= g.H) {  // the whole chunk inside the image: no per-row test
#pragma unroll
        for (int b = 0; b < (kC >> ZL); b++) {
#pragma unroll
          for (int r = 0; r < (1 << ZL); r++) q[r] = zv[(b << ZL) + r];
          q += step;
        }
      } else {
#pragma unroll
        for (int b = 0; b < (kC >> ZL); b++) {
#pragma unroll
          for (int r = 0; r < (1 << ZL); r++)
            if (y0 + (b << ZL) + r < g.H) q[r] = zv[(b << ZL) + r];
          q += step;
        }
      }
    }
  }
}
// The bodies copy the small argument structs into locals: read through a
// reference into memory they could alias the kernel's stores, and the
// compiler would keep their fields in vector registers.
template <typename Tin, int SV, int kC>
__device__ __forceinline__ void iir_v_body(const IirArgs &a, const Blk b) {
  const Geom g = a.g;
  const DevTables tab = a.tab;
  const DevState st = a.st;
  iir_v_impl<Tin, SV, kC>((const Tin *)a.f, g, tab, st, a.iir, a.k0, a.kcount, a.Z, a.glut, b);
}
// Workgroups per CU the vertical kernel is compiled for: 32 rows per thread
// hold 128 VGPRs of samples (two waves per SIMD), 16 rows half that (three
// waves fit 168 VGPRs without spills).
template <int kC>
constexpr int v_blocks_per_cu() {
  return kC == kCSmall ? 3 : 2;
}
template <typename Tin, int SV, int kC>
__global__ __launch_bounds__(kHThreads, v_blocks_per_cu<kC>()) void k_iir_v(IirArgs a) {
  iir_v_body<Tin, SV, kC>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin, int SV, int kC>
__global__ __launch_bounds__(kHThreads, v_blocks_per_cu<kC>()) void k_iir_v_grp(const IirArgs *__restrict__ a, const int *__restrict__ start,
                                                     int n) {
  const int i = group_find(start, n, blockIdx.x);
  const IirArgs ai = a[i];
  iir_v_body<Tin, SV, kC>(ai, group_blk(ai.gg, blockIdx.x - start[i]));
}

// ------------------------------------ horizontal pass + accumulate (a4, a5)
// One workgroup per (hrows image rows, pair group); S threads per row group,
// NG = 256/S groups: hrows rows of PW = NG/hrows groups each, the PW groups
// of a row taking every PW-th frequency of the pair group (hrows > 1 when a
// pair group holds too few pairs to keep NG groups busy).  Each group
// smooths its pair's four images along its row and combines them at once
// into the numerator and the denominator (eqs. (f1), (f2)) with the phases
// regenerated at each pixel.
template <typename Tin, int S, int kC>
__device__ __forceinline__ void iir_h_accum_impl(const Tin *__restrict__ f, float *__restrict__ out, const Geom &g, const DevTables &tab, const DevState &st, const float *__restrict__ iir, int k0, int kcount, const float4 *__restrict__ Z, float2 *__restrict__ PQ, int first, int last, const float2 *__restrict__ glut, const Blk b) {

  constexpr int NG = kHThreads / S;
  constexpr int NW = S > 64 ? S / 64 : 1;
  constexpr int PAD = S * (kC + 1);  // LDS row of one group, one slot skipped per kC
  // 8-bit inputs: the cos/sin tables of the groups' current pairs, copied to
  // LDS when that still leaves room for two workgroups per CU
  constexpr bool kLutLds = PhaseLut<Tin>::kOn && NG <= 8 && NG * PAD * 8 + NG * 2048 <= 80 * 1024;
  // (P, Q) per group and pixel; slot (grp, t, i) belongs to one thread until the
  // groups of a row are summed at the end
  __shared__ float2 spq[NG * PAD];
  __shared__ float4 xw[NG][NW][3];
  __shared__ float2 slut[kLutLds ? NG * 256 : 1];
  __shared__ IirLds L;
  const int hrows = g.hrows;      // rows per workgroup (a power of two <= NG)
  const int PW = NG / hrows;      // pairs in flight per row
  // row blocks in XCD order: the workgroups of consecutive rows (which share
  // the cache lines of tiled smoothed images) run on one XCD
  const int nrb = (g.H + hrows - 1) / hrows;
  const int per = (nrb + 7) / 8;
  const int rb = (b.x & 7) * per + (b.x >> 3);
  if (rb >= nrb) return;  // the whole workgroup: past the last row
  const int pg = b.y;  // pair group: launch-local pairs [kb, kb + hkpg)
  const int tid = threadIdx.x;
  const int t = tid % S;
  const int grp = tid / S;
  const int rsub = grp / PW, plane = grp % PW;
  // rows past the image (last block only) smooth a copy of the last row and
  // store nothing; they still take part in the group's barriers
  const int y = min(rb * hrows + rsub, g.H - 1);
  const UEntry e = uniform_entry(tab, st.T_used);
  const int kb = pg * g.hkpg;
  const int kend = min(min(kb + g.hkpg, kcount), e.K - k0);
  const int niter = kend > kb ? (kend - kb + PW - 1) / PW : 0;
  const bool finish = last && g.hgroups == 1;
  if (niter == 0 && !first && !finish) return;  // no pairs here: partial sums unchanged
  const float a1 = iir[kIirCoef + 0], g2 = iir[kIirCoef + 1], c2 = iir[kIirCoef + 2];
  cfloat_p Apow = as_const(iir + (kC == kCSmall ? kIirHSmall : kIirHLarge) + iir_h_apow(kC));
  const Tin *frow = f + (int64_t)y * g.pitch;
  const int x0 = t * kC;
  const int qs = 1 << g.zlog;  // position stride of the smoothed images
  const IirLdsRegs tr = fetch_iir_lds<kC>(iir, tid);
  // the row's samples and the first pair's smoothed images are requested
  // before the table set-up, so that their latency overlaps it
  Tin fv[kC];
#pragma unroll
  for (int i = 0; i < kC; i++) fv[i] = frow[min(x0 + i, g.W - 1)];
  // threads past the row's positions (t >= Seff) load from position 0.  The
  // line ends with thread Seff - 1, so that what they smooth reaches no one
  // (3 selects per pair instead of 4 kC).  16-bit input instead smooths zeros
  // there and keeps the line at the whole group: at its register budget the
  // other form spills one more register.
  constexpr bool kZeroTail = std::is_same<Tin, uint16_t>::value;
  const bool tin = t < g.Seff;
  const int tq = tin ? t : 0;
  const int tlast = kZeroTail ? S - 1 : g.Seff - 1;
  const size_t qstep = (size_t)g.Seff * qs;
  float4 zv[kC];
  {
    const int kl = kb + plane;
    const float4 *q = Z + (size_t)(kl < kend ? kl : 0) * g.Hz * g.Spos + z_index(g, y, tq);
#pragma unroll
    for (int i = 0; i < kC; i++, q += qstep) zv[i] = kZeroTail ? keep4(tin, *q) : *q;
  }
  store_iir_lds(L, tr, tid);
  __syncthreads();
  float2 *mypq = spq + grp * PAD + t * (kC + 1);
#pragma unroll
  for (int i = 0; i < kC; i++) mypq[i] = make_float2(0.f, 0.f);

  for (int it = 0; it < niter; it++) {
    const int kl = kb + it * PW + plane;
    const bool act = kl < kend;
    if constexpr (kLutLds) {
      __syncthreads();  // the previous pairs' tables are no longer read
      if (act && rsub == 0)  // one copy per pair in flight, shared by the rows
        for (int i = t; i < 256; i += S) slut[plane * 256 + i] = glut[(size_t)kl * 256 + i];
      __syncthreads();
    }
    if (it > 0) {
      const float4 *q = Z + (size_t)(act ? kl : 0) * g.Hz * g.Spos + z_index(g, y, tq);
#pragma unroll
      for (int i = 0; i < kC; i++, q += qstep) zv[i] = kZeroTail ? keep4(tin, *q) : *q;
    }
    group_blur<S, kC>(zv, a1, g2, c2, L, Apow, xw[grp], t, tid & 63, tlast);
    // eqs. (f1), (f2): weight by the phase at the output pixel
    if (act) {
      const int k = k0 + kl;
      const int32_t m = tab.pm[e.off + k];
      const float cp = tab.pc[e.off + k];
      const uint64_t q = e.qfix;
      const double at = e.alpha_turn;
      const float2 *lk = glut + (size_t)kl * 256;
      auto combine = [&](int i) {
        float2 pq = mypq[i];
        if constexpr (PhaseLut<Tin>::kOn) {
          // the table holds the pair's weight times cos and sin
          const float2 cs = kLutLds ? slut[plane * 256 + (int)fv[i]] : lk[(int)fv[i]];
          pq.x = fmaf(cs.x, zv[i].x, fmaf(cs.y, zv[i].y, pq.x));
          pq.y = fmaf(cs.x, zv[i].z, fmaf(cs.y, zv[i].w, pq.y));
        } else {
          float c, sn;
          turn_sincos(phase_turn<Tin>(m, fv[i], q, at), c, sn);
          pq.x = fmaf(cp, fmaf(c, zv[i].x, sn * zv[i].y), pq.x);
          pq.y = fmaf(cp, fmaf(c, zv[i].z, sn * zv[i].w), pq.y);
        }
        mypq[i] = pq;
      };
      if constexpr (PhaseLut<Tin>::kOn && !kLutLds) {
        // table reads from memory: none for the columns past the image
        // (the test kept in the loop: hoisted, the kC tests would hold lane
        // masks in scalar registers)
        int nx = min(max(g.W - x0, 0), kC);
        asm volatile("" : "+v"(nx));
#pragma unroll
        for (int i = 0; i < kC; i++)
          if (i < nx) combine(i);
      } else {
        // every slot of the thread, also those of columns past the image (its
        // samples there repeat the last column's, so the values stay finite):
        // they are in the thread's own LDS range and never read back, and no
        // per-column test is needed
#pragma unroll
        for (int i = 0; i < kC; i++) combine(i);
      }
    }
  }
  // sum the groups of each row in a fixed order
  __syncthreads();
  float2 *PQg = PQ + (size_t)pg * g.H * g.W;
  unsigned long long nbad = 0;
  const int nrow = min(hrows, g.H - rb * hrows);
  for (int idx = tid; idx < nrow * g.W; idx += kHThreads) {
    const int r = idx / g.W, x = idx - r * g.W;
    const int yr = rb * hrows + r;
    const int o = (x / kC) * (kC + 1) + (x % kC);
    float P = 0.f, Q = 0.f;
    for (int pl = 0; pl < PW; pl++) {
      const float2 pq = spq[(r * PW + pl) * PAD + o];
      P += pq.x;
      Q += pq.y;
    }
    const size_t pix = (size_t)yr * g.W + x;
    if (!first) {
      float2 pq = PQg[pix];
      P += pq.x;
      Q += pq.y;
    }
    if (finish) {
      float rr = P / Q;
      float v;
      if (Q > 0.f && isfinite(rr)) {
        v = g.center + rr;
      } else {
        v = fval(f[(int64_t)yr * g.pitch + x]);
        nbad++;
      }
      out[(int64_t)yr * g.opitch + x] = v;
    } else {
      PQg[pix] = make_float2(P, Q);
    }
  }
  if (finish) {
    for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off, 64);
    if ((tid & 63) == 0 && nbad) atomicAdd(st.q_nonpos, nbad);
  }
}
template <typename Tin, int S, int kC>
__device__ __forceinline__ void iir_h_accum_body(const IirArgs &a, const Blk b) {
  const Geom g = a.g;
  const DevTables tab = a.tab;
  const DevState st = a.st;
  iir_h_accum_impl<Tin, S, kC>((const Tin *)a.f, a.out, g, tab, st, a.iir, a.k0, a.kcount, a.Z, a.PQ, a.first, a.last, a.glut, b);
}

// Workgroups per CU the horizontal kernel is compiled for: with 16 samples
// per thread, 8- and 16-bit input fits 168 VGPRs (3 waves per SIMD, the
// recursion's dependent chains overlap better); float input would spill.
template <typename Tin, int kC>
constexpr int h_blocks_per_cu() {
  return kC == kCSmall ? (std::is_same<Tin, float>::value ? 2 : 3) : 1;
}
template <typename Tin, int S, int kC>
__global__ __launch_bounds__(kHThreads, (h_blocks_per_cu<Tin, kC>())) void k_iir_h_accum(IirArgs a) {
  iir_h_accum_body<Tin, S, kC>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin, int S, int kC>
__global__ __launch_bounds__(kHThreads, (h_blocks_per_cu<Tin, kC>())) void k_iir_h_accum_grp(const IirArgs *__restrict__ a, const int *__restrict__ start,
                                                     int n) {
  const int i = group_find(start, n, blockIdx.x);
  const IirArgs ai = a[i];
  iir_h_accum_body<Tin, S, kC>(ai, group_blk(ai.gg, blockIdx.x - start[i]));
}

// ------------------------------------------------ sum of the pair groups (a5)
// The groups' partial numerators and denominators summed in a fixed order,
// then eqs. (f1), (f2) divided out: one thread per pixel.
template <typename Tin>
__device__ __forceinline__ void finish_impl(const Tin *__restrict__ f, float *__restrict__ out, const Geom &g,
                                            const DevState &st, const float2 *__restrict__ PQ, int groups,
                                            float rscale, const Blk b) {
  const int64_t npx = (int64_t)g.H * g.W;
  const int64_t pix = (int64_t)b.x * 256 + threadIdx.x;
  unsigned long long nbad = 0;
  if (pix < npx) {
    float Pv = 0.f, Qv = 0.f;
    for (int gi = 0; gi < groups; gi++) {
      const float2 pq = PQ[gi * npx + pix];
      Pv += pq.x;
      Qv += pq.y;
    }
    const int y = (int)(pix / g.W), x = (int)(pix % g.W);
    const float r = Pv / Qv;
    float v;
    if (Qv > 0.f && isfinite(r)) {
      v = fmaf(rscale, r, g.center);
    } else {
      v = fval(f[(int64_t)y * g.pitch + x]);
      nbad = 1;
    }
    out[(int64_t)y * g.opitch + x] = v;
  }
  for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off, 64);
  if ((threadIdx.x & 63) == 0 && nbad) atomicAdd(st.q_nonpos, nbad);
}
template <typename Tin>
__device__ __forceinline__ void finish_body(const FinishArgs &a, const Blk b) {
  finish_impl<Tin>((const Tin *)a.f, a.out, a.g, a.st, a.PQ, a.groups, a.rscale, b);
}
template <typename Tin>
__global__ __launch_bounds__(256) void k_finish(FinishArgs a) {
  finish_body<Tin>(a, Blk{(int)blockIdx.x, 0, 0});
}
template <typename Tin>
__global__ __launch_bounds__(256) void k_finish_grp(const FinishArgs *__restrict__ a, const int *__restrict__ start,
                                                    int n) {
  const int i = group_find(start, n, blockIdx.x);
  finish_body<Tin>(a[i], group_blk(a[i].gg, blockIdx.x - start[i]));
}

// ------------------------------------------------------------- launchers
// Full-range test input of the autotuner: 0 and `top` alternating like a
// checkerboard, so that every window spans the whole range.
template <typename Tin>
__global__ __launch_bounds__(256) void k_fill_checker(Tin *__restrict__ f, int H, int W, float top) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)H * W) return;
  const int y = (int)(i / W), x = (int)(i % W);
  f[i] = ((x ^ y) & 1) ? (Tin)top : (Tin)0;
}
hipError_t launch_fill_checker(hipStream_t s, bf_dtype dt, void *f, int H, int W, double top) {
  const unsigned nb = (unsigned)(((int64_t)H * W + 255) / 256);
  switch (dt) {
    case BF_U8: hipLaunchKernelGGL(k_fill_checker<uint8_t>, dim3(nb), dim3(256), 0, s, (uint8_t *)f, H, W, (float)top); break;
    case BF_U16: hipLaunchKernelGGL(k_fill_checker<uint16_t>, dim3(nb), dim3(256), 0, s, (uint16_t *)f, H, W, (float)top); break;
    default: hipLaunchKernelGGL(k_fill_checker<float>, dim3(nb), dim3(256), 0, s, (float *)f, H, W, (float)top); break;
  }
  return hipGetLastError();
}

// Non-local means: each pixel's patch samples f(x + u_k), k < p, clamped
// into the image, packed into one word (byte k), one thread per pixel.
__global__ __launch_bounds__(256) void k_patch_pack(PatchArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)a.H * a.W) return;
  const int y = (int)(i / a.W), x = (int)(i % a.W);
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    if (k < a.p) {
      const int yy = min(max(y + a.dy[k], 0), a.H - 1), xx = min(max(x + a.dx[k], 0), a.W - 1);
      v |= (uint32_t)a.f[(int64_t)yy * a.pitch + xx] << (8 * k);
    }
  }
  a.out[i] = Patch8x4{v};
}
hipError_t launch_patch_pack(hipStream_t s, const PatchArgs &a) {
  const int64_t n = (int64_t)a.H * a.W;
  if (n <= 0 || a.p < 1 || a.p > 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_patch_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Zero fill of n 32-bit words (a kernel, so that it can sit in a captured
// graph where a memset node could not).
__global__ __launch_bounds__(256) void k_zero_words(uint32_t *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}
hipError_t launch_zero(hipStream_t s, void *p, size_t bytes) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t *)p, n);
  return hipGetLastError();
}

hipError_t launch_reset(hipStream_t s, DevState st, int32_t T_used, double T_raw) {
  ResetArgs a{GroupGrid{1, 1, 1}, st, T_used, T_raw};
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// Grids of the range stage for one image (also the per-image grids of a
// grouped launch).
GroupGrid range_row_grid(const Geom &g) { return GroupGrid{(g.W + kRowSeg - 1) / kRowSeg, g.H, 1}; }
GroupGrid range_col_grid(const Geom &g) { return GroupGrid{(g.W + 63) / 64, (g.H + kColBandSeq - 1) / kColBandSeq, 1}; }

// The one-launch range kernel covers R <= 48 (for float input with R > 32
// its row pass reads global memory); larger R use the two passes.
bool range_tile_ok(int R, bf_dtype dt) {
  (void)dt;
  return R >= 1 && R <= 48;
}
int range_tile_kr(int R) { return R <= 32 ? 32 : 48; }
GroupGrid range_tile_grid(const Geom &g) { return GroupGrid{(g.W + kTileW - 1) / kTileW, (g.H + kTileH - 1) / kTileH, 1}; }
template <typename Tin>
static size_t tile_lds_t(int R, int kr) {
  return kr == 32 ? tile_lds_bytes<Tin, 32>(R) : tile_lds_bytes<Tin, 48>(R);
}
size_t range_tile_lds(int R, bf_dtype dt, int kr) {
  if (kr == 0) kr = range_tile_kr(R);
  switch (dt) {
    case BF_U8: return tile_lds_t<uint8_t>(R, kr);
    case BF_U16: return tile_lds_t<uint16_t>(R, kr);
    default: return tile_lds_t<float>(R, kr);
  }
}

template <typename Tin>
static hipError_t range_t(hipStream_t s, const Tin *f, const Geom &g, int R, Tin *rowmax, DevState st,
                          RangeAcc acc, int32_t T_cap, const StageRec &rec) {
  if (range_tile_ok(R, dtype_of<Tin>())) {
    rec.begin(BF_STAGE_RANGE, s);
    const GroupGrid gt = range_tile_grid(g);
    const int tiles = gt.gx * gt.gy;
    const bool stats = tiles >= kRangeStatsMinTiles;
    RangeTileArgs ta{gt, f, g.pitch, g.H, g.W, R, st, acc, T_cap, stats ? (int2 *)rowmax : nullptr,
                     range_tile_wgs(tiles, tiles)};
    const GroupGrid gs = range_stats_grid(gt);
    if (stats) hipLaunchKernelGGL(k_range_stats<Tin>, dim3(gs.gx, gs.gy), dim3(kStatThreads), 0, s, ta);
    const size_t lds = range_tile_lds(R, dtype_of<Tin>());
    if (range_tile_kr(R) == 32)
      hipLaunchKernelGGL((k_range_tile<Tin, 32>), dim3(ta.nwg), dim3(kTileThreads), lds, s, ta);
    else
      hipLaunchKernelGGL((k_range_tile<Tin, 48>), dim3(ta.nwg), dim3(kTileThreads), lds, s, ta);
    rec.end(BF_STAGE_RANGE, s);
    return hipGetLastError();
  }
  hipError_t e = launch_reset(s, st, 0, 0.0);
  if (e != hipSuccess) return e;
  rec.begin(BF_STAGE_RANGE, s);
  const GroupGrid gr = range_row_grid(g), gc = range_col_grid(g);
  RowmaxArgs ra{gr, f, g.pitch, g.H, g.W, R, rowmax, st};
  hipLaunchKernelGGL(k_rowmax<Tin>, dim3(gr.gx, gr.gy), dim3(64), 0, s, ra);
  ColmaxArgs ca{gc, f, g.pitch, (const Tin *)rowmax, g.H, g.W, R, st, T_cap};
  hipLaunchKernelGGL(k_colmax_T_seq<Tin>, dim3(gc.gx, gc.gy), dim3(64), 0, s, ca);
  rec.end(BF_STAGE_RANGE, s);
  return hipGetLastError();
}

// Grouped range stage: the row pass of every image, then the column pass of
// every image.
template <typename Tin>
static hipError_t range_group_t(hipStream_t s, const RowmaxArgs *ra, const int *rstart, int rtotal,
                                const ColmaxArgs *ca, const int *cstart, int ctotal, int n) {
  if (rtotal > 0) hipLaunchKernelGGL(k_rowmax_grp<Tin>, dim3(rtotal), dim3(64), 0, s, ra, rstart, n);
  if (ctotal > 0) hipLaunchKernelGGL(k_colmax_T_seq_grp<Tin>, dim3(ctotal), dim3(64), 0, s, ca, cstart, n);
  return hipGetLastError();
}
hipError_t launch_range_group(hipStream_t s, bf_dtype dt, const RowmaxArgs *ra, const int *rstart, int rtotal,
                              const ColmaxArgs *ca, const int *cstart, int ctotal, int n) {
  switch (dt) {
    case BF_U8: return range_group_t<uint8_t>(s, ra, rstart, rtotal, ca, cstart, ctotal, n);
    case BF_U16: return range_group_t<uint16_t>(s, ra, rstart, rtotal, ca, cstart, ctotal, n);
    default: return range_group_t<float>(s, ra, rstart, rtotal, ca, cstart, ctotal, n);
  }
}
template <typename Tin>
static hipError_t range_tile_group_t(hipStream_t s, int kr, const RangeTileArgs *a, const int *start, int total,
                                     int n, size_t lds) {
  if (total > 0) {
    if (kr == 32)
      hipLaunchKernelGGL((k_range_tile_grp<Tin, 32>), dim3(total), dim3(kTileThreads), lds, s, a, start, n);
    else
      hipLaunchKernelGGL((k_range_tile_grp<Tin, 48>), dim3(total), dim3(kTileThreads), lds, s, a, start, n);
  }
  return hipGetLastError();
}
template <typename Tin>
static hipError_t range_stats_group_t(hipStream_t s, const RangeTileArgs *a, const int *start, int total, int n) {
  if (total > 0) hipLaunchKernelGGL(k_range_stats_grp<Tin>, dim3(total), dim3(kStatThreads), 0, s, a, start, n);
  return hipGetLastError();
}
hipError_t launch_range_stats_group(hipStream_t s, bf_dtype dt, const RangeTileArgs *a, const int *start, int total,
                                    int n) {
  switch (dt) {
    case BF_U8: return range_stats_group_t<uint8_t>(s, a, start, total, n);
    case BF_U16: return range_stats_group_t<uint16_t>(s, a, start, total, n);
    default: return range_stats_group_t<float>(s, a, start, total, n);
  }
}
hipError_t launch_range_tile_group(hipStream_t s, bf_dtype dt, int kr, const RangeTileArgs *a, const int *start,
                                   int total, int n, size_t lds) {
  switch (dt) {
    case BF_U8: return range_tile_group_t<uint8_t>(s, kr, a, start, total, n, lds);
    case BF_U16: return range_tile_group_t<uint16_t>(s, kr, a, start, total, n, lds);
    default: return range_tile_group_t<float>(s, kr, a, start, total, n, lds);
  }
}
hipError_t launch_reset_group(hipStream_t s, const ResetArgs *a, const int *start, int total, int n) {
  if (total > 0) hipLaunchKernelGGL(k_reset_grp, dim3(total), dim3(64), 0, s, a, start, n);
  return hipGetLastError();
}

hipError_t launch_range(hipStream_t s, bf_dtype dt, const void *f, const Geom &g, int R, void *rowmax,
                        DevState st, RangeAcc acc, int32_t T_cap, const StageRec &rec) {
  if (R > kMaxR) return hipErrorInvalidValue;
  switch (dt) {
    case BF_U8: return range_t<uint8_t>(s, (const uint8_t *)f, g, R, (uint8_t *)rowmax, st, acc, T_cap, rec);
    case BF_U16:
      return range_t<uint16_t>(s, (const uint16_t *)f, g, R, (uint16_t *)rowmax, st, acc, T_cap, rec);
    default: return range_t<float>(s, (const float *)f, g, R, (float *)rowmax, st, acc, T_cap, rec);
  }
}

// Per-image arguments of the two recursive-path kernels for pairs
// [k0, k0+kcount) (also the per-image entries of grouped launches) and of the
// sum of the pair groups.
void iir_args(const void *f, float *out, const Geom &g, DevTables tab, DevState st, const float *iir, int k0,
              int kcount, float4 *Z, float2 *PQ, bool first, bool last, float2 *glut, IirArgs a[2],
              FinishArgs &fa) {
  const IirArgs base{GroupGrid{1, 1, 1}, f, out, g, tab, st, iir, k0, kcount, Z, PQ, (int)first, (int)last, glut};
  a[0] = base;
  a[1] = base;
  const int ng = kHThreads / g.vS;  // columns per vertical workgroup
  const int per = ((g.Spos + ng - 1) / ng + 7) / 8;
  a[0].gg = GroupGrid{8 * per, (kcount + g.vppw - 1) / g.vppw, 1};  // vertical (column blocks in XCD order)
  const int nrb = (g.H + g.hrows - 1) / g.hrows;
  a[1].gg = GroupGrid{8 * ((nrb + 7) / 8), g.hgroups, 1};  // horizontal + combine (row blocks in XCD order)
  const int64_t npx = (int64_t)g.H * g.W;
  const int nfin = (last && g.hgroups > 1) ? (int)((npx + 255) / 256) : 0;
  fa = FinishArgs{GroupGrid{nfin > 0 ? nfin : 1, 1, 1}, f, out, g, st, (const float2 *)PQ, g.hgroups, 1.0f};
}

hipError_t launch_finish(hipStream_t s, bf_dtype dt, const FinishArgs *one, const FinishArgs *arr,
                         const int *start, int n, int total) {
  switch (dt) {
    case BF_U8:
      if (one) hipLaunchKernelGGL(k_finish<uint8_t>, dim3(one->gg.gx), dim3(256), 0, s, *one);
      else if (total > 0) hipLaunchKernelGGL(k_finish_grp<uint8_t>, dim3(total), dim3(256), 0, s, arr, start, n);
      break;
    case BF_U16:
      if (one) hipLaunchKernelGGL(k_finish<uint16_t>, dim3(one->gg.gx), dim3(256), 0, s, *one);
      else if (total > 0) hipLaunchKernelGGL(k_finish_grp<uint16_t>, dim3(total), dim3(256), 0, s, arr, start, n);
      break;
    case kDtPatch:  // non-local means: single images only
      if (one) hipLaunchKernelGGL(k_finish<Patch8x4>, dim3(one->gg.gx), dim3(256), 0, s, *one);
      else if (total > 0) return hipErrorInvalidValue;
      break;
    default:
      if (one) hipLaunchKernelGGL(k_finish<float>, dim3(one->gg.gx), dim3(256), 0, s, *one);
      else if (total > 0) hipLaunchKernelGGL(k_finish_grp<float>, dim3(total), dim3(256), 0, s, arr, start, n);
      break;
  }
  return hipGetLastError();
}

// Launches of the two kernels for a row group size and chunk, single image
// (one) or grouped (arr, start, n, total).
template <typename Tin, int S, int C>
static void launch_v(hipStream_t s, const IirArgs *one, const IirArgs *arr, const int *start, int n, int total) {
  if (one)
    hipLaunchKernelGGL((k_iir_v<Tin, S, C>), dim3(one->gg.gx, one->gg.gy), dim3(kHThreads), 0, s, *one);
  else if (total > 0)
    hipLaunchKernelGGL((k_iir_v_grp<Tin, S, C>), dim3(total), dim3(kHThreads), 0, s, arr, start, n);
}
template <typename Tin, int S, int C>
static void launch_h(hipStream_t s, const IirArgs *one, const IirArgs *arr, const int *start, int n, int total) {
  if (one)
    hipLaunchKernelGGL((k_iir_h_accum<Tin, S, C>), dim3(one->gg.gx, one->gg.gy), dim3(kHThreads), 0, s, *one);
  else if (total > 0)
    hipLaunchKernelGGL((k_iir_h_accum_grp<Tin, S, C>), dim3(total), dim3(kHThreads), 0, s, arr, start, n);
}
template <typename Tin, int C>
static bool launch_h_S(hipStream_t s, int S, const IirArgs *one, const IirArgs *arr, const int *start, int n,
                       int total) {
  switch (S) {
    case 1: launch_h<Tin, 1, C>(s, one, arr, start, n, total); return true;
    case 2: launch_h<Tin, 2, C>(s, one, arr, start, n, total); return true;
    case 4: launch_h<Tin, 4, C>(s, one, arr, start, n, total); return true;
    case 8: launch_h<Tin, 8, C>(s, one, arr, start, n, total); return true;
    case 16: launch_h<Tin, 16, C>(s, one, arr, start, n, total); return true;
    case 32: launch_h<Tin, 32, C>(s, one, arr, start, n, total); return true;
    case 64: launch_h<Tin, 64, C>(s, one, arr, start, n, total); return true;
    case 128: launch_h<Tin, 128, C>(s, one, arr, start, n, total); return true;
    case 256: launch_h<Tin, 256, C>(s, one, arr, start, n, total); return true;
    default: return false;
  }
}
template <typename Tin>
static bool launch_h_any(hipStream_t s, int S, int cC, const IirArgs *one, const IirArgs *arr, const int *start,
                         int n, int total) {
  return cC == kCSmall ? launch_h_S<Tin, kCSmall>(s, S, one, arr, start, n, total)
                       : launch_h_S<Tin, kCLarge>(s, S, one, arr, start, n, total);
}
// The vertical pass runs kCLarge or kCSmall rows per thread.
template <typename Tin, int C>
static bool launch_v_S(hipStream_t s, int S, const IirArgs *one, const IirArgs *arr, const int *start, int n,
                       int total) {
  switch (S) {
    case 1: launch_v<Tin, 1, C>(s, one, arr, start, n, total); return true;
    case 2: launch_v<Tin, 2, C>(s, one, arr, start, n, total); return true;
    case 4: launch_v<Tin, 4, C>(s, one, arr, start, n, total); return true;
    case 8: launch_v<Tin, 8, C>(s, one, arr, start, n, total); return true;
    case 16: launch_v<Tin, 16, C>(s, one, arr, start, n, total); return true;
    case 32: launch_v<Tin, 32, C>(s, one, arr, start, n, total); return true;
    case 64: launch_v<Tin, 64, C>(s, one, arr, start, n, total); return true;
    case 128: launch_v<Tin, 128, C>(s, one, arr, start, n, total); return true;
    case 256: launch_v<Tin, 256, C>(s, one, arr, start, n, total); return true;
    default: return false;
  }
}
template <typename Tin>
static bool launch_v_any(hipStream_t s, int S, int cV, const IirArgs *one, const IirArgs *arr, const int *start,
                         int n, int total) {
  if (cV == kCLarge) return launch_v_S<Tin, kCLarge>(s, S, one, arr, start, n, total);
  if (cV == kCSmall) return launch_v_S<Tin, kCSmall>(s, S, one, arr, start, n, total);
  return false;
}

static bool iir_geom_ok(const Geom &g, int kcount) {
  return g.hgroups >= 1 && g.hgroups <= 65535 && g.vppw >= 1 && g.hkpg >= 1 && (int64_t)g.hgroups * g.hkpg >= kcount &&
         g.hrows >= 1 && (kHThreads / g.S) % g.hrows == 0 && g.hkpg % (kHThreads / g.S / g.hrows) == 0 &&
         kcount >= 1 && kcount <= 65535 && g.vS >= 1 && g.vS <= kHThreads && (int64_t)g.vS * g.vC >= g.H &&
         g.Seff >= 1 && g.Seff <= g.S && (int64_t)g.Seff * g.cC >= g.W && g.Spos == g.Seff * g.cC && g.zlog >= 0 && g.zlog <= 3 && g.Hz >= g.H && g.Hz % (1 << g.zlog) == 0 &&
         ((kHThreads / g.vS) << g.zlog) >= z_tile_words(g.vS) && (g.zlog == 0 || ((kHThreads / g.vS) << g.zlog) == z_tile_words(g.vS));
}

template <typename Tin>
static hipError_t iir_chunk_t(hipStream_t s, const Tin *f, float *out, const Geom &g, DevTables tab,
                              DevState st, const float *iir, int k0, int kcount, float4 *Z, float2 *PQ,
                              bool first, bool last, float2 *glut, const StageRec &rec) {
  if (!iir_geom_ok(g, kcount)) return hipErrorInvalidValue;
  IirArgs a[2];
  FinishArgs fa;
  iir_args(f, out, g, tab, st, iir, k0, kcount, Z, PQ, first, last, glut, a, fa);
  rec.begin(BF_STAGE_V_IIR, s);
  if (!launch_v_any<Tin>(s, g.vS, g.vC, &a[0], nullptr, nullptr, 0, 0)) return hipErrorInvalidValue;
  rec.end(BF_STAGE_V_IIR, s);
  rec.begin(BF_STAGE_H_COMBINE, s);
  if (!launch_h_any<Tin>(s, g.S, g.cC, &a[1], nullptr, nullptr, 0, 0)) return hipErrorInvalidValue;
  if (last && g.hgroups > 1) (void)launch_finish(s, dtype_of<Tin>(), &fa, nullptr, nullptr, 0, 0);
  rec.end(BF_STAGE_H_COMBINE, s);
  return hipGetLastError();
}

hipError_t launch_iir_v_group(hipStream_t s, bf_dtype dt, int SV, int cV, const IirArgs *a, const int *start,
                              int n, int total, const StageRec &rec) {
  rec.begin(BF_STAGE_V_IIR, s);
  bool ok;
  switch (dt) {
    case BF_U8: ok = launch_v_any<uint8_t>(s, SV, cV, nullptr, a, start, n, total); break;
    case BF_U16: ok = launch_v_any<uint16_t>(s, SV, cV, nullptr, a, start, n, total); break;
    default: ok = launch_v_any<float>(s, SV, cV, nullptr, a, start, n, total); break;
  }
  rec.end(BF_STAGE_V_IIR, s);
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}
hipError_t launch_iir_h_group(hipStream_t s, bf_dtype dt, int S, int cC, const IirArgs *a, const int *start,
                              int n, int total, const FinishArgs *fa, const int *fstart, int ftotal,
                              const StageRec &rec) {
  rec.begin(BF_STAGE_H_COMBINE, s);
  bool ok;
  switch (dt) {
    case BF_U8: ok = launch_h_any<uint8_t>(s, S, cC, nullptr, a, start, n, total); break;
    case BF_U16: ok = launch_h_any<uint16_t>(s, S, cC, nullptr, a, start, n, total); break;
    default: ok = launch_h_any<float>(s, S, cC, nullptr, a, start, n, total); break;
  }
  if (ok && ftotal > 0) (void)launch_finish(s, dt, nullptr, fa, fstart, n, ftotal);
  rec.end(BF_STAGE_H_COMBINE, s);
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_iir_chunk(hipStream_t s, bf_dtype dt, const void *f, float *out, const Geom &g,
                            DevTables tab, DevState st, const float *iir, int k0, int kcount, float4 *Z,
                            float2 *PQ, bool first, bool last, float2 *glut, const StageRec &rec) {
  switch (dt) {
    case BF_U8:
      return iir_chunk_t<uint8_t>(s, (const uint8_t *)f, out, g, tab, st, iir, k0, kcount, Z, PQ, first, last,
                                  glut, rec);
    case BF_U16:
      return iir_chunk_t<uint16_t>(s, (const uint16_t *)f, out, g, tab, st, iir, k0, kcount, Z, PQ, first, last,
                                   glut, rec);
    default:
      return iir_chunk_t<float>(s, (const float *)f, out, g, tab, st, iir, k0, kcount, Z, PQ, first, last, glut,
                                rec);
  }
}

}  // namespace bfi
