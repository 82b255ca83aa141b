// gfx950 MFMA path of libbf.so: the spatial smoothing of SHIFTABLE-BF
// (Sec. 1.2 step 3, eq. (GF)) as the separable FIR with taps
// w[d] = exp(-(d-R)^2 / 2 sigma_s^2), d = 0..2R, zero extension, written as
// banded Toeplitz matrices times image tiles on FP16/BF16 matrix cores with
// FP32 accumulation.
//
// v_mfma_f32_16x16x32_{f16,bf16}: lane l holds A[l%16][8(l/16)+j] and
// B[8(l/16)+j][l%16] (j = 0..7), and receives D[4(l/16)+i][l%16] (i = 0..3).
//
// Vertical pass: 16 output rows x 16 pixel columns of one image plane are
//   D = T (16 x K) . In (K x 16),   T[i][t] = w[t - i] (zero off the band),
// K = 32 nks >= 16 + 2R input rows.  Horizontal pass: 16 rows x 16 output
// columns are D = In (16 x K) . T^T (K x 16).  The A fragment of T and the B
// fragment of T^T are the same registers.
//
// Operands: the difference images (f - c) cos, (f - c) sin are divided by the
// half range c so that every plane lies in [-1, 1]; with peak-one taps the
// smoothed planes stay below (2R+1)^2 in magnitude, far inside FP16's range.
// Both scale factors cancel in P/Q except the first, which the combine undoes.
// Single variants store the vertical result (Z) in FP16/BF16; the split
// variants store Z in FP32 and feed hi + lo halves to three MFMAs per product
// (hi.hi + hi.lo + lo.hi).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "bf_device.h"
#include "bf_phase.h"

namespace bfi {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <bool BF>
struct MT;
template <>
struct MT<false> {
  typedef _Float16 T;
  typedef h8 V;
  static __device__ __forceinline__ f4v mfma(V a, V b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MT<true> {
  typedef __bf16 T;
  typedef b8 V;
  static __device__ __forceinline__ f4v mfma(V a, V b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// Tile shapes (the host sizes the vertical tile height to the LDS budget).
template <bool SPLIT>
struct TShape {
  static constexpr int kVCols = SPLIT ? 16 : 32;   // pixel columns per vertical tile
  static constexpr int kHCols = SPLIT ? 64 : 128;  // output columns per horizontal tile
};
constexpr int kHRows = 16;

// Workgroups are dispatched to the eight XCDs in turn; map launch index id
// to tile (id mod 8) * per + id / 8 so that each XCD works through a
// contiguous run of neighbouring tiles, whose shared halos and cache lines
// then meet in that XCD's L2.  per = ceil(tiles / 8).
__device__ __forceinline__ int xcd_tile(int id, int per) { return (id & 7) * per + (id >> 3); }

// Tap fragments: lane l of K-step ks holds T[l%16][32 ks + 8 (l/16) + j],
// j = 0..7, with T[i][t] = w[t - i] on the band and 0 off it (hi and, for the
// split variants, lo halves).  The workgroup builds all nks x 64 fragments
// once into LDS (branch-free clamped reads of the taps); every K-step of
// every product then reads its fragment with one 16-byte LDS load.
template <bool BF, bool SPLIT>
__device__ __forceinline__ void build_tap_frags(typename MT<BF>::V *th, typename MT<BF>::V *tl,
                                                const float *__restrict__ w, int R, int nks, int tid) {
  typedef typename MT<BF>::T E;
  typedef typename MT<BF>::V V;
  for (int idx = tid; idx < nks * 64; idx += 256) {
    const int ks = idx >> 6, ln = idx & 63, i = ln & 15;
    float vals[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int d = 32 * ks + 8 * (ln >> 4) + j - i;
      const float t = w[min(max(d, 0), 2 * R)];
      vals[j] = (d >= 0 && d <= 2 * R) ? t : 0.f;
    }
    V h, l;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      h[j] = (E)vals[j];
      l[j] = (E)(vals[j] - (float)h[j]);
    }
    th[idx] = h;
    if (SPLIT) tl[idx] = l;
  }
}
// LDS bytes of the tap fragments.
constexpr size_t tap_frag_bytes(int nks, bool split) { return (size_t)(split ? 2 : 1) * nks * 64 * 16; }

// Eight FP32 values as 16-bit operands: hi alone (single variants, rounded to
// nearest), or hi + lo (split variants), where hi keeps the leading bits that
// the 16-bit format holds (a mask of the FP32 word, so hi converts exactly
// and lo = v - hi is exact in FP32) and lo is v - hi rounded.
template <bool BF, bool SPLIT>
__device__ __forceinline__ void to_operands(const float v[8], typename MT<BF>::V &h, typename MT<BF>::V &l) {
  typedef typename MT<BF>::T E;
  constexpr uint32_t kKeep = BF ? 0xFFFF0000u : 0xFFFFE000u;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    if constexpr (SPLIT) {
      const float hf = __uint_as_float(__float_as_uint(v[j]) & kKeep);
      h[j] = (E)hf;
      l[j] = (E)(v[j] - hf);
    } else {
      h[j] = (E)v[j];
    }
  }
}

// ------------------------------------------------------------ vertical pass
// Workgroup: `rows` output rows x kVCols pixel columns of one frequency pair.
// The four images of the pair on the input rows [y0 - R, y0 + rows + R) are
// generated from f into LDS as [plane][column][row] (row index contiguous, so
// a lane's eight K elements are one 16-byte read; the padded row length
// Kp = 8 mod 16 keeps both the staging writes and the fragment reads free of
// bank conflicts), then the waves share the (16-row block, 16-column block)
// products of all four planes.
template <typename Tin, bool BF, bool SPLIT>
__device__ __forceinline__ void toep_v_body(const ToepVArgs &a, const Blk b) {
  const Tin *__restrict__ f = (const Tin *)a.f;
  const Geom g = a.g;
  const DevTables tab = a.tab;
  const DevState st = a.st;
  const float *__restrict__ taps = a.tc.taps;
  const int R = a.tc.R, nks = a.tc.nks, rows = a.tc.rows;
  const int ntx = a.ntx, ntiles = a.ntiles, per = a.per, k0 = a.k0;
  void *__restrict__ Zv = a.Z;
  const size_t zplane = a.zplane;

  typedef typename MT<BF>::T E;
  typedef typename MT<BF>::V V;
  typedef typename std::conditional<SPLIT, float, E>::type ZT;
  constexpr int kCols = TShape<SPLIT>::kVCols;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float2 lut[PhaseLut<Tin>::kOn ? 256 : 1];
  const int t = xcd_tile(b.x, per);
  if (t >= ntiles) return;
  const int kl = b.y;
  const OrderEntry &e = lookup(tab, st.T_used);
  const int k = k0 + kl;
  if (k >= e.K) return;
  const int32_t m = tab.pm[e.off + k];
  const uint64_t q = e.qfix;
  const double at = e.alpha_turn;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int x0 = (t % ntx) * kCols;
  const int y0 = (t / ntx) * rows;
  const int Kl = rows - 16 + 32 * nks;  // rows read by the last 16-row block
  const int Kp = Kl + 8;
  V *tfh = (V *)smem;
  V *tfl = tfh + nks * 64;
  E *Bh = (E *)(smem + tap_frag_bytes(nks, SPLIT));
  E *Bl = Bh + 4 * kCols * Kp;
  const float inv = 1.f / g.center;
  build_tap_frags<BF, SPLIT>(tfh, tfl, taps, R, nks, tid);  // read after the staging barrier
  if constexpr (PhaseLut<Tin>::kOn) {
    if (tab.lut_gen) lut[tid] = tab.lut_gen[(size_t)(e.off + k) * 256 + tid];  // polynomial kernel
    else build_lut(lut, m, q, at, tid, 256);
    __syncthreads();
  }
  // staging: one work item = 8 consecutive rows of one column.  The eight
  // loads use clamped addresses and no branches, so they are all in flight
  // together; rows and columns outside the image are zeroed afterwards.
  const Freq fq = make_freq(m, q, at);
  const int nstrip = Kl / 8;
  for (int it = tid; it < nstrip * kCols; it += 256) {
    const int c = it % kCols, sidx = it / kCols;
    const int x = x0 + c;
    const int ybase = y0 - R + 8 * sidx;
    const bool inner = x < g.W && ybase >= 0 && ybase + 8 <= g.H;  // all eight pixels in the image
    Tin raw[8];
    if (inner) {
      const Tin *src = f + (int64_t)ybase * g.pitch + x;
#pragma unroll
      for (int j = 0; j < 8; j++) raw[j] = src[(int64_t)j * g.pitch];
    } else {
      const int xc = min(x, g.W - 1);
#pragma unroll
      for (int j = 0; j < 8; j++) raw[j] = f[(int64_t)min(max(ybase + j, 0), g.H - 1) * g.pitch + xc];
    }
    float pv[4][8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const float4 p = planes_any<Tin>(raw[j], lut, fq, g.center);
      pv[0][j] = p.x * inv;
      pv[1][j] = p.y * inv;
      pv[2][j] = p.z;
      pv[3][j] = p.w;
    }
    if (!inner) {  // pixels off the image contribute zeros
#pragma unroll
      for (int j = 0; j < 8; j++)
        if (!(x < g.W && ybase + j >= 0 && ybase + j < g.H)) pv[0][j] = pv[1][j] = pv[2][j] = pv[3][j] = 0.f;
    }
#pragma unroll
    for (int p = 0; p < 4; p++) {
      V h, l;
      to_operands<BF, SPLIT>(pv[p], h, l);
      *(V *)(Bh + (p * kCols + c) * Kp + 8 * sidx) = h;
      if (SPLIT) *(V *)(Bl + (p * kCols + c) * Kp + 8 * sidx) = l;
    }
  }
  __syncthreads();
  ZT *Z = (ZT *)Zv + (size_t)kl * 4 * zplane;
  const int nmb = rows / 16;
  const int ncomb = nmb * (kCols / 16);
  // D'[x][y] = In^T (16 columns x K) . T^T (K x 16 rows): the LDS column
  // fragment is the A operand and the tap fragment the B operand, so lane l
  // receives the 4 consecutive columns x0 + 16 nb + 4 (l/16) + i of row
  // y0 + 16 mb + l%16 and writes them with one packed store.
  typedef ZT Z4 __attribute__((ext_vector_type(4)));
  typedef ZT Z2 __attribute__((ext_vector_type(2)));
  const size_t pstride = (size_t)kCols * Kp;  // LDS elements between planes
  for (int cb = wv; cb < ncomb; cb += 4) {
    const int mb = cb % nmb, nb = cb / nmb;
    const int px = nb * 16 + (lane & 15);
    const int y = y0 + 16 * mb + (lane & 15);
    const int xs = x0 + nb * 16 + 4 * (lane >> 4);
    const E *colh = Bh + px * Kp + 16 * mb + 8 * (lane >> 4);
    const E *coll = Bl + px * Kp + 16 * mb + 8 * (lane >> 4);
    f4v acc[4];
#pragma unroll
    for (int p = 0; p < 4; p++) acc[p] = (f4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < nks; ks++) {
      const V tb = tfh[ks * 64 + lane];
#pragma unroll
      for (int p = 0; p < 4; p++) {
        const V bh = *(const V *)(colh + p * pstride + 32 * ks);
        acc[p] = MT<BF>::mfma(bh, tb, acc[p]);
        if (SPLIT) {
          const V tbl = tfl[ks * 64 + lane];
          const V bl = *(const V *)(coll + p * pstride + 32 * ks);
          acc[p] = MT<BF>::mfma(bl, tb, acc[p]);
          acc[p] = MT<BF>::mfma(bh, tbl, acc[p]);
        }
      }
    }
#pragma unroll
    for (int p = 0; p < 4; p++) {
      if (y < g.H && xs < g.W) {
        ZT *zp = Z + (size_t)p * zplane + (size_t)y * g.zpitch + g.padl + xs;
        const f4v v = acc[p];
        if (xs + 4 <= g.W && (g.padl & 3) == 0) {
          *(Z4 *)zp = (Z4){(ZT)v[0], (ZT)v[1], (ZT)v[2], (ZT)v[3]};
        } else if (xs + 4 <= g.W && (g.padl & 1) == 0) {
          *(Z2 *)zp = (Z2){(ZT)v[0], (ZT)v[1]};
          *(Z2 *)(zp + 2) = (Z2){(ZT)v[2], (ZT)v[3]};
        } else {
#pragma unroll
          for (int i = 0; i < 4; i++)
            if (xs + i < g.W) zp[i] = (ZT)v[i];
        }
      }
    }
  }
}
template <typename Tin, bool BF, bool SPLIT>
__global__ __launch_bounds__(256) void k_toep_v(ToepVArgs a) {
  toep_v_body<Tin, BF, SPLIT>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin, bool BF, bool SPLIT>
__global__ __launch_bounds__(256) void k_toep_v_grp(const ToepVArgs *__restrict__ a, const int *__restrict__ start,
                                                    int n) {
  const int i = group_find(start, n, blockIdx.x);
  toep_v_body<Tin, BF, SPLIT>(a[i], group_blk(a[i].gg, blockIdx.x - start[i]));
}

// -------------------------------------------------- horizontal pass + combine
// Workgroup: 16 rows x kHCols output columns and one group of consecutive
// pairs (blockIdx.y).  For each pair the four vertical results on the columns
// [x0 - R, x0 + kHCols + R) are staged in LDS as [plane][row][column] with
// 16-byte loads (Z rows carry a left pad congruent to R mod 8, so the staged
// window starts on an 8-element boundary); each wave multiplies its 16-column
// blocks for every plane and folds the four results of each pixel with its
// phases into the numerator and denominator of eqs. (f1), (f2).  With one
// group and the last launch the workgroup divides and writes the output;
// otherwise it leaves its partial sums in PQ[group] (added to what the
// previous launch left there unless `first`).
template <typename Tin, bool BF, bool SPLIT>
__device__ __forceinline__ void toep_h_body(const ToepHArgs &a, const Blk b) {
  const Tin *__restrict__ f = (const Tin *)a.f;
  float *__restrict__ out = a.out;
  const Geom g = a.g;
  const DevTables tab = a.tab;
  const DevState st = a.st;
  const float *__restrict__ taps = a.tc.taps;
  const int R = a.tc.R, nks = a.tc.nks, kpg = a.tc.kpg;
  const int ntx = a.ntx, ntiles = a.ntiles, per = a.per, k0 = a.k0, kcount = a.kcount;
  const void *__restrict__ Zv = a.Z;
  const size_t zplane = a.zplane;
  float2 *__restrict__ PQ = a.PQ;
  const int first = a.first, finish = a.finish;

  typedef typename MT<BF>::T E;
  typedef typename MT<BF>::V V;
  typedef typename std::conditional<SPLIT, float, E>::type ZT;
  constexpr int kCols = TShape<SPLIT>::kHCols;
  constexpr int kNbw = kCols / 64;  // 16-column blocks per wave
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float2 lut[PhaseLut<Tin>::kOn ? 256 : 1];
  const int t = xcd_tile(b.x, per);
  if (t >= ntiles) return;
  const OrderEntry &e = lookup(tab, st.T_used);
  const int kb = k0 + b.y * kpg;
  const int kend = min(min(kb + kpg, k0 + kcount), e.K);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int x0 = (t % ntx) * kCols;
  const int y0 = (t / ntx) * kHRows;
  const int Kl = kCols - 16 + 32 * nks;  // columns read by the last 16-column block
  const int Kp = Kl + 8;
  V *tfh = (V *)smem;
  V *tfl = tfh + nks * 64;
  E *Ah = (E *)(smem + tap_frag_bytes(nks, SPLIT));
  E *Al = Ah + 4 * kHRows * Kp;
  build_tap_frags<BF, SPLIT>(tfh, tfl, taps, R, nks, tid);  // read after the first barrier below
  const int rbase = 4 * (lane >> 4);
  Tin fv[kNbw][4];
  float P[kNbw][4], Q[kNbw][4];
#pragma unroll
  for (int bb = 0; bb < kNbw; bb++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int y = min(y0 + rbase + i, g.H - 1);
      const int x = min(x0 + (kNbw * wv + bb) * 16 + (lane & 15), g.W - 1);
      fv[bb][i] = f[(int64_t)y * g.pitch + x];
      P[bb][i] = 0.f;
      Q[bb][i] = 0.f;
    }
  const ZT *Zb = (const ZT *)Zv;
  const uint64_t q = e.qfix;
  const double at = e.alpha_turn;
  // Staging of one pair's Z tile: the 64 LDS rows (plane * 16 + image row) are
  // shared out to the waves, 16 each.  A row holds nvec = Kl / 8 <= 64 vectors
  // of 8 elements (the window starts on an 8-element boundary); Lr = 16, 32 or
  // 64 lanes (the smallest >= nvec) take one row, so one wave instruction
  // covers 64 / Lr rows, and four such instructions are in flight.  Vectors
  // that reach off the image are zeroed element-wise by a bit mask.
  typedef typename std::conditional<SPLIT, float4, V>::type LT;
  constexpr int kLw = SPLIT ? 2 : 1;  // LT loads per vector
  const int nvec = Kl / 8;
  const int lrs = nvec <= 16 ? 4 : (nvec <= 32 ? 5 : 6);  // log2 of lanes per row
  const int vl = lane & ((1 << lrs) - 1);                 // this lane's vector in its row
  const int sub = lane >> lrs;                            // this lane's row within an instruction
  const int rpi = 64 >> lrs;                              // rows per instruction
  const bool lane_on = vl < nvec;
  const int zc = x0 - R + g.padl + 8 * vl;  // first Z column of this lane's vector (multiple of 8)
  const int jlo = min(max(g.padl - zc, 0), 8), jhi = min(max(g.padl + g.W - zc, 0), 8);
  const uint32_t xmask = jhi > jlo ? ((1u << jhi) - 1u) & ~((1u << jlo) - 1u) : 0u;  // valid elements
  const int ninst = 16 >> (6 - lrs);  // instructions per wave per pair (16 rows / rpi)
  for (int k = kb; k < kend; k++) {
    const int kl = k - k0;
    const int32_t m = tab.pm[e.off + k];
    const float cp = tab.pc[e.off + k];
    const Freq fq = make_freq(m, q, at);
    __syncthreads();  // the previous pair's tile and table are consumed
    if constexpr (PhaseLut<Tin>::kOn) {
      if (tab.lut_comb) lut[tid] = tab.lut_comb[(size_t)(e.off + k) * 256 + tid];  // polynomial kernel
      else build_lut(lut, m, q, at, tid, 256);
    }
    const ZT *Zk = Zb + (size_t)kl * 4 * zplane;
    constexpr int kRU = 4;  // instructions in flight per lane
    for (int j0 = 0; j0 < ninst; j0 += kRU) {
      LT raw[kRU][kLw];
      uint32_t msk[kRU];
#pragma unroll
      for (int u = 0; u < kRU; u++) {
        const int rr = wv + 4 * ((j0 + u) * rpi + sub);  // LDS row: plane rr / 16, image row y0 + rr % 16
        const int y = y0 + (rr & 15);
        msk[u] = (lane_on && j0 + u < ninst && y < g.H) ? xmask : 0u;
        const ZT *src = Zk + (msk[u] ? (size_t)(rr >> 4) * zplane + (size_t)y * g.zpitch + zc : 0);
        raw[u][0] = *(const LT *)src;
        if constexpr (SPLIT) raw[u][kLw - 1] = *(const LT *)(src + 4);
      }
#pragma unroll
      for (int u = 0; u < kRU; u++) {
        const int rr = wv + 4 * ((j0 + u) * rpi + sub);
        V h, l;
        if constexpr (SPLIT) {
          const float4 a0 = raw[u][0], a1 = raw[u][kLw - 1];
          float vals[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
          if (msk[u] != 0xFFu) {  // edge vectors only
#pragma unroll
            for (int j = 0; j < 8; j++) vals[j] = ((msk[u] >> j) & 1u) ? vals[j] : 0.f;
          }
          to_operands<BF, true>(vals, h, l);
        } else {
          h = raw[u][0];
          if (msk[u] != 0xFFu) {  // edge vectors only
            union {
              V v;
              uint32_t w[4];
            } cv;
            cv.v = h;
#pragma unroll
            for (int w = 0; w < 4; w++)
              cv.w[w] &= (((msk[u] >> (2 * w)) & 1u) ? 0x0000FFFFu : 0u) |
                         (((msk[u] >> (2 * w + 1)) & 1u) ? 0xFFFF0000u : 0u);
            h = cv.v;
          }
        }
        if (lane_on && j0 + u < ninst) {
          *(V *)(Ah + rr * Kp + 8 * vl) = h;
          if (SPLIT) *(V *)(Al + rr * Kp + 8 * vl) = l;
        }
      }
    }
    __syncthreads();
    const size_t pstride = (size_t)kHRows * Kp;  // LDS elements between planes
#pragma unroll
    for (int bb = 0; bb < kNbw; bb++) {
      const int nb = kNbw * wv + bb;
      f4v acc[4];
#pragma unroll
      for (int p = 0; p < 4; p++) acc[p] = (f4v){0.f, 0.f, 0.f, 0.f};
      const E *rowh = Ah + (lane & 15) * Kp + 16 * nb + 8 * (lane >> 4);
      const E *rowl = Al + (lane & 15) * Kp + 16 * nb + 8 * (lane >> 4);
#pragma unroll 2
      for (int ks = 0; ks < nks; ks++) {
        const V tb = tfh[ks * 64 + lane];
#pragma unroll
        for (int p = 0; p < 4; p++) {
          const V ah = *(const V *)(rowh + p * pstride + 32 * ks);
          acc[p] = MT<BF>::mfma(ah, tb, acc[p]);
          if (SPLIT) {
            const V tbl = tfl[ks * 64 + lane];
            const V al = *(const V *)(rowl + p * pstride + 32 * ks);
            acc[p] = MT<BF>::mfma(al, tb, acc[p]);
            acc[p] = MT<BF>::mfma(ah, tbl, acc[p]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; i++) {
        float c, s;
        if constexpr (PhaseLut<Tin>::kOn) {
          const float2 cs = lut[(int)fv[bb][i]];
          c = cs.x;
          s = cs.y;
        } else {
          turn_sincos(phase_turn<Tin>(fv[bb][i], fq), c, s);
        }
        P[bb][i] = fmaf(cp, fmaf(c, acc[0][i], s * acc[1][i]), P[bb][i]);
        Q[bb][i] = fmaf(cp, fmaf(c, acc[2][i], s * acc[3][i]), Q[bb][i]);
      }
      // keep the column blocks apart: interleaving them only raises register pressure
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (kb >= kend && !first && !finish) return;  // no pairs here: partial sums unchanged
  float2 *PQg = PQ + (size_t)b.y * g.H * g.W;
  unsigned long long nbad = 0;
#pragma unroll
  for (int bb = 0; bb < kNbw; bb++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int y = y0 + rbase + i, x = x0 + (kNbw * wv + bb) * 16 + (lane & 15);
      if (y >= g.H || x >= g.W) continue;
      float Pv = P[bb][i], Qv = Q[bb][i];
      const size_t pix = (size_t)y * g.W + x;
      if (!first) {
        const float2 pq = PQg[pix];
        Pv += pq.x;
        Qv += pq.y;
      }
      if (finish) {
        const float r = Pv / Qv;
        float v;
        if (Qv > 0.f && isfinite(r)) {
          v = fmaf(g.center, r, g.center);
        } else {
          v = fval(fv[bb][i]);
          nbad++;
        }
        out[(int64_t)y * g.opitch + x] = v;
      } else {
        PQg[pix] = make_float2(Pv, Qv);
      }
    }
  if (finish) {
    for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off, 64);
    if (lane == 0 && nbad) atomicAdd(st.q_nonpos, nbad);
  }
}
template <typename Tin, bool BF, bool SPLIT>
__global__ __launch_bounds__(256, SPLIT ? 3 : 2) void k_toep_h(ToepHArgs a) {
  toep_h_body<Tin, BF, SPLIT>(a, Blk{(int)blockIdx.x, (int)blockIdx.y, 0});
}
template <typename Tin, bool BF, bool SPLIT>
__global__ __launch_bounds__(256, SPLIT ? 3 : 2) void k_toep_h_grp(const ToepHArgs *__restrict__ a, const int *__restrict__ start,
                                                    int n) {
  const int i = group_find(start, n, blockIdx.x);
  toep_h_body<Tin, BF, SPLIT>(a[i], group_blk(a[i].gg, blockIdx.x - start[i]));
}

// ------------------------------------------------------------- launchers
static bool split_of(int variant) { return variant == BF_BLUR_TOEPLITZ_F16X2 || variant == BF_BLUR_TOEPLITZ_BF16X2; }

size_t toeplitz_v_lds(int variant, int rows, int nks) {
  const bool split = split_of(variant);
  const int cols = split ? TShape<true>::kVCols : TShape<false>::kVCols;
  const int Kp = rows - 16 + 32 * nks + 8;
  return tap_frag_bytes(nks, split) + (size_t)(split ? 2 : 1) * 4 * cols * Kp * 2;
}
size_t toeplitz_h_lds(int variant, int nks) {
  const bool split = split_of(variant);
  const int cols = split ? TShape<true>::kHCols : TShape<false>::kHCols;
  const int Kp = cols - 16 + 32 * nks + 8;
  return tap_frag_bytes(nks, split) + (size_t)(split ? 2 : 1) * 4 * kHRows * Kp * 2;
}
int toeplitz_h_tiles(int variant, int H, int W) {
  const int cols = split_of(variant) ? TShape<true>::kHCols : TShape<false>::kHCols;
  return ((W + cols - 1) / cols) * ((H + kHRows - 1) / kHRows);
}

// Per-image arguments of the three Toeplitz kernels for pairs [k0, k0+kcount).
void toeplitz_args(int variant, const void *f, float *out, const Geom &g, DevTables tab, DevState st,
                   const ToepCfg &tc, int k0, int kcount, void *Z, float2 *PQ, bool first, bool last,
                   ToepVArgs &va, ToepHArgs &ha, FinishArgs &fa) {
  const bool split = split_of(variant);
  const int vcols = split ? TShape<true>::kVCols : TShape<false>::kVCols;
  const int hcols = split ? TShape<true>::kHCols : TShape<false>::kHCols;
  const size_t zplane = (size_t)g.H * g.zpitch;
  {
    const int ntx = (g.W + vcols - 1) / vcols, nt = ntx * ((g.H + tc.rows - 1) / tc.rows), per = (nt + 7) / 8;
    va = ToepVArgs{GroupGrid{8 * per, kcount, 1}, f, g, tab, st, tc, ntx, nt, per, k0, Z, zplane};
  }
  {
    const int ntx = (g.W + hcols - 1) / hcols, nt = ntx * ((g.H + kHRows - 1) / kHRows), per = (nt + 7) / 8;
    const bool finish = last && tc.groups == 1;
    ha = ToepHArgs{GroupGrid{8 * per, tc.groups, 1}, f, out, g, tab, st, tc, ntx, nt, per, k0, kcount,
                   (const void *)Z, zplane, PQ, (int)first, (int)finish};
  }
  const int64_t npx = (int64_t)g.H * g.W;
  const int nfin = (last && tc.groups > 1) ? (int)((npx + 255) / 256) : 0;
  // the difference images were divided by the center value
  fa = FinishArgs{GroupGrid{nfin > 0 ? nfin : 1, 1, 1}, f, out, g, st, (const float2 *)PQ, tc.groups, g.center};
}

template <typename Tin, bool BF, bool SPLIT>
static hipError_t toep_t(hipStream_t s, const Tin *f, float *out, const Geom &g, DevTables tab, DevState st,
                         const ToepCfg &tc, int k0, int kcount, void *Z, float2 *PQ, bool first, bool last,
                         const StageRec &rec) {
  const int variant = SPLIT ? (BF ? BF_BLUR_TOEPLITZ_BF16X2 : BF_BLUR_TOEPLITZ_F16X2)
                            : (BF ? BF_BLUR_TOEPLITZ_BF16 : BF_BLUR_TOEPLITZ_F16);
  if (tc.nks < 1 || tc.nks > 8 || 32 * tc.nks < 16 + 2 * tc.R || tc.rows < 16 || tc.rows % 16 || tc.groups < 1 ||
      tc.kpg < 1 || kcount < 1 || kcount > 65535 || tc.groups > 65535)
    return hipErrorInvalidValue;
  ToepVArgs va;
  ToepHArgs ha;
  FinishArgs fa;
  toeplitz_args(variant, f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last, va, ha, fa);
  rec.begin(BF_STAGE_V_TOEPLITZ, s);
  hipLaunchKernelGGL((k_toep_v<Tin, BF, SPLIT>), dim3(va.gg.gx, va.gg.gy), dim3(256),
                     toeplitz_v_lds(variant, tc.rows, tc.nks), s, va);
  rec.end(BF_STAGE_V_TOEPLITZ, s);
  rec.begin(BF_STAGE_H_COMBINE, s);
  hipLaunchKernelGGL((k_toep_h<Tin, BF, SPLIT>), dim3(ha.gg.gx, ha.gg.gy), dim3(256), toeplitz_h_lds(variant, tc.nks),
                     s, ha);
  if (last && !ha.finish) (void)launch_finish(s, dtype_of<Tin>(), &fa, nullptr, nullptr, 0, 0);
  rec.end(BF_STAGE_H_COMBINE, s);
  return hipGetLastError();
}

// Grouped Toeplitz stages over n images of one dtype and variant: the
// vertical pass of all, the horizontal pass of all, then the finishing sums
// of the images that split their pairs into several groups.
template <typename Tin, bool BF, bool SPLIT>
static hipError_t toep_group_t(hipStream_t s, const ToepGroup &tg, const StageRec &rec) {
  rec.begin(BF_STAGE_V_TOEPLITZ, s);
  if (tg.vtotal > 0)
    hipLaunchKernelGGL((k_toep_v_grp<Tin, BF, SPLIT>), dim3(tg.vtotal), dim3(256), tg.vlds, s, tg.va, tg.vstart,
                       tg.n);
  rec.end(BF_STAGE_V_TOEPLITZ, s);
  rec.begin(BF_STAGE_H_COMBINE, s);
  if (tg.htotal > 0)
    hipLaunchKernelGGL((k_toep_h_grp<Tin, BF, SPLIT>), dim3(tg.htotal), dim3(256), tg.hlds, s, tg.ha, tg.hstart,
                       tg.n);
  if (tg.ftotal > 0) (void)launch_finish(s, dtype_of<Tin>(), nullptr, tg.fa, tg.fstart, tg.n, tg.ftotal);
  rec.end(BF_STAGE_H_COMBINE, s);
  return hipGetLastError();
}
template <typename Tin>
static hipError_t toep_group_dt(hipStream_t s, int variant, const ToepGroup &tg, const StageRec &rec) {
  switch (variant) {
    case BF_BLUR_TOEPLITZ_F16: return toep_group_t<Tin, false, false>(s, tg, rec);
    case BF_BLUR_TOEPLITZ_BF16: return toep_group_t<Tin, true, false>(s, tg, rec);
    case BF_BLUR_TOEPLITZ_F16X2: return toep_group_t<Tin, false, true>(s, tg, rec);
    case BF_BLUR_TOEPLITZ_BF16X2: return toep_group_t<Tin, true, true>(s, tg, rec);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_toeplitz_group(hipStream_t s, bf_dtype dt, int variant, const ToepGroup &tg,
                                 const StageRec &rec) {
  switch (dt) {
    case BF_U8: return toep_group_dt<uint8_t>(s, variant, tg, rec);
    case BF_U16: return toep_group_dt<uint16_t>(s, variant, tg, rec);
    default: return toep_group_dt<float>(s, variant, tg, rec);
  }
}

// Dynamic LDS above 64 KB must be allowed per kernel before its launch: the
// kernel's static LDS plus the dynamic allowance may not exceed the CU's LDS.
static hipError_t allow_one(const void *fn) {
  hipFuncAttributes a;
  hipError_t e = hipFuncGetAttributes(&a, fn);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kToepLdsMax - (int)a.sharedSizeBytes);
}
template <typename Tin, bool BF, bool SPLIT>
static hipError_t allow_lds() {
  hipError_t e = allow_one((const void *)k_toep_v<Tin, BF, SPLIT>);
  if (e == hipSuccess) e = allow_one((const void *)k_toep_h<Tin, BF, SPLIT>);
  if (e == hipSuccess) e = allow_one((const void *)k_toep_v_grp<Tin, BF, SPLIT>);
  if (e == hipSuccess) e = allow_one((const void *)k_toep_h_grp<Tin, BF, SPLIT>);
  return e;
}
template <typename Tin>
static hipError_t allow_lds_dt() {
  hipError_t e;
  if ((e = allow_lds<Tin, false, false>()) != hipSuccess) return e;
  if ((e = allow_lds<Tin, true, false>()) != hipSuccess) return e;
  if ((e = allow_lds<Tin, false, true>()) != hipSuccess) return e;
  return allow_lds<Tin, true, true>();
}
hipError_t toeplitz_setup() {
  hipError_t e;
  // non-local means: single-image kernels of the split variants
  if ((e = allow_one((const void *)k_toep_v<Patch8x4, false, true>)) != hipSuccess) return e;
  if ((e = allow_one((const void *)k_toep_h<Patch8x4, false, true>)) != hipSuccess) return e;
  if ((e = allow_one((const void *)k_toep_v<Patch8x4, true, true>)) != hipSuccess) return e;
  if ((e = allow_one((const void *)k_toep_h<Patch8x4, true, true>)) != hipSuccess) return e;
  if ((e = allow_lds_dt<uint8_t>()) != hipSuccess) return e;
  if ((e = allow_lds_dt<uint16_t>()) != hipSuccess) return e;
  return allow_lds_dt<float>();
}

template <typename Tin>
static hipError_t toep_dt(hipStream_t s, int variant, const Tin *f, float *out, const Geom &g, DevTables tab,
                          DevState st, const ToepCfg &tc, int k0, int kcount, void *Z, float2 *PQ, bool first,
                          bool last, const StageRec &rec) {
  switch (variant) {
    case BF_BLUR_TOEPLITZ_F16:
      return toep_t<Tin, false, false>(s, f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last, rec);
    case BF_BLUR_TOEPLITZ_BF16:
      return toep_t<Tin, true, false>(s, f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last, rec);
    case BF_BLUR_TOEPLITZ_F16X2:
      return toep_t<Tin, false, true>(s, f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last, rec);
    case BF_BLUR_TOEPLITZ_BF16X2:
      return toep_t<Tin, true, true>(s, f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last, rec);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_toeplitz_chunk(hipStream_t s, bf_dtype dt, int variant, const void *f, float *out, const Geom &g,
                                 DevTables tab, DevState st, const ToepCfg &tc, int k0, int kcount, void *Z,
                                 float2 *PQ, bool first, bool last, const StageRec &rec) {
  switch (dt) {
    case kDtPatch:  // non-local means: the patch image, split variants only
      if (variant == BF_BLUR_TOEPLITZ_F16X2)
        return toep_t<Patch8x4, false, true>(s, (const Patch8x4 *)f, out, g, tab, st, tc, k0, kcount, Z, PQ, first,
                                             last, rec);
      if (variant == BF_BLUR_TOEPLITZ_BF16X2)
        return toep_t<Patch8x4, true, true>(s, (const Patch8x4 *)f, out, g, tab, st, tc, k0, kcount, Z, PQ, first,
                                            last, rec);
      return hipErrorInvalidValue;
    case BF_U8:
      return toep_dt<uint8_t>(s, variant, (const uint8_t *)f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last,
                              rec);
    case BF_U16:
      return toep_dt<uint16_t>(s, variant, (const uint16_t *)f, out, g, tab, st, tc, k0, kcount, Z, PQ, first,
                               last, rec);
    default:
      return toep_dt<float>(s, variant, (const float *)f, out, g, tab, st, tc, k0, kcount, Z, PQ, first, last,
                            rec);
  }
}

}  // namespace bfi
