// Device helpers shared by the kernel files of libbf.so: the order-table
// lookup and the exact phase generation of the four images of eqs. (f1), (f2).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "bf_device.h"

namespace bfi {

template <typename Tin>
__device__ __forceinline__ float fval(Tin v) {
  return (float)v;
}
// a patch word stands for its centre sample (u_1 = 0)
template <>
__device__ __forceinline__ float fval<Patch8x4>(Patch8x4 v) {
  return (float)(v.v & 0xFFu);
}

__device__ __forceinline__ const OrderEntry &lookup(const DevTables &tab, const int32_t *Tu) {
  int T = *Tu;
  T = T < 0 ? 0 : (T > tab.T_cap ? tab.T_cap : T);
  return tab.ent[tab.idx_of_T[T]];
}

// The order entry of the device's T in registers that are the same in every
// lane.  T and the tables are the same for the whole launch; read through
// pointers that come from memory (grouped launches) the compiler would
// otherwise treat them as per-lane values.
struct UEntry {
  int32_t K, off;
  uint64_t qfix;
  double alpha_turn;
};
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
  return ((uint64_t)(uint32_t)uni((int32_t)(v >> 32)) << 32) | (uint32_t)uni((int32_t)(uint32_t)v);
}
// Tables and T are not written while a blur kernel runs, so they may be read
// through the constant address space: scalar loads, no per-lane wait.
template <typename T>
__device__ __forceinline__ T const_load(const T *p) {
  return *(const __attribute__((address_space(4))) T *)p;
}
__device__ __forceinline__ UEntry uniform_entry(const DevTables &tab, const int32_t *Tu) {
  int T = const_load(Tu);
  T = T < 0 ? 0 : (T > tab.T_cap ? tab.T_cap : T);
  const OrderEntry *e = tab.ent + const_load(tab.idx_of_T + T);
  UEntry u;
  u.K = const_load(&e->K);
  u.off = const_load(&e->off);
  u.qfix = const_load(&e->qfix);
  u.alpha_turn = const_load(&e->alpha_turn);
  return u;
}

// ------------------------------------------------------- phase generation
// Turn (fraction of 2 pi) of the angle m * alpha * v, as an unsigned 32-bit
// fixed-point number.  For integer v the turn is reduced exactly modulo 1 in
// 64-bit arithmetic: with q = frac(alpha/2pi) 2^64, the turn is the top half
// of v * (m q mod 2^64) mod 2^64 (the factor m q is the same for every pixel
// of a frequency and is hoisted by the compiler).  A float v is split into
// its integer part (same exact path) and a fraction r in [0,1) whose small
// angle m*r*alpha is added in double precision.
// Per-frequency constants of the phase: qm = m q mod 2^64 and the turns per
// intensity unit m alpha / 2pi.
struct Freq {
  uint64_t qm;
  double mat;
  uint64_t q;  // non-local means: frac(alpha/2pi) 2^64 and the packed
  int32_t mp;  // multi-index (p signed bytes)
};
__device__ __forceinline__ Freq make_freq(int32_t m, uint64_t q, double at) {
  return Freq{(uint64_t)(int64_t)m * q, (double)m * at, q, m};
}
template <typename Tin>
__device__ __forceinline__ uint32_t phase_turn(Tin v, const Freq &fq) {
  if constexpr (std::is_same<Tin, float>::value) {
    const float fl = floorf(v);
    const int32_t fi = (int32_t)fl;  // intensities lie far inside +-2^31
    const uint32_t ti = (uint32_t)(((uint64_t)(int64_t)fi * fq.qm) >> 32);
    double x = (double)(v - fl) * fq.mat;
    x -= rint(x);  // |x| <= 1/2: x 2^32 fits an int32 but for the single value +2^31
    const int32_t xi = (int32_t)fmin(x * 4294967296.0, 2147483647.0);
    return ti + (uint32_t)xi;
  } else {
    return (uint32_t)(((uint64_t)(uint32_t)v * fq.qm) >> 32);
  }
}
// Non-local means: the phase alpha sum_k m_k f(x + u_k) of a multi-index;
// sum_k m_k f_k is an exact integer (|m_k| <= 127, f_k <= 255, p <= 4),
// reduced like a single frequency's m f.
template <>
__device__ __forceinline__ uint32_t phase_turn<Patch8x4>(Patch8x4 v, const Freq &fq) {
  int32_t u = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) u += (int32_t)(int8_t)(fq.mp >> (8 * k)) * (int32_t)((v.v >> (8 * k)) & 0xFFu);
  return (uint32_t)(((uint64_t)(int64_t)u * fq.q) >> 32);
}
template <typename Tin>
__device__ __forceinline__ uint32_t phase_turn(int32_t m, Tin v, uint64_t q, double at) {
  return phase_turn<Tin>(v, make_freq(m, q, at));
}

// cos and sin of 2 pi tau / 2^32.  The integer turn is reduced exactly to
// [-1/2, 1/2) by the signed reinterpretation, converted to float and passed
// to the hardware sine and cosine, which take their argument in turns
// (max abs error 1.8e-7 measured over 2^24 sampled turns on gfx950).
__device__ __forceinline__ void turn_sincos(uint32_t tau, float &c, float &s) {
  const float x = (float)(int32_t)tau * 2.3283064365386963e-10f;  // 2^-32
  s = __builtin_amdgcn_sinf(x);
  c = __builtin_amdgcn_cosf(x);
}

// 8-bit images: cos and sin of one frequency for all 256 intensities, built
// once per workgroup in LDS (one sincos per thread) instead of once per pixel.
template <typename Tin>
struct PhaseLut {
  static constexpr bool kOn = sizeof(Tin) == 1;
};
__device__ __forceinline__ void build_lut(float2 *lut, int32_t m, uint64_t q, double at, int tid, int nthreads) {
  for (int v = tid; v < 256; v += nthreads) {
    float c, sn;
    turn_sincos(phase_turn<uint8_t>(m, (uint8_t)v, q, at), c, sn);
    lut[v] = make_float2(c, sn);
  }
}

// The four images of one frequency at one pixel: (f-c) cos, (f-c) sin, cos, sin.
template <typename Tin>
__device__ __forceinline__ float4 planes(Tin v, const Freq &fq, float center) {
  float c, s;
  turn_sincos(phase_turn<Tin>(v, fq), c, s);
  const float d = fval(v) - center;
  return make_float4(d * c, d * s, c, s);
}
template <typename Tin>
__device__ __forceinline__ float4 planes(Tin v, int32_t m, uint64_t q, double at, float center) {
  return planes<Tin>(v, make_freq(m, q, at), center);
}
// Same, reading cos/sin from the workgroup's table for 8-bit images.
template <typename Tin>
__device__ __forceinline__ float4 planes_any(Tin v, const float2 *lut, const Freq &fq, float center) {
  if constexpr (PhaseLut<Tin>::kOn) {
    const float2 cs = lut[(int)v];
    const float d = fval(v) - center;
    return make_float4(d * cs.x, d * cs.y, cs.x, cs.y);
  } else {
    return planes<Tin>(v, fq, center);
  }
}
template <typename Tin>
__device__ __forceinline__ float4 planes_any(Tin v, const float2 *lut, int32_t m, uint64_t q, double at,
                                             float center) {
  return planes_any<Tin>(v, lut, make_freq(m, q, at), center);
}

}  // namespace bfi
