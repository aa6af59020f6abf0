// Binary32 sine and cosine for the interpreter, within about 1.5 ulp of the
// exact values over the whole binary32 range.
//
// |x| = q * pi/2 + r with |r| <= pi/4 (approximately), then sin x and cos x
// are +-sin r or +-cos r by the quadrant q mod 4.
//  - |x| < 2^30: Cody-Waite reduction in binary64 with pi/2 split into two
//    binary64 numbers (binary64 FMA issues at the binary32 rate on this GPU);
//    the error of r is far below binary32 resolution for every binary32 x in
//    this range.
//  - larger finite |x|: Payne-Hanek reduction, an exact integer product of
//    the 24-bit significand with a 96-bit window of the bits of 2/pi chosen
//    by the exponent; quadrant from its integer bits, r from 64 fraction bits.
//  - sin r = r + r^3 S(r^2), cos r = 1 - r^2/2 + r^4 C(r^2): minimax
//    polynomials in binary32.
// Constants: csrc/minimax.py derives every one of them (2/pi bits from an
// integer evaluation of pi, the pi/2 split, the polynomial fits).
//
// The interpreter calls the cheap path for a whole wave when no lane holds a
// large or non-finite argument, and the general one otherwise; the general
// path evaluates one case at a time, so its temporaries do not multiply by
// the cases per lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgl {

constexpr float TRIG_SMALL = 1073741824.0f;  // 2^30: bound of the binary64 reduction

__device__ __forceinline__ float sin_poly(float r) {
  const float r2 = r * r;
  float p = __builtin_fmaf(r2, -0x1.99407200p-13f, 0x1.11073200p-7f);
  p = __builtin_fmaf(r2, p, -0x1.55554600p-3f);
  return __builtin_fmaf(r2 * r, p, r);
}

__device__ __forceinline__ float cos_poly(float r) {
  const float r2 = r * r;
  float p = __builtin_fmaf(r2, 0x1.99e87400p-16f, -0x1.6c0c2800p-10f);
  p = __builtin_fmaf(r2, p, 0x1.55554a00p-5f);
  return __builtin_fmaf(r2 * r2, p, __builtin_fmaf(r2, -0.5f, 1.0f));
}

// r and q of ax = |x| < 2^30.
__device__ __forceinline__ float trig_reduce_small(float ax, int& q) {
  const double xd = double(ax);
  const double qd = __builtin_rint(xd * 0x1.45f306dc9c883p-1);  // 2/pi
  double rd = __builtin_fma(-qd, 0x1.921fb54442d18p+0, xd);     // pi/2, high part
  rd = __builtin_fma(-qd, 0x1.1a62633145c07p-54, rd);           // pi/2, low part
  q = int(qd);
  return float(rd);
}

// r and q (mod 4) of a finite ax >= 2^30 (exponent e >= 30).
__device__ __forceinline__ float trig_reduce_large(float ax, int& q) {
  // bits 1..224 of the binary fraction 2/pi
  static constexpr uint32_t two_over_pi[7] = {0xA2F9836Eu, 0x4E441529u, 0xFC2757D1u, 0xF534DDC0u,
                                              0xDB629599u, 0x3C439041u, 0xFE5163ABu};
  const uint32_t bits = __float_as_uint(ax);
  const int e = int((bits >> 23) & 0xFFu) - 127;  // ax = m * 2^(e - 23)
  const uint64_t m = (bits & 0x7FFFFFu) | 0x800000u;
  // bits of 2/pi above position e - 24 only add multiples of 4 to
  // ax * 2/pi; the window starts there (0-based index g = e - 25 >= 5 for
  // ax >= 2^30; clamped so that the table reads stay in bounds whatever ax)
  const int g = e - 25 > 0 ? e - 25 : 0;
  const int j = g >> 5, sh = g & 31;
  const uint32_t t0 = two_over_pi[j], t1 = two_over_pi[j + 1], t2 = two_over_pi[j + 2], t3 = two_over_pi[j + 3];
  const uint32_t w2 = __funnelshift_l(t1, t0, sh);
  const uint32_t w1 = __funnelshift_l(t2, t1, sh);
  const uint32_t w0 = __funnelshift_l(t3, t2, sh);
  // P = m * (w2:w1:w0) = 2^94 * (ax * 2/pi mod 4) up to the truncated bits
  const uint64_t a0 = m * w0;
  const uint64_t a1 = m * w1 + (a0 >> 32);
  const uint64_t a2 = m * w2 + (a1 >> 32);
  int qq = int((a2 >> 30) & 3u);
  // fraction bits 30..93 of P as a signed fixed-point number: a set top bit
  // means fraction >= 1/2, i.e. the nearest quadrant is the next one
  const uint64_t f = ((a2 & 0x3FFFFFFFull) << 34) | ((a1 & 0xFFFFFFFFull) << 2) | ((a0 & 0xFFFFFFFFull) >> 30);
  const int64_t fs = int64_t(f);
  qq += fs < 0 ? 1 : 0;
  q = qq;
  return float(double(fs) * 0x1.921fb54442d18p-64);  // fraction * pi/2
}

// +-sin r or +-cos r for the quadrant q, sign bit flipped by `neg`.
__device__ __forceinline__ float trig_finish(float r, int q, uint32_t neg) {
  const float v = (q & 1) ? cos_poly(r) : sin_poly(r);
  return __uint_as_float(__float_as_uint(v) ^ ((uint32_t(q) & 2u) << 30) ^ neg);
}

// COS = false: sin x, true: cos x; for |x| < 2^30 only.
template <bool COS>
__device__ __forceinline__ float trig_small(float x) {
  int q;
  const float r = trig_reduce_small(__builtin_fabsf(x), q);
  return trig_finish(r, COS ? q + 1 : q, COS ? 0u : (__float_as_uint(x) & 0x80000000u));
}

// Any binary32 x (NaN and +-Inf give NaN).
template <bool COS>
__device__ __forceinline__ float trig_any(float x) {
  const float ax = __builtin_fabsf(x);
  if (!(ax <= 3.4028234664e38f)) return __builtin_nanf("");
  int q;
  const float r = ax < TRIG_SMALL ? trig_reduce_small(ax, q) : trig_reduce_large(ax, q);
  return trig_finish(r, COS ? q + 1 : q, COS ? 0u : (__float_as_uint(x) & 0x80000000u));
}

// sin or cos of K values per lane: the cheap reduction for the whole wave
// when every argument of every lane is below 2^30, else one case at a time
// through the general path.
template <bool COS, int K>
__device__ __forceinline__ void trig_tile(float (&v)[K]) {
  bool big = false;
#pragma unroll
  for (int k = 0; k < K; ++k) big |= !(__builtin_fabsf(v[k]) < TRIG_SMALL);
  if (__builtin_amdgcn_ballot_w64(big) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = trig_small<COS>(v[k]);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = trig_any<COS>(v[k]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace bgl
