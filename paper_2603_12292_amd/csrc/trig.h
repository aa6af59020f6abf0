// Binary32 sine and cosine for the interpreter, within 2 ulp of the exact
// values over the whole binary32 range.
//
// One odd polynomial serves both functions: |x| = k pi + r (sine) or
// |x| = (j + 1/2) pi + r (cosine) with |r| <= pi/2, and then
//     sin x = sign(x) (-1)^k sin r,      cos x = (-1)^(j+1) sin r.
//  - |x| < 2^30: Cody-Waite reduction in binary64 with pi split into two
//    binary64 numbers (binary64 FMA issues at the binary32 rate on this GPU);
//    the error of r is far below binary32 resolution for every binary32 x in
//    this range.  The integer k comes from one FMA whose addend 1.5 * 2^52
//    makes the sum's unit in the last place 1: the sum is that constant plus
//    the nearest integer, and its low word holds k's parity; for the
//    cosine j = k - 1 with k the integer nearest to |x| / pi + 1/2.
//  - larger finite |x|: Payne-Hanek reduction, an exact integer product of
//    the 24-bit significand with a 96-bit window of the bits of 1/pi chosen
//    by the exponent; k mod 2 from its integer bit, r from 64 fraction bits.
//  - sin r = r + r^3 S(r^2) on [-pi/2, pi/2], S a minimax polynomial of
//    degree 3 evaluated in binary32.
// Constants: csrc/minimax.py derives every one of them (the bits of 1/pi
// from an integer evaluation of pi, the split of pi, the polynomial fit).
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
  float p = __builtin_fmaf(r2, 0x1.5db8e2p-19f, -0x1.9f6fa8p-13f);
  p = __builtin_fmaf(r2, p, 0x1.110ed2p-7f);
  p = __builtin_fmaf(r2, p, -0x1.55554cp-3f);
  return __builtin_fmaf(r2 * r, p, r);
}

constexpr double TRIG_ROUND = 0x1.8p52;  // 1.5 * 2^52

// r (in binary64) for a = |x| < 2^30, and in bit 0 of p the parity of k
// (sine: a = k pi + r) or of j + 1 = k (cosine: a = (j + 1/2) pi + r).
// Takes x itself: the absolute value is taken in binary64, where it is a
// source modifier of the instructions that read it.
template <bool COS>
__device__ __forceinline__ double trig_reduce_small_d(float x, int& p) {
  const double xd = __builtin_fabs(double(x));
  // 1/pi; t = TRIG_ROUND + k
  const double t = COS ? __builtin_fma(xd, 0x1.45f306dc9c883p-2, 0.5) + TRIG_ROUND
                       : __builtin_fma(xd, 0x1.45f306dc9c883p-2, TRIG_ROUND);
  const double h = COS ? (t - TRIG_ROUND) - 0.5 : t - TRIG_ROUND;
  double r = __builtin_fma(-h, 0x1.921fb54442d18p+1, xd);  // pi, high part
  r = __builtin_fma(-h, 0x1.1a62633145c07p-53, r);         // pi, low part
  p = int(uint32_t(uint64_t(__builtin_bit_cast(uint64_t, t))));
  return r;
}

template <bool COS>
__device__ __forceinline__ float trig_reduce_small(float x, int& p) {
  return float(trig_reduce_small_d<COS>(x, p));
}

// The same for a finite a >= 2^30 (exponent e >= 30).
template <bool COS>
__device__ __forceinline__ float trig_reduce_large(float a, int& p) {
  // bits 1..224 of the binary fraction 2/pi; bit j of 1/pi is bit j - 1 of 2/pi
  static constexpr uint32_t two_over_pi[7] = {0xA2F9836Eu, 0x4E441529u, 0xFC2757D1u, 0xF534DDC0u,
                                              0xDB629599u, 0x3C439041u, 0xFE5163ABu};
  const uint32_t bits = __float_as_uint(a);
  const int e = int((bits >> 23) & 0xFFu) - 127;  // a = m * 2^(e - 23)
  const uint64_t m = (bits & 0x7FFFFFu) | 0x800000u;
  // bits of 1/pi above position e - 23 only add even integers to a / pi;
  // the window starts there, i.e. at bit e - 24 of 2/pi (0-based index
  // g = e - 25 >= 5 for a >= 2^30; clamped so that the table reads stay in
  // bounds whatever a)
  const int g = e - 25 > 0 ? e - 25 : 0;
  const int j = g >> 5, sh = g & 31;
  const uint32_t t0 = two_over_pi[j], t1 = two_over_pi[j + 1], t2 = two_over_pi[j + 2], t3 = two_over_pi[j + 3];
  const uint32_t w2 = __funnelshift_l(t1, t0, sh);
  const uint32_t w1 = __funnelshift_l(t2, t1, sh);
  const uint32_t w0 = __funnelshift_l(t3, t2, sh);
  // P = m * (w2:w1:w0) = 2^95 * (a / pi mod 2) up to the truncated bits
  const uint64_t a0 = m * w0;
  const uint64_t a1 = m * w1 + (a0 >> 32);
  const uint64_t a2 = m * w2 + (a1 >> 32);
  const int k0 = int((a2 >> 31) & 1u);
  // fraction bits 31..94 of P: f in [0, 1) as a 64-bit fixed-point number
  const uint64_t f = ((a2 & 0x7FFFFFFFull) << 33) | ((a1 & 0xFFFFFFFFull) << 1) | ((a0 & 0xFFFFFFFFull) >> 31);
  // sine: the nearest k (f >= 1/2 rounds up), r = (f - [f >= 1/2]) pi;
  // cosine: k = k0, r = (f - 1/2) pi; both as signed 64-bit fixed point
  const int64_t v = COS ? int64_t(f ^ 0x8000000000000000ull) : int64_t(f);
  p = COS ? k0 + 1 : k0 + int(f >> 63);
  return float(double(v) * 0x1.921fb54442d18p-63);  // * pi * 2^-64
}

// (-1)^p sin r, sign bit also flipped by `neg` (0 or the sign bit).  Adding
// p << 31 flips the sign bit exactly as an exclusive or would (the carry
// leaves the word), in one instruction with the shift.
__device__ __forceinline__ float trig_finish(float r, int p, uint32_t neg) {
  return __uint_as_float((__float_as_uint(sin_poly(r)) + (uint32_t(p) << 31)) ^ neg);
}

// COS = false: sin x, true: cos x; for |x| < 2^30 only.
template <bool COS>
__device__ __forceinline__ float trig_small(float x) {
  int p;
  const float r = trig_reduce_small<COS>(x, p);
  return trig_finish(r, p, COS ? 0u : (__float_as_uint(x) & 0x80000000u));
}

// Any binary32 x (NaN and +-Inf give NaN); the same value as trig_small
// where both apply.
template <bool COS>
__device__ __forceinline__ float trig_any(float x) {
  const float a = __builtin_fabsf(x);
  if (!(a <= 3.4028234664e38f)) return __builtin_nanf("");
  if (a < TRIG_SMALL) return trig_small<COS>(x);
  int p;
  const float r = trig_reduce_large<COS>(a, p);
  return trig_finish(r, p, COS ? 0u : (__float_as_uint(x) & 0x80000000u));
}

// x as a value the compiler cannot see through (an empty asm, no
// instruction): |x| of the fast paths, taken in binary64 as a source
// modifier, is then not merged with |x| of the range test, which would be
// kept in a register by a separate AND.
__device__ __forceinline__ float trig_fresh(float x) {
  float y;
  asm("" : "=v"(y) : "0"(x));
  return y;
}

// sin or cos of K values per lane: the cheap reduction for the whole wave
// when every argument of every lane is below 2^30, else one case at a time
// through the general path.
template <bool COS, int K>
__device__ __forceinline__ void trig_tile(float (&v)[K]) {
  uint64_t big = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) big |= __builtin_amdgcn_ballot_w64(!(__builtin_fabsf(v[k]) < TRIG_SMALL));
  if (big == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = trig_small<COS>(trig_fresh(v[k]));
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = trig_any<COS>(v[k]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// sin x (the interpreter's value, bit for bit) and cos x from one reduction
// of K values per lane; s holds x on entry.  With x = k pi + r, |r| <= pi/2:
// cos x = (-1)^k cos r = (-1)^k sin(pi/2 - |r|), the argument formed in
// binary64 (pi/2 as the halves of the split of pi), so cos x is as accurate
// as the sine's polynomial allows away from its zeros and within ~1e-8
// absolute near them.  Large or non-finite arguments of any lane: the
// general path per case.
template <int K>
__device__ __forceinline__ void sincos_tile(float (&s)[K], float (&c)[K]) {
  uint64_t big = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) big |= __builtin_amdgcn_ballot_w64(!(__builtin_fabsf(s[k]) < TRIG_SMALL));
  if (big == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float x = trig_fresh(s[k]);
      int p;
      const double r = trig_reduce_small_d<false>(x, p);
      s[k] = trig_finish(float(r), p, __float_as_uint(x) & 0x80000000u);
      const double u = (0x1.921fb54442d18p+0 - __builtin_fabs(r)) + 0x1.1a62633145c07p-54;
      c[k] = trig_finish(float(u), p, 0u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float x = s[k];
      s[k] = trig_any<false>(x);
      c[k] = trig_any<true>(x);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// cos x (the interpreter's value, bit for bit) and -sin x of K values per
// lane from the cosine's reduction: with |x| = (j + 1/2) pi + r,
// sin x = sign(x) (-1)^j cos r and cos r = sin(pi/2 - |r|), the argument
// formed in binary64 -- as accurate as sincos_tile's cosine.  c holds x on
// entry.  Large or non-finite arguments of any lane: the general path per
// case.
template <int K>
__device__ __forceinline__ void cos_nsin_tile(float (&c)[K], float (&ns)[K]) {
  uint64_t big = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) big |= __builtin_amdgcn_ballot_w64(!(__builtin_fabsf(c[k]) < TRIG_SMALL));
  if (big == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float x = trig_fresh(c[k]);
      int p;
      const double r = trig_reduce_small_d<true>(x, p);
      c[k] = trig_finish(float(r), p, 0u);
      const double u = (0x1.921fb54442d18p+0 - __builtin_fabs(r)) + 0x1.1a62633145c07p-54;
      ns[k] = trig_finish(float(u), p, __float_as_uint(x) & 0x80000000u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float x = c[k];
      c[k] = trig_any<true>(x);
      ns[k] = -trig_any<false>(x);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace bgl
