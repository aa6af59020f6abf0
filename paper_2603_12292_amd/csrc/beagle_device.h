// Device-side definitions shared by the library's kernels: token format,
// the decoded instruction word, and the operator conventions.
//
// Programs arrive as reverse-Polish token arrays (paper, section 2.1.4).
// A preparation kernel validates each program, re-serialises it so that its
// stack never holds more values than the register need of its expression
// tree (Sethi-Ullman order: at every binary node the operand with the larger
// need is evaluated first; for SUB and DIV the swap is recorded as a
// reversed operator, so values are unchanged), and writes one 32-bit
// instruction word per token:
//
//     word = handler | (arg << 8) | (wslot << 16) | (i0 << 24)
//
// arg is the variable index of VAR words, the constant slot of CONST words
// (their value also sits in a side table by word position) and 0 otherwise.
//
// The interpreter keeps the value on top of the stack in `top` and the n-1
// values below it in stk[0..n-2] (n = stack size before the token).  Every
// token first stores `top` into stk[wslot] with wslot = max(n-1, 0): for a
// push that is the push itself, for any other token it writes a dead slot.
// That store is unconditional, so the stack array has one definition per
// token and the compiler keeps it in place (an indexed register write)
// instead of copying it at the join after the dispatch.  Handlers:
//
//     0                  VAR push (arg = variable)
//     1                  CONST push (value in the side table)
//     2 + 15*o + (n-2)   binary operator o at n = 2..16 values, o in
//                        ADD, SUB, MUL, DIV, RSUB (b - a), RDIV (b / a);
//                        its left operand is stk[n-2], a register named at
//                        compile time
//     92 + u             unary operator u in SIN, COS, EXP, LOG, SQRT,
//                        SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH
//     104 + 6*s + o      fused "push a terminal, then binary operator o"
//                        (s = 0 VAR, 1 CONST): top = top op value; the
//                        stack below top is untouched, so the pair costs one
//                        dispatch and no stack traffic
//
// i0 is the handler of the small-stack interpreter (programs of register
// need <= 4), which keeps no cached top: its handlers are specialised by n
// as well and rewrite stack slots in place (push writes slot n, a binary
// operator slot n-2, unary and fused words slot n-1), so no word moves data
// between registers:
//
//     n                   VAR push at n = 0..3
//     4 + n               CONST push at n
//     8 + 3*o + (n-2)     binary operator o at n = 2..4
//     26 + 4*u + (n-1)    unary operator u (the first five) at n = 1..4
//     46 + 3*(6*s+o) + (n-1)   fused pair at n = 1..3
//     255                 (a word of a program that needs a deeper stack or
//                         uses one of the seven further operators)
//
// Fused pairs make the decoded program shorter than the token program;
// ProgMeta::len counts decoded words.  Programs are grouped by register
// need into classes of 4, 8 and 16 stack slots, each run by a kernel
// instantiated for that stack size.  A program that uses any of the seven
// further operators of the paper's table (SQUARE .. TANH) runs in class 1 at
// least: the small-stack kernels, the hot path of the nine-operator
// programs, carry no code for them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgl {

enum Opcode : uint32_t {
  OP_ADD = 0,
  OP_SUB = 1,
  OP_MUL = 2,
  OP_DIV = 3,
  OP_SIN = 4,
  OP_COS = 5,
  OP_EXP = 6,
  OP_LOG = 7,
  OP_SQRT = 8,
  OP_VAR = 9,
  OP_CONST = 10,
  // the rest of the paper's operator table (unary, unprotected)
  OP_SQUARE = 11,
  OP_RECIP = 12,
  OP_TAN = 13,
  OP_ASIN = 14,
  OP_ACOS = 15,
  OP_ATAN = 16,
  OP_TANH = 17,
  N_OPCODES = 18
};

constexpr uint32_t N_UNARY = 12;  // SIN..SQRT, SQUARE..TANH
constexpr uint32_t U_FIRST_EXT = 5;  // unary index of SQUARE

// unary index u of a unary opcode (0..4: SIN..SQRT, 5..11: SQUARE..TANH)
__host__ __device__ constexpr uint32_t unary_index(uint32_t op) { return op <= OP_SQRT ? op - OP_SIN : op - 6u; }
__host__ __device__ constexpr bool is_extended(uint32_t op) { return op >= OP_SQUARE && op < N_OPCODES; }

enum BinIdx : uint32_t { B_ADD = 0, B_SUB = 1, B_MUL = 2, B_DIV = 3, B_RSUB = 4, B_RDIV = 5 };

constexpr int MAX_STACK = 16;  // largest register need any kernel supports
constexpr int N_CLASSES = 3;   // register-need classes: <= 4, <= 8, <= 16
__host__ __device__ constexpr int class_stack(int c) { return c == 0 ? 4 : (c == 1 ? 8 : 16); }
__host__ __device__ constexpr int need_class(int need) { return need <= 4 ? 0 : (need <= 8 ? 1 : 2); }
constexpr uint32_t H_VAR = 0;
constexpr uint32_t H_CONST = 1;
constexpr uint32_t H_BIN = 2;
constexpr uint32_t H_UN = 2 + 15 * 6;         // 92
constexpr uint32_t H_FUSED = H_UN + N_UNARY;  // 104
constexpr uint32_t I0_PUSH_VAR = 0;
constexpr uint32_t I0_PUSH_CONST = 4;
constexpr uint32_t I0_BIN = 8;
constexpr uint32_t I0_UN = 26;
constexpr uint32_t I0_FUSED = 46;
constexpr uint32_t I0_NONE = 255;
constexpr int MAX_LEN = 4096;
constexpr int MAX_D = 16;

__host__ __device__ constexpr uint32_t h_bin(uint32_t o, int n) { return H_BIN + 15u * o + uint32_t(n - 2); }

__device__ __forceinline__ int arity(uint32_t op) { return op < 4 ? 2 : (op < 9 || (op > OP_CONST && op < N_OPCODES) ? 1 : 0); }

// ---- operator conventions (binary32) -------------------------------------
// The protected quotient b == 0 ? 1 : a / b, correctly rounded.
__device__ __forceinline__ float op_div_cr(float a, float b) { return b == 0.0f ? 1.0f : a / b; }

// binary32 classes (the mask of v_cmp_class_f32): +-normal numbers
constexpr int CLASS_NORMAL = (1 << 3) | (1 << 8);
// NaN, +-Inf, +-0 and +-subnormal numbers
constexpr int CLASS_NOT_NORMAL = 0x3FF & ~CLASS_NORMAL;
// +-0 and +-subnormal numbers
constexpr int CLASS_ZERO_SUB = (1 << 4) | (1 << 5) | (1 << 6) | (1 << 7);

// The protected quotient of K pairs per lane.  Each case first takes the
// faithful quotient q = q0 + (a - b q0) r with r the hardware reciprocal of
// b and q0 = a r (the residual by one FMA; at most 1 ulp from a / b -- the
// reciprocal's error enters only squared); when that q is not a normal
// number (a zero divisor, a zero, subnormal, infinite or NaN quotient, or a
// reciprocal out of range), or when |a| < 2^-100 (below about 2^-102 the
// residual underflows and is no longer exact), the case takes the correctly
// rounded protected quotient instead.  The choice depends on the case
// alone, so every grouping of cases into waves gives the same values; the
// correctly rounded path runs only when some lane of the wave needs it.
// div_tile_r also returns the hardware reciprocals r[k] of b[k] it used
// (the adjoint's derivatives 1/b and -a/b^2 take the same ones).
template <int K>
__device__ __forceinline__ void div_tile_r(const float (&a)[K], const float (&b)[K], float (&q)[K], float (&rr)[K]) {
  uint64_t any = 0;
  bool odd_any = false;
  bool bad[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float r = __builtin_amdgcn_rcpf(b[k]);
    rr[k] = r;
    const float q0 = a[k] * r;
    q[k] = __builtin_fmaf(__builtin_fmaf(-b[k], q0, a[k]), r, q0);
    // q not a normal number (one class test), or a tiny dividend
    const bool odd = __builtin_amdgcn_classf(q[k], CLASS_NOT_NORMAL);
    const bool tiny = __builtin_fabsf(a[k]) < 0x1p-100f;
    bad[k] = odd | tiny;
    odd_any |= odd;
    any |= __builtin_amdgcn_ballot_w64(tiny);
  }
  // (a comparison's ballot is its own result mask; the class tests' lane
  // masks are OR-ed first and turned into one ballot)
  any |= __builtin_amdgcn_ballot_w64(odd_any);
  if (any) {
#pragma unroll
    for (int k = 0; k < K; ++k) q[k] = bad[k] ? op_div_cr(a[k], b[k]) : q[k];
  }
}

template <int K>
__device__ __forceinline__ void div_tile(const float (&a)[K], const float (&b)[K], float (&q)[K]) {
  float r[K];
  div_tile_r<K>(a, b, q, r);
}

__device__ __forceinline__ float op_div(float a, float b) {
  const float av[1] = {a}, bv[1] = {b};
  float q[1];
  div_tile<1>(av, bv, q);
  return q[0];
}
// exp(clamp(x, -80, 80)) = 2^n 2^f with n = rint(x log2 e) and
// f = x log2 e - n in [-1/2, 1/2], f formed with log2 e split into two
// binary32 numbers so that its error stays below 2^-25; 2^f from the hardware
// base-2 exponential, then an exact scaling.  The clamp keeps the result
// normal (e^80 < 2^116, e^-80 > 2^-116), so no range checks are needed.
// Comparisons keep NaN as NaN and map +-Inf to the clamp bounds.
__device__ __forceinline__ float op_exp(float x) {
  const float c = x > 80.0f ? 80.0f : (x < -80.0f ? -80.0f : x);
  const float n = __builtin_rintf(c * 0x1.715476p+0f);
  float f = __builtin_fmaf(c, 0x1.715476p+0f, -n);   // log2 e, high part
  f = __builtin_fmaf(c, 0x1.4ae0c0p-26f, f);        // log2 e, low part
  return __builtin_amdgcn_ldexpf(__builtin_amdgcn_exp2f(f), int(n));
}
// log|x| = log2|x| ln 2 (hardware base-2 logarithm; subnormal |x| scaled by
// 2^32 first, whose log2 is then reduced by 32 exactly), ln 2 split into two
// binary32 numbers of one sign (so log of +Inf stays +Inf); log of 0 is 0.
__device__ __forceinline__ float op_log(float x) {
  const float a = __builtin_fabsf(x);
  const bool tiny = a < 0x1p-126f;
  float y = __builtin_amdgcn_logf(tiny ? a * 0x1p32f : a);
  y = tiny ? y - 32.0f : y;
  const float r = __builtin_fmaf(y, 0x1.62e42ep-1f, y * 0x1.efa39ep-25f);  // ln 2, high and low parts
  return x == 0.0f ? 0.0f : r;
}
// sqrt|x| from the hardware square root, faithful (at most 1 ulp from the
// correctly rounded result over every binary32 input; inputs below 2^-96 are
// scaled by 2^32 first and the result by 2^-16)
__device__ __forceinline__ float op_sqrt(float x) {
  const float a = __builtin_fabsf(x);
  const bool tiny = a < 0x1p-96f;
  const float s = __builtin_amdgcn_sqrtf(tiny ? a * 0x1p32f : a);
  return tiny ? s * 0x1p-16f : s;
}

// Whether any of the K values of any lane satisfies `cond`, a comparison:
// each comparison's result is already a wave mask, OR-ed in scalar
// registers.  (A class test's result is not folded into its ballot that
// way: those are OR-ed as lane masks first and balloted once.)
template <int K, class F>
__device__ __forceinline__ bool wave_any(F cond) {
  uint64_t m = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) m |= __builtin_amdgcn_ballot_w64(cond(k));
  return m != 0;
}

// The same three operators on K values per lane: where no lane holds an
// argument that needs the range handling above (exp: |x| > 80 or NaN; log:
// a zero or subnormal argument; sqrt: |x| < 2^-96), the wave runs the same
// arithmetic without it -- bit-identical results, fewer instructions.
template <int K>
__device__ __forceinline__ void exp_tile(float (&v)[K]) {
  if (!wave_any<K>([&](int k) { return !(__builtin_fabsf(v[k]) <= 80.0f); })) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float n = __builtin_rintf(v[k] * 0x1.715476p+0f);
      float f = __builtin_fmaf(v[k], 0x1.715476p+0f, -n);
      f = __builtin_fmaf(v[k], 0x1.4ae0c0p-26f, f);
      v[k] = __builtin_amdgcn_ldexpf(__builtin_amdgcn_exp2f(f), int(n));
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = op_exp(v[k]);
  }
}

template <int K>
__device__ __forceinline__ void log_tile(float (&v)[K]) {
  bool z = false;
#pragma unroll
  for (int k = 0; k < K; ++k) z |= __builtin_amdgcn_classf(v[k], CLASS_ZERO_SUB);
  if (__builtin_amdgcn_ballot_w64(z) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float y = __builtin_amdgcn_logf(__builtin_fabsf(v[k]));
      v[k] = __builtin_fmaf(y, 0x1.62e42ep-1f, y * 0x1.efa39ep-25f);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = op_log(v[k]);
  }
}

template <int K>
__device__ __forceinline__ void sqrt_tile(float (&v)[K]) {
  if (!wave_any<K>([&](int k) { return __builtin_fabsf(v[k]) < 0x1p-96f; })) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = __builtin_amdgcn_sqrtf(__builtin_fabsf(v[k]));
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = op_sqrt(v[k]);
  }
}

// The seven further operators (unary index U_FIRST_EXT + j), IEEE semantics:
// x * x; 1 / x (correctly rounded, +-Inf at +-0); tan, asin, acos, atan and
// tanh from the device math library (a few ulp; NaN outside the domain of
// asin and acos and for tan of +-Inf).
template <uint32_t U>
__device__ __forceinline__ float op_ext(float x) {
  if constexpr (U == 5) return x * x;
  if constexpr (U == 6) return 1.0f / x;
  if constexpr (U == 7) return tanf(x);
  if constexpr (U == 8) return asinf(x);
  if constexpr (U == 9) return acosf(x);
  if constexpr (U == 10) return atanf(x);
  if constexpr (U == 11) return tanhf(x);
  return 0.0f;
}

// One DPP move of a binary64 value (both halves, the same lane pattern);
// lanes whose source is outside the row, and rows outside ROW_MASK, get 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, ROW_MASK, 0xF, true));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, ROW_MASK, 0xF, true));
  return __longlong_as_double((long long)((uint64_t(hi) << 32) | lo));
}

// Sum of a binary64 value over the 64 lanes, returned in every lane (all
// lanes active).  Row shifts by 1, 2, 4 and 8 leave each row's sum in its
// lane 15; broadcasting lane 15 into rows 1 and 3, then lane 31 into rows 2
// and 3, leaves the total in lane 63.  All register-to-register (the
// butterfly of lane shuffles it replaces went through the LDS crossbar).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(b), 63);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(b >> 32), 63);
  return __longlong_as_double((long long)((uint64_t(hi) << 32) | lo));
}

// Per-program metadata written by the preparation kernel.
struct ProgMeta {
  int32_t status;  // BEAGLE_PROG_* code
  int32_t need;    // register need of the expression tree (max stack size)
  int32_t len;     // decoded instruction words (fused pairs count once)
  float shift;     // correlation fitness: the program's output at case 0
  uint32_t vmask;  // bit d set: the program reads input variable d (staged only then)
};

}  // namespace bgl
