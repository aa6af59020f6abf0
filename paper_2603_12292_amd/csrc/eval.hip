// Population evaluation: the stack interpreter, per-case fitness terms,
// in-block reductions and the cross-chunk finalize.
//
// Work decomposition.  A workgroup of 4 waves evaluates ONE program on one
// chunk of fitness cases; each wave walks the chunk in tiles of 64 lanes x
// K cases, so every token of the program is decoded once per tile (a
// wave-uniform scalar branch on the handler byte) and applied to K cases per
// lane.  All lanes of a wave run the same program on different cases, the
// mapping the paper's kernel uses to avoid divergence (section 2.1.2), but
// with no cap on the number of cases.
//
// The decoded program stays in two VGPRs per 64 tokens (one word per lane,
// fetched with v_readlane); constants come from a side table read the same
// way.  The operand stack lives in registers with compile-time names: the
// handler byte fixes the stack size at which a token runs.
#include <hip/hip_ext.h>

#include <cmath>

#include "beagle_device.h"
#include "kernels.h"
#include "trig.h"

namespace bgl {

template <uint32_t O>
__device__ __forceinline__ float binop(float a, float b) {
  if constexpr (O == B_ADD) return a + b;
  if constexpr (O == B_SUB) return a - b;
  if constexpr (O == B_MUL) return a * b;
  if constexpr (O == B_DIV) return op_div(a, b);
  if constexpr (O == B_RSUB) return b - a;
  if constexpr (O == B_RDIV) return op_div(b, a);
  return 0.0f;
}

// r[k] = a[k] op b[k] on the K cases of a lane; the protected division
// (and its reversed form) through div_tile, one check per wave
template <uint32_t O, int K>
__device__ __forceinline__ void binop_tile(const float (&a)[K], const float (&b)[K], float (&r)[K]) {
  if constexpr (O == B_DIV) {
    div_tile<K>(a, b, r);
  } else if constexpr (O == B_RDIV) {
    div_tile<K>(b, a, r);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = binop<O>(a[k], b[k]);
  }
}

// The wave's input tile in LDS: variable d of case k (k-th of this lane's K
// cases) lives at  ((d * G + k / 4) * 64 + lane) * 4 + k % 4  floats, G =
// ceil(K / 4): every 16-byte access of a wave is contiguous across lanes
// (no bank conflicts).  xl points at lane * 4 floats of the tile.
template <int K>
struct XRow {
  float v[K];
};

template <int K>
__device__ __forceinline__ XRow<K> load_row(const float* xl, uint32_t d) {
  constexpr int G = (K + 3) / 4;
  XRow<K> r;
  if constexpr (K >= 4) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float4 q = *reinterpret_cast<const float4*>(xl + (d * G + g) * 256);
      r.v[4 * g + 0] = q.x;
      r.v[4 * g + 1] = q.y;
      r.v[4 * g + 2] = q.z;
      r.v[4 * g + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = xl[d * 256 + k];
  }
  return r;
}

template <int K>
__device__ __forceinline__ void store_row(float* xl, uint32_t d, const XRow<K>& r) {
  constexpr int G = (K + 3) / 4;
  if constexpr (K >= 4) {
#pragma unroll
    for (int g = 0; g < G; ++g)
      *reinterpret_cast<float4*>(xl + (d * G + g) * 256) =
          make_float4(r.v[4 * g + 0], r.v[4 * g + 1], r.v[4 * g + 2], r.v[4 * g + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) xl[d * 256 + k] = r.v[k];
  }
}

// The stack interpreter for one program on K cases per lane.
//   vc0/vv0, vc1/vv1: instruction words / constant values of tokens 0..63
//   and 64..127 (one per lane); longer programs read later tokens from
//   memory.  xl points at this lane's inputs in the wave's LDS tile (see
//   load_row).
template <int K, int S>
__device__ __forceinline__ void interpret(uint32_t vc0, float vv0, uint32_t vc1, float vv1,
                                          const uint32_t* __restrict__ code, const float* __restrict__ cval,
                                          int L, int lane, const float* xl, float (&top)[K]) {
  // S slots: the unconditional store of a token at stack size n = S lands in
  // slot S-1, above the S-1 live values
  float stk[K][S];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    top[k] = 0.0f;
#pragma unroll
    for (int j = 0; j < S; ++j) stk[k][j] = 0.0f;
  }
  for (int base = 0; base < L; base += 64) {
    uint32_t vc;
    float vv;
    if (base == 0) {
      vc = vc0;
      vv = vv0;
    } else if (base == 64) {
      vc = vc1;
      vv = vv1;
    } else {
      const int i = base + lane;
      vc = i < L ? code[i] : 0u;
      vv = i < L ? cval[i] : 0.0f;
    }
    const int n = __builtin_amdgcn_readfirstlane(L - base < 64 ? L - base : 64);
    for (int t = 0; t < n; ++t) {
      const uint32_t w = __builtin_amdgcn_readlane(vc, t);
      const uint32_t arg = (w >> 8) & 0xFFu;
      const uint32_t ws = (w >> 16) & 0xFu;
#pragma unroll
      for (int k = 0; k < K; ++k) stk[k][ws] = top[k];
      switch (w & 0xFFu) {
        case H_VAR: {
          const XRow<K> xv = load_row<K>(xl, arg);
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = xv.v[k];
          break;
        }
        case H_CONST: {
          const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t));
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = v;
          break;
        }
#define BGL_BIN(O, N)                                                          \
  case H_BIN + 15 * O + (N - 2):                                               \
    if constexpr (N <= S) {                                                    \
      float a_[K], t_[K];                                                      \
      _Pragma("unroll") for (int k = 0; k < K; ++k) {                          \
        a_[k] = stk[k][N <= S ? N - 2 : 0];                                    \
        t_[k] = top[k];                                                        \
      }                                                                        \
      binop_tile<O, K>(a_, t_, top);                                           \
    }                                                                          \
    break;
#define BGL_BIN_ALL(O)                                                          \
  BGL_BIN(O, 2) BGL_BIN(O, 3) BGL_BIN(O, 4) BGL_BIN(O, 5) BGL_BIN(O, 6) BGL_BIN(O, 7) \
  BGL_BIN(O, 8) BGL_BIN(O, 9) BGL_BIN(O, 10) BGL_BIN(O, 11) BGL_BIN(O, 12)     \
  BGL_BIN(O, 13) BGL_BIN(O, 14) BGL_BIN(O, 15) BGL_BIN(O, 16)
        BGL_BIN_ALL(B_ADD)
        BGL_BIN_ALL(B_SUB)
        BGL_BIN_ALL(B_MUL)
        BGL_BIN_ALL(B_DIV)
        BGL_BIN_ALL(B_RSUB)
        BGL_BIN_ALL(B_RDIV)
#undef BGL_BIN
#undef BGL_BIN_ALL
#define BGL_FUSED(O)                                                           \
  case H_FUSED + O: {                                                          \
    const XRow<K> xv = load_row<K>(xl, arg);                                   \
    float t_[K];                                                               \
    _Pragma("unroll") for (int k = 0; k < K; ++k) t_[k] = top[k];              \
    binop_tile<O, K>(t_, xv.v, top);                                           \
    break;                                                                     \
  }                                                                            \
  case H_FUSED + 6 + O: {                                                      \
    const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t)); \
    float t_[K], c_[K];                                                        \
    _Pragma("unroll") for (int k = 0; k < K; ++k) {                            \
      t_[k] = top[k];                                                          \
      c_[k] = v;                                                               \
    }                                                                          \
    binop_tile<O, K>(t_, c_, top);                                             \
    break;                                                                     \
  }
        BGL_FUSED(B_ADD)
        BGL_FUSED(B_SUB)
        BGL_FUSED(B_MUL)
        BGL_FUSED(B_DIV)
        BGL_FUSED(B_RSUB)
        BGL_FUSED(B_RDIV)
#undef BGL_FUSED
        case H_UN + 0:
          trig_tile<false, K>(top);
          break;
        case H_UN + 1:
          trig_tile<true, K>(top);
          break;
        case H_UN + 2:
          exp_tile<K>(top);
          break;
        case H_UN + 3:
          log_tile<K>(top);
          break;
        case H_UN + 4:
          sqrt_tile<K>(top);
          break;
#define BGL_EXT(U)                                                             \
  case H_UN + U:                                                               \
    _Pragma("unroll") for (int k = 0; k < K; ++k) top[k] = op_ext<U>(top[k]);  \
    break;
        BGL_EXT(5) BGL_EXT(6) BGL_EXT(7) BGL_EXT(8) BGL_EXT(9) BGL_EXT(10) BGL_EXT(11)
#undef BGL_EXT
        default:
          break;
      }
    }
  }
}

// The small-stack interpreter (programs of register need <= 4): no cached
// top; the handler index i0 (word bits 24..31) names the stack size, so each
// handler reads and rewrites its slots in place and no word moves values
// between registers.  st[k][j] is stack slot j of case k; the result is slot 0.
template <int K>
__device__ __forceinline__ void interpret_small(uint32_t vc0, float vv0, uint32_t vc1, float vv1,
                                                const uint32_t* __restrict__ code, const float* __restrict__ cval,
                                                int L, int lane, const float* xl, float (&res)[K]) {
  constexpr int S = 4;
  float st[K][S];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int j = 0; j < S; ++j) st[k][j] = 0.0f;
  for (int base = 0; base < L; base += 64) {
    uint32_t vc;
    float vv;
    if (base == 0) {
      vc = vc0;
      vv = vv0;
    } else if (base == 64) {
      vc = vc1;
      vv = vv1;
    } else {
      const int i = base + lane;
      vc = i < L ? code[i] : 0u;
      vv = i < L ? cval[i] : 0.0f;
    }
    const int n = __builtin_amdgcn_readfirstlane(L - base < 64 ? L - base : 64);
    for (int t = 0; t < n; ++t) {
      const uint32_t w = __builtin_amdgcn_readlane(vc, t);
      const uint32_t arg = (w >> 8) & 0xFFu;
      switch (w >> 24) {
#define BGL_S_PUSH(N)                                                           \
  case I0_PUSH_VAR + N: {                                                       \
    const XRow<K> xv = load_row<K>(xl, arg);                                    \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N] = xv.v[k];           \
    break;                                                                      \
  }                                                                             \
  case I0_PUSH_CONST + N: {                                                     \
    const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t)); \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N] = v;                 \
    break;                                                                      \
  }
        BGL_S_PUSH(0) BGL_S_PUSH(1) BGL_S_PUSH(2) BGL_S_PUSH(3)
#undef BGL_S_PUSH
#define BGL_S_BIN(O, N)                                                         \
  case I0_BIN + 3 * O + (N - 2): {                                              \
    float a_[K], b_[K], r_[K];                                                  \
    _Pragma("unroll") for (int k = 0; k < K; ++k) {                             \
      a_[k] = st[k][N - 2];                                                     \
      b_[k] = st[k][N - 1];                                                     \
    }                                                                           \
    binop_tile<O, K>(a_, b_, r_);                                               \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 2] = r_[k];         \
    break;                                                                      \
  }
#define BGL_S_BIN3(O) BGL_S_BIN(O, 2) BGL_S_BIN(O, 3) BGL_S_BIN(O, 4)
        BGL_S_BIN3(B_ADD) BGL_S_BIN3(B_SUB) BGL_S_BIN3(B_MUL) BGL_S_BIN3(B_DIV) BGL_S_BIN3(B_RSUB) BGL_S_BIN3(B_RDIV)
#undef BGL_S_BIN3
#undef BGL_S_BIN
#define BGL_S_UN(N)                                                             \
  case I0_UN + 0 * 4 + (N - 1): {                                               \
    float c[K];                                                                 \
    _Pragma("unroll") for (int k = 0; k < K; ++k) c[k] = st[k][N - 1];          \
    trig_tile<false, K>(c);                                                     \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = c[k];          \
    break;                                                                      \
  }                                                                             \
  case I0_UN + 1 * 4 + (N - 1): {                                               \
    float c[K];                                                                 \
    _Pragma("unroll") for (int k = 0; k < K; ++k) c[k] = st[k][N - 1];          \
    trig_tile<true, K>(c);                                                      \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = c[k];          \
    break;                                                                      \
  }                                                                             \
  case I0_UN + 2 * 4 + (N - 1): {                                               \
    float c[K];                                                                 \
    _Pragma("unroll") for (int k = 0; k < K; ++k) c[k] = st[k][N - 1];          \
    exp_tile<K>(c);                                                             \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = c[k];          \
    break;                                                                      \
  }                                                                             \
  case I0_UN + 3 * 4 + (N - 1): {                                               \
    float c[K];                                                                 \
    _Pragma("unroll") for (int k = 0; k < K; ++k) c[k] = st[k][N - 1];          \
    log_tile<K>(c);                                                             \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = c[k];          \
    break;                                                                      \
  }                                                                             \
  case I0_UN + 4 * 4 + (N - 1): {                                               \
    float c[K];                                                                 \
    _Pragma("unroll") for (int k = 0; k < K; ++k) c[k] = st[k][N - 1];          \
    sqrt_tile<K>(c);                                                            \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = c[k];          \
    break;                                                                      \
  }
        BGL_S_UN(1) BGL_S_UN(2) BGL_S_UN(3) BGL_S_UN(4)
#undef BGL_S_UN
#define BGL_S_FUSED(O, N)                                                       \
  case I0_FUSED + 3 * O + (N - 1): {                                            \
    const XRow<K> xv = load_row<K>(xl, arg);                                    \
    float a_[K], r_[K];                                                         \
    _Pragma("unroll") for (int k = 0; k < K; ++k) a_[k] = st[k][N - 1];         \
    binop_tile<O, K>(a_, xv.v, r_);                                             \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = r_[k];         \
    break;                                                                      \
  }                                                                             \
  case I0_FUSED + 3 * (6 + O) + (N - 1): {                                      \
    const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t)); \
    float a_[K], c_[K], r_[K];                                                  \
    _Pragma("unroll") for (int k = 0; k < K; ++k) {                             \
      a_[k] = st[k][N - 1];                                                     \
      c_[k] = v;                                                                \
    }                                                                           \
    binop_tile<O, K>(a_, c_, r_);                                               \
    _Pragma("unroll") for (int k = 0; k < K; ++k) st[k][N - 1] = r_[k];         \
    break;                                                                      \
  }
#define BGL_S_FUSED3(O) BGL_S_FUSED(O, 1) BGL_S_FUSED(O, 2) BGL_S_FUSED(O, 3)
        BGL_S_FUSED3(B_ADD) BGL_S_FUSED3(B_SUB) BGL_S_FUSED3(B_MUL) BGL_S_FUSED3(B_DIV) BGL_S_FUSED3(B_RSUB)
        BGL_S_FUSED3(B_RDIV)
#undef BGL_S_FUSED3
#undef BGL_S_FUSED
        default:
          break;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) res[k] = st[k][0];
}

// Eq. 3 for one case (the paper's point-to-point score, see beagle.h): the
// products and differences rounded separately (no contraction), so that the
// rounding decision is the one a plain binary64 evaluation takes.
__device__ __forceinline__ double point_case(float yh, float y, double smax, double s11) {
  const bool vh = isfinite(yh), vy = isfinite(y);
  if (!(vh && vy)) return vh == vy ? smax : -smax;
  const double a = fabs(double(yh)), b = fabs(double(y));
  const double hi = a > b ? a : b, lo = a > b ? b : a;
  if (hi == 0.0) return smax;
  double t = __dmul_rn(smax, lo / hi);
  if ((yh < 0.0f && y > 0.0f) || (yh > 0.0f && y < 0.0f)) t = __dsub_rn(t, s11);
  return __builtin_rint(t);
}

// Per-lane accumulators of one fitness kind over the cases a lane adds, and
// their wave sums in partial order (see eval_block).
template <int KIND>
struct Acc {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  uint32_t n1 = 0u, n2 = 0u;
  __device__ __forceinline__ void add(float yh, float yt, bool valid, double shift, double ybar, double smax,
                                      double s11) {
    // masks act on the terms' inputs and every product is an explicit FMA,
    // so a case adds the same bits whether its tile is masked or not
    if constexpr (KIND == BEAGLE_FIT_MSE) {
      const double d = valid ? double(yh) - double(yt) : 0.0;
      s0 = __builtin_fma(d, d, s0);
    } else if constexpr (KIND == BEAGLE_FIT_CORR) {
      const double u = valid ? double(yh) - shift : 0.0;
      const double w = valid ? double(yt) - ybar : 0.0;
      s0 += u;
      s1 = __builtin_fma(u, u, s1);
      s2 = __builtin_fma(u, w, s2);
    } else if constexpr (KIND == BEAGLE_FIT_POINT) {
      s0 += valid ? point_case(yh, yt, smax, s11) : 0.0;
    } else {
      const bool vh = isfinite(yh), vy = isfinite(yt);
      const bool both = valid && vh && vy;
      n1 += valid && vh != vy ? 1u : 0u;
      n2 += valid && !vh && !vy ? 1u : 0u;
      const double u = both ? double(yh) - shift : 0.0;
      const double w = both ? double(yt) - ybar : 0.0;
      s0 += u;
      s1 = __builtin_fma(u, u, s1);
      s2 = __builtin_fma(u, w, s2);
      s3 += w;
      s4 = __builtin_fma(w, w, s4);
    }
  }
  // the wave's sums in partial order: MSE, POINT {s0}; CORR {s0, s1, s2};
  // R4 {c1, c2, s0, s1, s2, s3, s4}
  __device__ __forceinline__ void wave_sums(double (&v)[MAX_SUMS]) const {
    if constexpr (KIND == BEAGLE_FIT_R4) {
      v[0] = wave_sum(double(n1));
      v[1] = wave_sum(double(n2));
      v[2] = wave_sum(s0);
      v[3] = wave_sum(s1);
      v[4] = wave_sum(s2);
      v[5] = wave_sum(s3);
      v[6] = wave_sum(s4);
    } else {
      v[0] = wave_sum(s0);
      if constexpr (KIND == BEAGLE_FIT_CORR) {
        v[1] = wave_sum(s1);
        v[2] = wave_sum(s2);
      }
    }
  }
};

// One workgroup: program p on case chunk c.  Writes the chunk's partial sums
//   MSE  : part[0][c][p] = sum (yhat - y)^2
//   CORR : part[j][c][p] = sum u, sum u^2, sum u*w   (u = yhat - shift_p,
//          w = y - ybar), all in binary64
//   POINT: part[0][c][p] = sum of the Eq. 3 case scores (integers, exact)
//   R4   : part[j][c][p] = c1, c2 (cases with one / two invalid values), and
//          over the cases where both are valid sum u, sum u^2, sum u*w,
//          sum w, sum w^2.
template <int KIND, int K, int S>
__device__ __forceinline__ void eval_block(const EvalArgs& a, int p, int c, float* xtile) {
  const ProgMeta m = a.meta[p];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t off = a.tok_offset[p];
  const uint32_t* code = a.code + off;
  const float* cval = a.cval + off;
  const int L = m.len;
  const uint32_t vc0 = lane < L ? code[lane] : 0u;
  const float vv0 = lane < L ? cval[lane] : 0.0f;
  const uint32_t vc1 = lane + 64 < L ? code[lane + 64] : 0u;
  const float vv1 = lane + 64 < L ? cval[lane + 64] : 0.0f;
  const double shift = double(m.shift);
  const uint32_t vmask = uint32_t(__builtin_amdgcn_readfirstlane(int(m.vmask)));
  const double ybar = KIND == BEAGLE_FIT_CORR || KIND == BEAGLE_FIT_R4 ? a.stats[0] : 0.0;
  const double smax = a.smax, s11 = a.smax / 11.0;
  Acc<KIND> acc;
  const int64_t c0 = int64_t(c) * a.chunk;
  const int64_t c1 = c0 + a.chunk < a.M ? c0 + a.chunk : a.M;
  // this wave's input tile (layout: load_row); G * 256 floats per variable
  constexpr int G = (K + 3) / 4;
  float* xw = xtile + wave * (a.D * G * 256);
  float* xl = xw + lane * 4;
  // Case order.  A sub-tile is 64 lanes x min(K, 4) cases; the block's
  // waves take consecutive sub-tiles, and a lane with K = 8 holds two
  // sub-tiles EVAL_WAVES sub-tiles apart.  Lane l holds cases 4l .. 4l+3 of a
  // sub-tile (K >= 4; k * 64 + l for K = 2).  So each lane adds exactly the
  // cases it would add with K = 4, in the same order: the tile width of
  // class 0 changes no result bit.
  constexpr int SUB = K < 4 ? K : 4;
  constexpr int SPAN = EVAL_WAVES * 64 * SUB;  // cases of one sub-tile row of the block
  constexpr int NSUB = K / SUB;
  for (int64_t base = c0 + int64_t(wave) * (64 * SUB); base < c1; base += int64_t(NSUB) * SPAN) {
    float yk[K];
    if constexpr (K >= 4) {
      // the tile's inputs go straight from global memory to LDS (16 bytes =
      // 4 cases per lane, the layout load_row reads); every variable's loads
      // are issued before one wait
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the last tile's LDS reads are done
      for (int d = 0; d < a.D; ++d) {
        if (!((vmask >> d) & 1u)) continue;  // a variable the program never reads
#pragma unroll
        for (int g = 0; g < NSUB; ++g)
          __builtin_amdgcn_global_load_lds(a.Xt + int64_t(d) * a.Mp + base + g * SPAN + 4 * lane,
                                           xw + (d * NSUB + g) * 256, 16, 0, 0);
      }
#pragma unroll
      for (int g = 0; g < NSUB; ++g) {
        const float4 q = *reinterpret_cast<const float4*>(a.yp + base + g * SPAN + 4 * lane);
        yk[4 * g + 0] = q.x;
        yk[4 * g + 1] = q.y;
        yk[4 * g + 2] = q.z;
        yk[4 * g + 3] = q.w;
      }
      __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the tile is in LDS
      __builtin_amdgcn_wave_barrier();
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) yk[k] = a.yp[base + k * 64 + lane];
      // coalesced global reads, one LDS write per variable; the wave's tile
      // is private to it, so a wave barrier suffices
      for (int d = 0; d < a.D; ++d) {
        if (!((vmask >> d) & 1u)) continue;
        XRow<K> xv;
#pragma unroll
        for (int k = 0; k < K; ++k) xv.v[k] = a.Xt[int64_t(d) * a.Mp + base + k * 64 + lane];
        __builtin_amdgcn_wave_barrier();
        store_row<K>(xl, d, xv);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the tile is in LDS
    }
    float top[K];
    if constexpr (S == 4)
      interpret_small<K>(vc0, vv0, vc1, vv1, code, cval, L, lane, xl, top);
    else
      interpret<K, S>(vc0, vv0, vc1, vv1, code, cval, L, lane, xl, top);
    // a tile wholly inside the case set (every tile but the last) adds
    // without per-case validity masks
    if (base + int64_t(NSUB - 1) * SPAN + 64 * SUB <= a.M) {
#pragma unroll
      for (int k = 0; k < K; ++k) acc.add(top[k], yk[k], true, shift, ybar, smax, s11);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool valid = base + (k / SUB) * SPAN + (K >= 4 ? 4 * lane + (k % 4) : k * 64 + lane) < a.M;
        acc.add(top[k], yk[k], valid, shift, ybar, smax, s11);
      }
    }
  }
  // the waves' sums meet in the start of each wave's own tile (its tiles
  // are done; no LDS beyond the tiles, so that eight workgroups of four
  // waves fit a CU at D = 5)
  constexpr int NS = kind_sums(KIND);
  const int wstride = a.D * G * 256;  // floats per wave tile
  double v[MAX_SUMS];
  acc.wave_sums(v);
  if (lane == 0) {
    double* mine = reinterpret_cast<double*>(xw);
#pragma unroll
    for (int j = 0; j < NS; ++j) mine[j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    const int j = threadIdx.x;
    auto red = [&](int w) { return reinterpret_cast<const double*>(xtile + w * wstride)[j]; };
    const double t = ((red(0) + red(1)) + red(2)) + red(3);
    a.part[(int64_t(j) * a.n_chunks + c) * a.n_programs + p] = t;
  }
  __syncthreads();
}

// One register-need class: a persistent grid pulls (chunk, program) work
// items from an atomic counter, chunk-major so that the workgroups running
// at any moment share one chunk of cases in L2.  Which workgroup takes which
// item does not change any result: each item writes its own partial.
// The 4-case class-0 variant is held to CLASS0_NARROW_WAVES waves per SIMD
// (7: 72 VGPRs instead of its natural 85, five waves; eight would not fit
// the LDS of seven workgroups' input tiles at D = 5 anyway); the values this
// moves to scratch are per-item and per-tile bookkeeping, none inside the
// per-token loop.
#ifndef CLASS0_NARROW_WAVES
#define CLASS0_NARROW_WAVES 7
#endif
template <int KIND, int CLS, int KV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CLS == 0 && KV == 1 ? CLASS0_NARROW_WAVES : 1)))
k_eval_class(EvalArgs a) {
  constexpr int S = class_stack(CLS);
  constexpr int K = class_k(CLS, KV);
  extern __shared__ float xtile[];
  // the claimed item passes through the tiles' LDS (no tile is in use
  // between items)
  long long* s_item = reinterpret_cast<long long*>(xtile);
  const int32_t count = a.class_count[CLS];
  const int64_t items = int64_t(count) * a.n_chunks;
  const int32_t* list = a.class_list + int64_t(CLS) * a.n_total;
  // workgroups beyond the item count leave at once: on a short (or empty)
  // list, one same-address atomic per workgroup of the persistent grid
  // would serialise at the counter for longer than the work takes
  if (int64_t(blockIdx.x) >= items) return;
  for (;;) {
    if (threadIdx.x == 0) *s_item = (long long)atomicAdd(a.work + CLS, 1ull);
    __syncthreads();
    const int64_t it = *s_item;
    __syncthreads();
    if (it >= items) break;  // uniform across the workgroup
    const int c = int(it / count);
    const int p = list[it % count] - a.prog_begin;
    if (p < 0 || p >= a.n_programs) continue;  // a program of another slice
    eval_block<KIND, K, S>(a, p, c, xtile);
  }
}

// Small case sets (one chunk of at most RESIDENT_MAX_BYTES of inputs): every
// workgroup copies the whole input set into LDS once, laid out per pass of
// 64 K cases as the block kernel lays out a tile ([pass][variable][64 K]),
// and each wave then takes whole programs of register-need class 0 from the
// list and runs every pass, so that nothing is staged per program, no case
// is padding beyond the last pass and no workgroup barrier is taken per
// program.  A lane adds its cases in the order it would with either tile
// width, so the width changes no result bit here either.
template <int KIND, int K, int CLS>
__device__ __forceinline__ void eval_wave_resident(const EvalArgs& a, int p, const float* xres, int passes) {
  constexpr int K64 = K * 64;
  const ProgMeta m = a.meta[p];
  const int lane = threadIdx.x & 63;
  const int64_t off = a.tok_offset[p];
  const uint32_t* code = a.code + off;
  const float* cval = a.cval + off;
  const int L = m.len;
  const uint32_t vc0 = lane < L ? code[lane] : 0u;
  const float vv0 = lane < L ? cval[lane] : 0.0f;
  const uint32_t vc1 = lane + 64 < L ? code[lane + 64] : 0u;
  const float vv1 = lane + 64 < L ? cval[lane + 64] : 0.0f;
  constexpr bool SHIFTED = KIND == BEAGLE_FIT_CORR || KIND == BEAGLE_FIT_R4;
  double shift = double(m.shift);
  const double ybar = SHIFTED ? a.stats[0] : 0.0;
  const double smax = a.smax, s11 = a.smax / 11.0;
  Acc<KIND> acc;
  for (int ps = 0; ps < passes; ++ps) {
    const int64_t base = int64_t(ps) * K64;
    float yk[K];
#pragma unroll
    for (int g = 0; g < K / 4; ++g) {
      const float4 q = *reinterpret_cast<const float4*>(a.yp + base + g * 256 + 4 * lane);
      yk[4 * g + 0] = q.x;
      yk[4 * g + 1] = q.y;
      yk[4 * g + 2] = q.z;
      yk[4 * g + 3] = q.w;
    }
    float top[K];
    if constexpr (CLS == 0)
      interpret_small<K>(vc0, vv0, vc1, vv1, code, cval, L, lane, xres + ps * (a.D * K64) + 4 * lane, top);
    else
      interpret<K, class_stack(CLS)>(vc0, vv0, vc1, vv1, code, cval, L, lane, xres + ps * (a.D * K64) + 4 * lane, top);
    if (SHIFTED && ps == 0 && a.meta_shift) {
      // the shift is the output at case 0 (lane 0, first case) when finite:
      // the value the shift pass computes, from the same arithmetic
      const float y0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(top[0]), 0));
      const float sh = isfinite(y0) ? y0 : 0.0f;
      if (lane == 0) a.meta_shift[p].shift = sh;
      shift = double(sh);
    }
    if (base + K64 <= a.M) {
#pragma unroll
      for (int k = 0; k < K; ++k) acc.add(top[k], yk[k], true, shift, ybar, smax, s11);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool valid = base + (k / 4) * 256 + 4 * lane + (k % 4) < a.M;
        acc.add(top[k], yk[k], valid, shift, ybar, smax, s11);
      }
    }
  }
  double v[MAX_SUMS];
  acc.wave_sums(v);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kind_sums(KIND); ++j) a.part[int64_t(j) * a.n_programs + p] = v[j];
  }
}

template <int KIND, int K, int CLS>
__global__ void __launch_bounds__(256) k_eval_resident(EvalArgs a) {
  constexpr int K64 = K * 64;
  extern __shared__ float xres[];
  // A list of at most four programs per wave is walked statically (wave w
  // takes programs w, w + W, ...: no atomics); a longer one through the
  // shared counter, RESIDENT_BATCH programs per claim.  Workgroups whose
  // waves would find nothing leave before staging the inputs.
  const int32_t n_list = a.class_count[CLS];
  const int32_t n_waves = int32_t(gridDim.x) * 4;
  if (int64_t(blockIdx.x) * 4 >= n_list) return;
  const int passes = int((a.M + K64 - 1) / K64);
  const int per_pass = a.D * K64;
  for (int i = threadIdx.x; i < passes * per_pass; i += blockDim.x) {
    const int ps = i / per_pass, r = i - ps * per_pass, d = r / K64, j = r - d * K64;
    xres[i] = a.Xt[int64_t(d) * a.Mp + int64_t(ps) * K64 + j];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // The wave's loop must stay free of divergent branches: a lane-0-only
  // branch around the atomic lets the compiler restructure the loop so that
  // after the first program only lane 0 goes back to the atomic while the
  // other lanes re-run the old item forever.  So every lane takes part in
  // the atomic (lane 0 adds 1, the others 0: one atomic after the wave
  // reduction), the item is read from lane 0 explicitly, the count is a
  // scalar and no early continue splits the body.
  // Each atomic claims RESIDENT_BATCH consecutive programs (one
  // same-address atomic per program would serialise at the counter).
  const int32_t count = __builtin_amdgcn_readfirstlane(a.class_count[CLS]);
  const int32_t* list = a.class_list + int64_t(CLS) * a.n_total;
  // Both walks in one loop around one call of the per-program routine (two
  // inlined copies of the interpreter would not fit the instruction cache
  // together): the static walk steps by the wave count from the wave's
  // index; the claimed walk steps by one through each claimed batch and
  // claims the next one at its end.  Every value deciding a branch is
  // wave-uniform, so the atomic runs on all lanes.
  const bool claimed = count > 4 * n_waves;
  const int32_t wave_id = __builtin_amdgcn_readfirstlane(int32_t(blockIdx.x) * 4 + int32_t(threadIdx.x >> 6));
  int64_t item = claimed ? 0 : wave_id;
  int64_t end = claimed ? 0 : count;  // the walk's current range [item, end)
  const int64_t step = claimed ? 1 : n_waves;
  for (;;) {
    if (item >= end) {
      if (!claimed) break;
      const unsigned long long it = atomicAdd(a.work + CLS, lane == 0 ? (unsigned long long)RESIDENT_BATCH : 0ull);
      const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(it), 0);
      const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(it >> 32), 0);
      const int64_t first = int64_t((uint64_t(hi) << 32) | lo);
      if (first >= count) break;
      item = first;
      end = first + RESIDENT_BATCH < count ? first + RESIDENT_BATCH : count;
    }
    const int p = __builtin_amdgcn_readfirstlane(list[item] - a.prog_begin);
    if (p >= 0 && p < a.n_programs) eval_wave_resident<KIND, K, CLS>(a, p, xres, passes);  // else another slice's
    item += step;
  }
}

// One work list of a batched evaluation (list vl: a work list of the
// class and tile variant, for one bucket of variable counts): the same
// persistent scheme over the (problem, chunk, program) items of the table's
// problems in that list, problem by problem in table order and chunk-major
// within a problem.  Items are claimed in increasing order, so a
// workgroup's next item lies in its previous item's problem or a later one:
// the problem is found by stepping forward from there when it is near, by
// bisection otherwise.
template <int KIND, int CLS, int KV>
__global__ void __launch_bounds__(256) k_eval_batch(BatchArgs b, int vl) {
  constexpr int S = class_stack(CLS);
  constexpr int K = class_k(CLS, KV);
  extern __shared__ float xtile[];
  long long* s_item = reinterpret_cast<long long*>(xtile);  // (as in k_eval_class)
  const int64_t* off = b.item_off + int64_t(vl) * (b.n_problems + 1);
  const int64_t items = off[b.n_problems];
  if (int64_t(blockIdx.x) >= items) return;  // (as in k_eval_class)
  int lo = 0;  // the problem of the previous item (a lower bound for the next)
  for (;;) {
    if (threadIdx.x == 0) *s_item = (long long)atomicAdd(b.work + vl, 1ull);
    __syncthreads();
    const uint64_t raw = uint64_t(*s_item);
    __syncthreads();
    const int64_t it = int64_t((uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(raw >> 32)))) << 32) |
                               uint32_t(__builtin_amdgcn_readfirstlane(int(raw))));
    if (it >= items) break;  // uniform across the workgroup
    // the last problem q >= lo with off[q] <= it (problems without items in
    // this list have empty ranges and are stepped over)
    int steps = 0;
    while (steps < 4 && lo + 1 < b.n_problems && off[lo + 1] <= it) {
      ++lo;
      ++steps;
    }
    if (steps == 4) {
      int hi = b.n_problems;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= it)
          lo = mid;
        else
          hi = mid;
      }
    }
    const BatchProblem& P = b.table[lo];
    const int32_t count = P.prep.class_count[CLS];
    const int64_t local = it - off[lo];
    const int c = int(local / count);
    const int p = P.prep.class_list[int64_t(CLS) * P.prep.n_programs + local % count];
    EvalArgs a;
    a.code = P.prep.code;
    a.cval = P.prep.cval;
    a.tok_offset = P.prep.tok_offset;
    a.meta = P.prep.meta;
    a.Xt = P.Xt;
    a.yp = P.yp;
    a.M = P.M;
    a.Mp = P.Mp;
    a.D = P.prep.D;
    a.n_programs = P.prep.n_programs;
    a.n_chunks = P.n_chunks;
    a.chunk = P.chunk;
    a.part = P.part;
    a.stats = P.stats;
    a.class_count = nullptr;
    a.class_list = nullptr;
    a.work = nullptr;
    a.n_total = P.prep.n_programs;
    a.prog_begin = 0;
    eval_block<KIND, K, S>(a, p, c, xtile);
  }
}

// Per-case outputs of every program on cases [0, m): one wave per
// (program, 64 cases).  In shift mode (m = 1) it stores the output at case
// 0 as the program's shift for correlation sums.
__device__ static void values_program(const ValuesArgs& a, int p, int64_t tile, float* xl_all) {
  const int lane = threadIdx.x;
  const int64_t i = tile * 64 + lane;
  const ProgMeta m = a.meta[p];
  if (m.status != BEAGLE_PROG_OK) {
    if (!a.shift_mode && i < a.m) a.out[int64_t(p) * a.m + i] = __int_as_float(0x7FC00000);
    return;
  }
  const int64_t off = a.tok_offset[p];
  const uint32_t* code = a.code + off;
  const float* cval = a.cval + off;
  const int L = m.len;
  const uint32_t vc0 = lane < L ? code[lane] : 0u;
  const float vv0 = lane < L ? cval[lane] : 0.0f;
  const uint32_t vc1 = lane + 64 < L ? code[lane + 64] : 0u;
  const float vv1 = lane + 64 < L ? cval[lane + 64] : 0.0f;
  const int64_t ii = i < a.m ? i : 0;
  float* xl = xl_all + lane * 4;
  for (int d = 0; d < a.D; ++d) xl[d * 256] = a.Xt[int64_t(d) * a.Mp + ii];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);
  float top[1];
  interpret<1, MAX_STACK>(vc0, vv0, vc1, vv1, code, cval, L, lane, xl, top);
  if (a.shift_mode) {
    // a finite shift (a non-finite output at case 0 is either the whole
    // fitness, NaN, or an invalid pair of the paper's scores)
    if (tile == 0 && lane == 0) a.meta[p].shift = isfinite(top[0]) ? top[0] : 0.0f;
  } else if (i < a.m) {
    a.out[int64_t(p) * a.m + i] = top[0];
  }
}

// (dynamic LDS: D * 256 floats, so that more waves fit per CU for small D)
__global__ void __launch_bounds__(64) k_values(ValuesArgs a) {
  extern __shared__ float xl_all[];
  values_program(a, blockIdx.x, blockIdx.y, xl_all);
}

// Correlation shifts of the class-2 programs only (the resident-inputs
// kernels compute those of classes 0 and 1): a fixed grid striding over the
// list, no counters.
__global__ void __launch_bounds__(64) k_values_deep(ValuesArgs a, const int32_t* class_count,
                                                    const int32_t* class_list, int32_t stride) {
  extern __shared__ float xl_all[];  // D * 256 floats
  const int32_t c2 = class_count[2];
  for (int32_t item = blockIdx.x; item < c2; item += gridDim.x) {
    values_program(a, class_list[2 * int64_t(stride) + item], 0, xl_all);
    __builtin_amdgcn_wave_barrier();
  }
}

// Correlation shifts of every program of the table (one wave per program).
__global__ void __launch_bounds__(64) k_values_batch(BatchArgs b) {
  __shared__ float xl_all[MAX_D * 256];
  const int64_t g = blockIdx.x;
  const int q = batch_find(b, g, [](const BatchProblem& t) { return t.prog_begin; });
  const BatchProblem& P = b.table[q];
  ValuesArgs a;
  a.code = P.prep.code;
  a.cval = P.prep.cval;
  a.tok_offset = P.prep.tok_offset;
  a.meta = P.prep.meta;
  a.Xt = P.Xt;
  a.Mp = P.Mp;
  a.m = 1;
  a.D = P.prep.D;
  a.n_programs = P.prep.n_programs;
  a.out = nullptr;
  a.shift_mode = 1;
  values_program(a, int(g - P.prog_begin), 0, xl_all);
}

// Fitness of every program from its chunk partials, summed in chunk order.
__device__ static void finalize_program(const FinalizeArgs& a, int p) {
  const ProgMeta m = a.meta[p];
  const double nan = __longlong_as_double(0x7FF8000000000000LL);
  double F;
  if (m.status != BEAGLE_PROG_OK) {
    F = nan;
  } else if (a.kind == BEAGLE_FIT_MSE) {
    double s = 0.0;
    for (int c = 0; c < a.n_chunks; ++c) s += a.part[int64_t(c) * a.n_programs + p];
    F = s / double(a.M);
  } else if (a.kind == BEAGLE_FIT_POINT) {
    double s = 0.0;
    for (int c = 0; c < a.n_chunks; ++c) s += a.part[int64_t(c) * a.n_programs + p];
    F = s;
  } else if (a.kind == BEAGLE_FIT_R4) {
    double s[7];
    for (int j = 0; j < 7; ++j) {
      s[j] = 0.0;
      for (int c = 0; c < a.n_chunks; ++c) s[j] += a.part[(int64_t(j) * a.n_chunks + c) * a.n_programs + p];
    }
    const double c1 = s[0], c2 = s[1], n = double(a.M) - c1 - c2;
    double r = 0.0;
    if (n >= 2.0) {
      const double sxx = s[3] - s[2] * s[2] / n;
      const double syy = s[6] - s[5] * s[5] / n;
      const double sxy = s[4] - s[2] * s[5] / n;
      if (sxx > 0.0 && syy > 0.0) r = sxy / sqrt(sxx * syy);
    }
    const double r2 = r * r;
    F = a.smax * (r2 * r2) * n - a.smax * (c1 - c2);
  } else {
    double s[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < a.n_chunks; ++c) s[j] += a.part[(int64_t(j) * a.n_chunks + c) * a.n_programs + p];
    const double Md = double(a.M);
    const double syy = a.stats[2], sw = a.stats[1];
    // gradient seed (1 - r^2 differentiated, unclamped; zero for a constant
    // output, NaN for a NaN fitness): with u = yhat - shift and w = y - ybar,
    // Sxx = sum u^2 - (sum u)^2 / M, Sxy = sum u w - sum u sum w / M, so
    // dSxx/dyhat_i = 2 (yhat_i - mu), dSxy/dyhat_i = w_i - mean w and
    // dF/dyhat_i = -2 r (dSxy/dyhat_i / sqrt(Sxx Syy) - r (yhat_i - mu) / Sxx)
    double alpha = nan, beta = nan, mu = nan;
    if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2])) {
      F = nan;
    } else if (!(syy > 0.0)) {
      F = nan;
    } else {
      const double sxx = s[1] - s[0] * s[0] / Md;
      const double sxy = s[2] - s[0] * sw / Md;
      mu = double(m.shift) + s[0] / Md;
      if (!(sxx > 0.0)) {
        F = 1.0;
        alpha = beta = 0.0;
      } else {
        const double q = sqrt(sxx * syy);
        const double r = sxy / q;
        F = 1.0 - r * r;
        F = F < 0.0 ? 0.0 : (F > 1.0 ? 1.0 : F);
        alpha = -2.0 * r / q;
        beta = 2.0 * r * r / sxx;
      }
    }
    if (a.coef) {
      a.coef[3 * int64_t(p)] = alpha;
      a.coef[3 * int64_t(p) + 1] = beta;
      a.coef[3 * int64_t(p) + 2] = mu;
    }
  }
  a.fitness[p] = F;
}

__global__ void k_finalize(FinalizeArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < a.n_programs) finalize_program(a, p);
}

// One thread per program of every problem of the table.
__global__ void k_finalize_batch(BatchArgs b) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= b.n_programs) return;
  const int q = batch_find(b, g, [](const BatchProblem& t) { return t.prog_begin; });
  const BatchProblem& P = b.table[q];
  FinalizeArgs a;
  a.meta = P.prep.meta;
  a.part = P.part;
  a.stats = P.stats;
  a.M = P.M;
  a.n_programs = P.prep.n_programs;
  a.n_chunks = P.n_chunks;
  a.kind = b.kind;
  a.fitness = P.fitness;
  a.coef = nullptr;
  finalize_program(a, int(g - P.prog_begin));
}

// First work item of every problem in each work list (exclusive prefix sums
// in table order), from the class counts that k_prepare_batch produced.
__global__ void k_batch_items(BatchArgs b) {
  const int vl = threadIdx.x;  // list v, bucket db
  if (vl >= N_BATCH_LISTS) return;
  const int v = vl / N_DBUCKETS, db = vl % N_DBUCKETS;
  const int cls = v == 0 ? 0 : v - 1;
  int64_t* off = b.item_off + int64_t(vl) * (b.n_problems + 1);
  int64_t acc = 0;
  for (int q = 0; q < b.n_problems; ++q) {
    off[q] = acc;
    const BatchProblem& P = b.table[q];
    if ((v >= 2 || P.kv == v) && d_bucket(P.prep.D) == db) acc += int64_t(P.prep.class_count[cls]) * P.n_chunks;
  }
  off[b.n_problems] = acc;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// resident workgroups per CU of a class kernel at a given LDS size
template <int KIND, int CLS, int KV>
static int resident_blocks(size_t lds) {
  static size_t cached_lds = size_t(-1);
  static int cached = 0;
  if (lds != cached_lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_class<KIND, CLS, KV>, 256, lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    cached = nb;
    cached_lds = lds;
  }
  return cached;
}

static int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 1;
  }
  return n;
}

template <int KIND, int CLS, int KV>
static hipError_t launch_class(const EvalArgs& a, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  const size_t lds = size_t(EVAL_WAVES) * a.D * ((class_k(CLS, KV) + 3) / 4) * 256 * sizeof(float);
  const int grid = resident_blocks<KIND, CLS, KV>(lds) * cu_count();
  // timing events, when asked for, are taken by the dispatch itself
  if (ev0 || ev1)
    hipExtLaunchKernelGGL((k_eval_class<KIND, CLS, KV>), dim3(grid), dim3(256), uint32_t(lds), s, ev0, ev1, 0u, a);
  else
    hipLaunchKernelGGL((k_eval_class<KIND, CLS, KV>), dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

// input bytes of the resident kernel with K cases per lane (the case set
// padded to whole passes of 64 K cases)
static size_t resident_bytes(const EvalArgs& a, int K) {
  const int64_t k64 = 64 * K;
  return size_t((a.M + k64 - 1) / k64) * size_t(a.D) * size_t(k64) * sizeof(float);
}

// The resident kernel takes the call when there is one chunk, enough programs
// to give every SIMD several waves, and inputs within RESIDENT_MAX_BYTES at
// the wider tile's padding: the choice never depends on the tile width, so
// the tuner's pick cannot switch kernels (and summation orders).
bool resident_eligible(int64_t M, int32_t D, int32_t n_chunks, int32_t n_total) {
  const size_t b8 = size_t((M + 511) / 512) * size_t(D) * 512u * sizeof(float);
  return n_chunks == 1 && n_total >= RESIDENT_MIN_PROGRAMS && b8 <= RESIDENT_MAX_BYTES;
}

static bool resident_eligible(const EvalArgs& a) { return resident_eligible(a.M, a.D, a.n_chunks, a.n_total); }

template <int KIND, int K, int CLS>
static hipError_t launch_resident(const EvalArgs& a, size_t lds, hipStream_t s, hipEvent_t ev0 = nullptr,
                                  hipEvent_t ev1 = nullptr) {
  static size_t cached_lds = size_t(-1);
  static int cached = 0;
  if (lds != cached_lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_resident<KIND, K, CLS>, 256, lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    cached = nb;
    cached_lds = lds;
  }
  if (ev0 || ev1)
    hipExtLaunchKernelGGL((k_eval_resident<KIND, K, CLS>), dim3(cached * cu_count()), dim3(256), uint32_t(lds), s,
                          ev0, ev1, 0u, a);
  else
    hipLaunchKernelGGL((k_eval_resident<KIND, K, CLS>), dim3(cached * cu_count()), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_kind(int kv, const EvalArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                              bool counters_clear) {
  if (!counters_clear) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, a.work, N_CLASSES);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool wide = kv == 0 && a.D <= WIDE_TILE_MAX_D;
  const bool resident = resident_eligible(a);
  if (resident)
    e = wide ? launch_resident<KIND, 8, 0>(a, resident_bytes(a, 8), s, ev0, ev1)
             : launch_resident<KIND, 4, 0>(a, resident_bytes(a, 4), s, ev0, ev1);
  else
    e = wide ? launch_class<KIND, 0, 0>(a, s, ev0, ev1) : launch_class<KIND, 0, 1>(a, s, ev0, ev1);
  if (e != hipSuccess) return e;
  // class 1 (register need 5..8, and every program with one of the further
  // operators) resident too when the shape allows, 4 cases per lane
  e = resident ? launch_resident<KIND, 4, 1>(a, resident_bytes(a, 4), s) : launch_class<KIND, 1, 0>(a, s);
  if (e != hipSuccess) return e;
  return launch_class<KIND, 2, 0>(a, s);
}

hipError_t launch_eval(int kind, int kv, const EvalArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                       bool counters_clear) {
  switch (kind) {
    case BEAGLE_FIT_MSE:
      return launch_kind<BEAGLE_FIT_MSE>(kv, a, s, ev0, ev1, counters_clear);
    case BEAGLE_FIT_CORR:
      return launch_kind<BEAGLE_FIT_CORR>(kv, a, s, ev0, ev1, counters_clear);
    case BEAGLE_FIT_POINT:
      return launch_kind<BEAGLE_FIT_POINT>(kv, a, s, ev0, ev1, counters_clear);
    default:
      return launch_kind<BEAGLE_FIT_R4>(kv, a, s, ev0, ev1, counters_clear);
  }
}

// Persistent grid of a work-list kernel: resident workgroups per CU at the
// list's LDS tile size, times the CUs (cached per largest D, 1..MAX_D, so
// that the occupancy queries all happen before a graph capture).
template <int KIND, int CLS, int KV>
static int list_grid(int max_d) {
  static int cached[MAX_D + 1] = {0};
  const int d = max_d < 1 ? 1 : (max_d > MAX_D ? MAX_D : max_d);
  if (cached[d] == 0) {
    const size_t lds = size_t(EVAL_WAVES) * d * ((class_k(CLS, KV) + 3) / 4) * 256 * sizeof(float);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_batch<KIND, CLS, KV>, 256, lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    cached[d] = nb * cu_count();
  }
  return cached[d];
}

template <int KIND, int CLS, int KV>
static hipError_t launch_list(const BatchArgs& b, int vl, int max_d, hipStream_t s) {
  const size_t lds = size_t(EVAL_WAVES) * max_d * ((class_k(CLS, KV) + 3) / 4) * 256 * sizeof(float);
  hipLaunchKernelGGL((k_eval_batch<KIND, CLS, KV>), dim3(list_grid<KIND, CLS, KV>(max_d)), dim3(256), lds, s, b, vl);
  return hipGetLastError();
}

// every bucket of list v (its lists are v * N_DBUCKETS + bucket)
template <int KIND, int CLS, int KV>
static hipError_t launch_buckets(const BatchArgs& b, int v, const int* max_d, const int* has, hipStream_t s) {
  for (int db = 0; db < N_DBUCKETS; ++db) {
    const int vl = v * N_DBUCKETS + db;
    if (!has[vl]) continue;
    const hipError_t e = launch_list<KIND, CLS, KV>(b, vl, max_d[vl], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int KIND, int CLS, int KV>
static void prime_buckets(int v, const int* max_d, const int* has) {
  for (int db = 0; db < N_DBUCKETS; ++db)
    if (has[v * N_DBUCKETS + db]) (void)list_grid<KIND, CLS, KV>(max_d[v * N_DBUCKETS + db]);
}

template <int KIND>
static void prime_kind(const int* max_d, const int* has) {
  prime_buckets<KIND, 0, 0>(0, max_d, has);
  prime_buckets<KIND, 0, 1>(1, max_d, has);
  prime_buckets<KIND, 1, 0>(2, max_d, has);
  prime_buckets<KIND, 2, 0>(3, max_d, has);
}

void prime_eval_batch(int kind, const int* max_d, const int* has_items) {
  if (kind == BEAGLE_FIT_MSE)
    prime_kind<BEAGLE_FIT_MSE>(max_d, has_items);
  else
    prime_kind<BEAGLE_FIT_CORR>(max_d, has_items);
}

template <int KIND>
static hipError_t launch_batch_kind(const BatchArgs& b, const int* max_d, const int* has, hipStream_t s,
                                    hipEvent_t ev0, hipEvent_t ev1) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, b.work, N_BATCH_LISTS);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev0) (void)hipEventRecord(ev0, s);
  if ((e = launch_buckets<KIND, 0, 0>(b, 0, max_d, has, s)) != hipSuccess) return e;
  if ((e = launch_buckets<KIND, 0, 1>(b, 1, max_d, has, s)) != hipSuccess) return e;
  if (ev1) (void)hipEventRecord(ev1, s);
  if ((e = launch_buckets<KIND, 1, 0>(b, 2, max_d, has, s)) != hipSuccess) return e;
  if ((e = launch_buckets<KIND, 2, 0>(b, 3, max_d, has, s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_eval_batch(int kind, const BatchArgs& b, const int* max_d, const int* has_items, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1) {
  return kind == BEAGLE_FIT_MSE ? launch_batch_kind<BEAGLE_FIT_MSE>(b, max_d, has_items, s, ev0, ev1)
                                : launch_batch_kind<BEAGLE_FIT_CORR>(b, max_d, has_items, s, ev0, ev1);
}

}  // namespace bgl
