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
#include <cmath>

#include "beagle_device.h"
#include "kernels.h"

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

// K consecutive floats read as one LDS access.
template <int K>
struct alignas(4 * K) Vec {
  float v[K];
};

// The stack interpreter for one program on K cases per lane.
//   vc0/vv0, vc1/vv1: instruction words / constant values of tokens 0..63
//   and 64..127 (one per lane); longer programs read later tokens from
//   memory.  xl points at this lane's inputs in the wave's LDS tile:
//   variable d of case k is xl[d * 64 * K + k].
template <int K, int S>
__device__ __forceinline__ void interpret(uint32_t vc0, float vv0, uint32_t vc1, float vv1,
                                          const uint32_t* __restrict__ code, const float* __restrict__ cval,
                                          int L, int lane, const float* xl, float (&top)[K]) {
  float stk[K][S - 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    top[k] = 0.0f;
#pragma unroll
    for (int j = 0; j < S - 1; ++j) stk[k][j] = 0.0f;
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
    const int n = L - base < 64 ? L - base : 64;
    for (int t = 0; t < n; ++t) {
      const uint32_t w = __builtin_amdgcn_readlane(vc, t);
      const uint32_t arg = w >> 8;
      switch (w & 0xFFu) {
#define BGL_PUSH_VAR(N)                                                        \
  case H_VAR + N:                                                              \
    if constexpr (N < S) {                                                     \
      if constexpr (N > 0) {                                                   \
        _Pragma("unroll") for (int k = 0; k < K; ++k) stk[k][N > 0 ? N - 1 : 0] = top[k]; \
      }                                                                        \
      const Vec<K> xv = *reinterpret_cast<const Vec<K>*>(xl + arg * (64 * K)); \
      _Pragma("unroll") for (int k = 0; k < K; ++k) top[k] = xv.v[k];          \
    }                                                                          \
    break;
#define BGL_PUSH_CONST(N)                                                      \
  case H_CONST + N:                                                            \
    if constexpr (N < S) {                                                     \
      if constexpr (N > 0) {                                                   \
        _Pragma("unroll") for (int k = 0; k < K; ++k) stk[k][N > 0 ? N - 1 : 0] = top[k]; \
      }                                                                        \
      const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t)); \
      _Pragma("unroll") for (int k = 0; k < K; ++k) top[k] = v;                \
    }                                                                          \
    break;
#define BGL_BIN(O, N)                                                          \
  case H_BIN + 15 * O + (N - 2):                                               \
    if constexpr (N <= S) {                                                    \
      _Pragma("unroll") for (int k = 0; k < K; ++k) top[k] =                   \
          binop<O>(stk[k][N <= S ? N - 2 : 0], top[k]);                        \
    }                                                                          \
    break;
#define BGL_BIN_ALL(O)                                                          \
  BGL_BIN(O, 2) BGL_BIN(O, 3) BGL_BIN(O, 4) BGL_BIN(O, 5) BGL_BIN(O, 6) BGL_BIN(O, 7) \
  BGL_BIN(O, 8) BGL_BIN(O, 9) BGL_BIN(O, 10) BGL_BIN(O, 11) BGL_BIN(O, 12)     \
  BGL_BIN(O, 13) BGL_BIN(O, 14) BGL_BIN(O, 15) BGL_BIN(O, 16)
#define BGL_PUSH_ALL(M)                                                         \
  M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15)
        BGL_PUSH_ALL(BGL_PUSH_VAR)
        BGL_PUSH_ALL(BGL_PUSH_CONST)
        BGL_BIN_ALL(B_ADD)
        BGL_BIN_ALL(B_SUB)
        BGL_BIN_ALL(B_MUL)
        BGL_BIN_ALL(B_DIV)
        BGL_BIN_ALL(B_RSUB)
        BGL_BIN_ALL(B_RDIV)
#undef BGL_PUSH_VAR
#undef BGL_PUSH_CONST
#undef BGL_BIN
#undef BGL_BIN_ALL
#undef BGL_PUSH_ALL
        case H_UN + 0:
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = sinf(top[k]);
          break;
        case H_UN + 1:
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = cosf(top[k]);
          break;
        case H_UN + 2:
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = op_exp(top[k]);
          break;
        case H_UN + 3:
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = op_log(top[k]);
          break;
        case H_UN + 4:
#pragma unroll
          for (int k = 0; k < K; ++k) top[k] = op_sqrt(top[k]);
          break;
        default:
          break;
      }
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// One workgroup: program p on case chunk c.  Writes the chunk's partial sums
//   MSE : part[0][c][p] = sum (yhat - y)^2
//   CORR: part[j][c][p] = sum u, sum u^2, sum u*w   (u = yhat - shift_p,
//         w = y - ybar), all in binary64.
template <int KIND, int K, int S>
__device__ __forceinline__ void eval_block(const EvalArgs& a, int p, int c, double* red, float* xtile) {
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
  const double ybar = KIND == BEAGLE_FIT_CORR ? a.stats[0] : 0.0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const int64_t c0 = int64_t(c) * a.chunk;
  const int64_t c1 = c0 + a.chunk < a.M ? c0 + a.chunk : a.M;
  // this wave's input tile: [d][lane][k], K consecutive cases per lane
  float* xw = xtile + wave * (a.D * 64 * K);
  float* xl = xw + lane * K;
  for (int64_t base = c0 + int64_t(wave) * (64 * K); base < c1; base += int64_t(EVAL_WAVES) * 64 * K) {
    float yk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) yk[k] = a.yp[base + k * 64 + lane];
    // coalesced global reads (case = base + k*64 + lane), one LDS write per
    // variable; the wave's tile is private to it, so a wave barrier suffices
    for (int d = 0; d < a.D; ++d) {
      Vec<K> xv;
#pragma unroll
      for (int k = 0; k < K; ++k) xv.v[k] = a.Xt[int64_t(d) * a.Mp + base + k * 64 + lane];
      __builtin_amdgcn_wave_barrier();
      *reinterpret_cast<Vec<K>*>(xl + d * (64 * K)) = xv;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the tile is in LDS
    float top[K];
    interpret<K, S>(vc0, vv0, vc1, vv1, code, cval, L, lane, xl, top);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool valid = base + k * 64 + lane < a.M;
      if constexpr (KIND == BEAGLE_FIT_MSE) {
        const double d = double(top[k]) - double(yk[k]);
        s0 += valid ? d * d : 0.0;
      } else {
        const double u = valid ? double(top[k]) - shift : 0.0;
        const double w = valid ? double(yk[k]) - ybar : 0.0;
        s0 += u;
        s1 += u * u;
        s2 += u * w;
      }
    }
  }
  constexpr int NS = KIND == BEAGLE_FIT_MSE ? 1 : 3;
  s0 = wave_sum(s0);
  if constexpr (NS == 3) {
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
  }
  if (lane == 0) {
    red[wave * 3 + 0] = s0;
    red[wave * 3 + 1] = s1;
    red[wave * 3 + 2] = s2;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    const int j = threadIdx.x;
    const double t = ((red[j] + red[3 + j]) + red[6 + j]) + red[9 + j];
    a.part[(int64_t(j) * a.n_chunks + c) * a.n_programs + p] = t;
  }
  __syncthreads();
}

template <int KIND>
__global__ void __launch_bounds__(256) k_eval_fast(EvalArgs a) {
  __shared__ double red[12];
  extern __shared__ float xtile[];
  const int p = int(blockIdx.x % uint32_t(a.n_programs));
  const int c = int(blockIdx.x / uint32_t(a.n_programs));
  const ProgMeta m = a.meta[p];
  if (m.status != BEAGLE_PROG_OK || m.need > FAST_STACK) return;
  eval_block<KIND, EVAL_K, FAST_STACK>(a, p, c, red, xtile);
}

// Programs whose register need exceeds FAST_STACK (long, bushy trees): a
// grid-stride loop over (program, chunk) pairs of the list built by the
// preparation kernel; an empty list makes every workgroup exit at once.
template <int KIND>
__global__ void __launch_bounds__(256) k_eval_deep(EvalArgs a) {
  __shared__ double red[12];
  extern __shared__ float xtile[];
  const int64_t items = int64_t(*a.deep_count) * a.n_chunks;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int p = a.deep_list[it / a.n_chunks] - a.prog_begin;
    const int c = int(it % a.n_chunks);
    if (p < 0 || p >= a.n_programs) continue;  // another slice's program (uniform)
    eval_block<KIND, DEEP_K, MAX_STACK>(a, p, c, red, xtile);
  }
}

// Per-case outputs of every program on cases [0, m): one wave per
// (program, 64 cases).  In shift mode (m = 1) it stores the output at case
// 0 as the program's shift for correlation sums.
__global__ void __launch_bounds__(64) k_values(ValuesArgs a) {
  __shared__ float xl_all[MAX_D * 64];
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t i = int64_t(blockIdx.y) * 64 + lane;
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
  float* xl = xl_all + lane;
  for (int d = 0; d < a.D; ++d) xl[d * 64] = a.Xt[int64_t(d) * a.Mp + ii];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);
  float top[1];
  interpret<1, MAX_STACK>(vc0, vv0, vc1, vv1, code, cval, L, lane, xl, top);
  if (a.shift_mode) {
    if (blockIdx.y == 0 && lane == 0) a.meta[p].shift = top[0];
  } else if (i < a.m) {
    a.out[int64_t(p) * a.m + i] = top[0];
  }
}

// Fitness of every program from its chunk partials, summed in chunk order.
__global__ void k_finalize(FinalizeArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_programs) return;
  const ProgMeta m = a.meta[p];
  const double nan = __longlong_as_double(0x7FF8000000000000LL);
  double F;
  if (m.status != BEAGLE_PROG_OK) {
    F = nan;
  } else if (a.kind == BEAGLE_FIT_MSE) {
    double s = 0.0;
    for (int c = 0; c < a.n_chunks; ++c) s += a.part[int64_t(c) * a.n_programs + p];
    F = s / double(a.M);
  } else {
    double s[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < a.n_chunks; ++c) s[j] += a.part[(int64_t(j) * a.n_chunks + c) * a.n_programs + p];
    const double Md = double(a.M);
    const double syy = a.stats[2], sw = a.stats[1];
    if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2])) {
      F = nan;
    } else if (!(syy > 0.0)) {
      F = nan;
    } else {
      const double sxx = s[1] - s[0] * s[0] / Md;
      const double sxy = s[2] - s[0] * sw / Md;
      if (!(sxx > 0.0)) {
        F = 1.0;
      } else {
        const double r = sxy / sqrt(sxx * syy);
        F = 1.0 - r * r;
        F = F < 0.0 ? 0.0 : (F > 1.0 ? 1.0 : F);
      }
    }
  }
  a.fitness[p] = F;
}

template <int KIND>
static hipError_t launch_kind(const EvalArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 grid(uint32_t(a.n_programs) * uint32_t(a.n_chunks));
  const size_t lds_fast = size_t(EVAL_WAVES) * a.D * 64 * EVAL_K * sizeof(float);
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL((k_eval_fast<KIND>), grid, dim3(256), lds_fast, s, a);
  if (ev1) (void)hipEventRecord(ev1, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds_deep = size_t(EVAL_WAVES) * a.D * 64 * DEEP_K * sizeof(float);
  hipLaunchKernelGGL((k_eval_deep<KIND>), dim3(512), dim3(256), lds_deep, s, a);
  return hipGetLastError();
}

hipError_t launch_eval(int kind, const EvalArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  return kind == BEAGLE_FIT_MSE ? launch_kind<BEAGLE_FIT_MSE>(a, s, ev0, ev1)
                                : launch_kind<BEAGLE_FIT_CORR>(a, s, ev0, ev1);
}

}  // namespace bgl
