// Reverse-mode gradient of the MSE fitness with respect to every program's
// constants (not in the paper: an adjoint over the postfix tape so that a
// program's ephemeral constants can be tuned by gradient steps).
//
// One wave evaluates one program on one chunk of cases, one case per lane.
// Per 64-case tile:
//  forward  the decoded words run as in the evaluator and every word's
//           output is stored in a tape (a register array indexed by the
//           wave-uniform word position for programs of <= 64 decoded words,
//           a per-wave LDS array for <= 256);
//  seed     g = dF/dyhat = 2 (yhat - y) / M for the case (0 for padding);
//  reverse  the words run backwards with an adjoint stack that mirrors the
//           forward stack (adjoint of stack position j in astk[j], the top
//           cached in g).  A binary word at forward stack size n reads its
//           operands from the tape -- the top operand is word t-1's output,
//           the one below it word pa's -- and leaves the left operand's
//           adjoint in astk[n-2] and the right one's in g; a terminal pops
//           (CONST words add g to their slot's gradient); unary and fused
//           words scale g.  Every word writes astk[rws] unconditionally
//           (rws precomputed by the decoder; a dead slot unless the word is
//           binary), so the adjoint stack is updated in place.
// Constant gradients are summed per lane in binary64 (LDS, slots < 8) or per
// wave (slots >= 8), reduced in a fixed order and written as per-chunk
// partials; a finalize kernel sums the chunks in order.
#include "beagle_device.h"
#include "grad.h"
#include "trig.h"

namespace bgl {

constexpr int GRAD_S = MAX_STACK;
constexpr int LANE_SLOTS = 8;  // constant slots accumulated per lane

template <uint32_t O>
__device__ __forceinline__ float gbinop(float a, float b) {
  if constexpr (O == B_ADD) return a + b;
  if constexpr (O == B_SUB) return a - b;
  if constexpr (O == B_MUL) return a * b;
  if constexpr (O == B_DIV) return op_div(a, b);
  if constexpr (O == B_RSUB) return b - a;
  if constexpr (O == B_RDIV) return op_div(b, a);
  return 0.0f;
}

// partial derivatives of binop<O>(A, B): (d/dA, d/dB); 0 where a protected
// division replaces the quotient by 1
template <uint32_t O>
__device__ __forceinline__ void dbinop(float A, float B, float& dA, float& dB) {
  if constexpr (O == B_ADD) { dA = 1.0f; dB = 1.0f; }
  if constexpr (O == B_SUB) { dA = 1.0f; dB = -1.0f; }
  if constexpr (O == B_MUL) { dA = B; dB = A; }
  if constexpr (O == B_DIV) {
    const bool nz = B != 0.0f;
    const float r = 1.0f / (nz ? B : 1.0f);
    dA = nz ? r : 0.0f;
    dB = nz ? -A * r * r : 0.0f;
  }
  if constexpr (O == B_RSUB) { dA = -1.0f; dB = 1.0f; }
  if constexpr (O == B_RDIV) {
    const bool nz = A != 0.0f;
    const float r = 1.0f / (nz ? A : 1.0f);
    dA = nz ? -B * r * r : 0.0f;
    dB = nz ? r : 0.0f;
  }
}

// sin (COS = false) or cos of one value per lane, the interpreter's functions
template <bool COS>
__device__ __forceinline__ float trig1(float x) {
  float v[1] = {x};
  trig_tile<COS, 1>(v);
  return v[0];
}

__device__ __forceinline__ float dunary(uint32_t u, float x, float y) {
  switch (u) {
    case 0: return trig1<true>(x);
    case 1: return -trig1<false>(x);
    case 2: return (x > 80.0f || x < -80.0f) ? 0.0f : y;
    case 3: return x != 0.0f ? 1.0f / x : 0.0f;
    default: return x != 0.0f ? copysignf(0.5f, x) / y : 0.0f;
  }
}

// An opaque copy: keeps two loaded values from being folded into one load
// through a selected address (which would force the arrays out of registers).
__device__ __forceinline__ float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Decoded words of one program: broadcast from VGPRs (short) or read with
// uniform loads (long).
template <bool LONG>
struct Words;

template <>
struct Words<false> {
  uint32_t vc, va;
  float vv;
  __device__ Words(const uint32_t* code, const uint32_t* aux, const float* cval, int L, int lane) {
    vc = lane < L ? code[lane] : 0u;
    va = lane < L ? aux[lane] : 0u;
    vv = lane < L ? cval[lane] : 0.0f;
  }
  __device__ __forceinline__ uint32_t word(int t) const { return __builtin_amdgcn_readlane(vc, t); }
  __device__ __forceinline__ uint32_t auxw(int t) const { return __builtin_amdgcn_readlane(va, t); }
  __device__ __forceinline__ float cv(int t) const {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t));
  }
};

template <>
struct Words<true> {
  const uint32_t* code;
  const uint32_t* aux;
  const float* cval;
  __device__ Words(const uint32_t* c, const uint32_t* a, const float* v, int, int) : code(c), aux(a), cval(v) {}
  __device__ __forceinline__ uint32_t word(int t) const { return __builtin_amdgcn_readfirstlane(code[t]); }
  __device__ __forceinline__ uint32_t auxw(int t) const { return __builtin_amdgcn_readfirstlane(aux[t]); }
  __device__ __forceinline__ float cv(int t) const {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cval[t])));
  }
};

template <bool LONG>
__device__ void grad_item(const GradArgs& a, int p, int c, float* lds) {
  const int lane = threadIdx.x;
  const ProgMeta m = a.meta[p];
  const int L = m.len;
  const int64_t off = a.tok_offset[p];
  const int64_t coff = a.const_offset[p];
  const int cc = a.const_count[p];
  const Words<LONG> W(a.code + off, a.aux + off, a.cval + off, L, lane);
  // LDS: input tile [D][64] | lane gradients [8][64] doubles | wave gradients
  // [256] doubles | (long) tape [256][64]
  float* xl = lds + lane;
  double* lg = reinterpret_cast<double*>(lds + a.D * 64) + lane;
  double* wg = reinterpret_cast<double*>(lds + a.D * 64) + LANE_SLOTS * 64;
  // the tape: two separate 32-entry register arrays for programs of <= 64
  // words (32 dwords is the widest register tuple an index can address),
  // LDS [GRAD_LONG_WORDS][64] for longer ones
  float tape_lo[32], tape_hi[32];
  float* const tape_lds = lds + a.D * 64 + 2 * (LANE_SLOTS * 64 + 256) + lane;
  auto tget = [&](int t) -> float {
    if constexpr (LONG) {
      return tape_lds[t * 64];
    } else {
      const float a = opaque(tape_lo[t & 31]);
      const float b = opaque(tape_hi[t & 31]);
      return t < 32 ? a : b;
    }
  };
  for (int j = 0; j < LANE_SLOTS; ++j) lg[j * 64] = 0.0;
  for (int j = lane; j < 256; j += 64) wg[j] = 0.0;
  __builtin_amdgcn_wave_barrier();
  double s_mse = 0.0;
  const float inv2m = float(2.0 / double(a.M));
  const int64_t c0 = int64_t(c) * a.chunk;
  const int64_t c1 = c0 + a.chunk < a.M ? c0 + a.chunk : a.M;
  for (int64_t base = c0; base < c1; base += 64) {
    const int64_t i = base + lane;
    const bool valid = i < a.M;
    for (int d = 0; d < a.D; ++d) xl[d * 64] = a.Xt[int64_t(d) * a.Mp + i];
    const float yk = a.yp[i];
    __builtin_amdgcn_wave_barrier();
    // ---- forward with tape
    float top = 0.0f;
    float stk[GRAD_S];
#pragma unroll
    for (int j = 0; j < GRAD_S; ++j) stk[j] = 0.0f;
    auto step = [&](int t) {
      const uint32_t w = W.word(t);
      const uint32_t arg = (w >> 8) & 0xFFu;
      stk[(w >> 16) & 0xFu] = top;
      switch (w & 0xFFu) {
        case H_VAR: top = xl[arg * 64]; break;
        case H_CONST: top = W.cv(t); break;
#define BGL_GBIN(O, N) \
  case H_BIN + 15 * O + (N - 2): top = gbinop<O>(stk[N - 2], top); break;
#define BGL_GBIN_ALL(O)                                                                         \
  BGL_GBIN(O, 2) BGL_GBIN(O, 3) BGL_GBIN(O, 4) BGL_GBIN(O, 5) BGL_GBIN(O, 6) BGL_GBIN(O, 7)     \
  BGL_GBIN(O, 8) BGL_GBIN(O, 9) BGL_GBIN(O, 10) BGL_GBIN(O, 11) BGL_GBIN(O, 12) BGL_GBIN(O, 13) \
  BGL_GBIN(O, 14) BGL_GBIN(O, 15) BGL_GBIN(O, 16)
        BGL_GBIN_ALL(B_ADD)
        BGL_GBIN_ALL(B_SUB)
        BGL_GBIN_ALL(B_MUL)
        BGL_GBIN_ALL(B_DIV)
        BGL_GBIN_ALL(B_RSUB)
        BGL_GBIN_ALL(B_RDIV)
#undef BGL_GBIN
#undef BGL_GBIN_ALL
        case H_UN + 0: top = trig1<false>(top); break;
        case H_UN + 1: top = trig1<true>(top); break;
        case H_UN + 2: top = op_exp(top); break;
        case H_UN + 3: top = op_log(top); break;
        case H_UN + 4: top = op_sqrt(top); break;
#define BGL_GFUSED(O)                                                     \
  case H_FUSED + O: top = gbinop<O>(top, xl[arg * 64]); break;            \
  case H_FUSED + 6 + O: top = gbinop<O>(top, W.cv(t)); break;
        BGL_GFUSED(B_ADD)
        BGL_GFUSED(B_SUB)
        BGL_GFUSED(B_MUL)
        BGL_GFUSED(B_DIV)
        BGL_GFUSED(B_RSUB)
        BGL_GFUSED(B_RDIV)
#undef BGL_GFUSED
        default: break;
      }
    };
    if constexpr (LONG) {
      for (int t = 0; t < L; ++t) {
        step(t);
        tape_lds[t * 64] = top;
      }
    } else {
      // one loop per register array, so each array is written once per word
      const int L0 = L < 32 ? L : 32;
      for (int t = 0; t < L0; ++t) {
        step(t);
        tape_lo[t] = top;
      }
      for (int t = 32; t < L; ++t) {
        step(t);
        tape_hi[t - 32] = top;
      }
    }
    // ---- seed and fitness term
    const double dd = double(top) - double(yk);
    s_mse += valid ? dd * dd : 0.0;
    float g = valid ? float(dd) * inv2m : 0.0f;
    // ---- reverse
    float astk[GRAD_S];
#pragma unroll
    for (int j = 0; j < GRAD_S; ++j) astk[j] = 0.0f;
    for (int t = L - 1; t >= 0; --t) {
      const uint32_t w = W.word(t);
      const uint32_t xw = W.auxw(t);
      const uint32_t arg = (w >> 8) & 0xFFu;
      const uint32_t ws = (w >> 16) & 0xFu;
      const int pa = int(xw & 0xFFFFu);
      float wv = g;            // written to astk[rws]: meaningful for binary words only
      float gc = 0.0f;         // gradient contribution of a CONST slot
      bool has_c = false;
      switch (w & 0xFFu) {
        case H_VAR: g = astk[ws]; break;
        case H_CONST:
          gc = g;
          has_c = true;
          g = astk[ws];
          break;
#define BGL_RBIN(O, N)                                 \
  case H_BIN + 15 * O + (N - 2): {                     \
    float dA, dB;                                      \
    dbinop<O>(tget(pa), tget(t - 1), dA, dB);  \
    wv = g * dA;                                       \
    g = g * dB;                                        \
    break;                                             \
  }
#define BGL_RBIN_ALL(O)                                                                         \
  BGL_RBIN(O, 2) BGL_RBIN(O, 3) BGL_RBIN(O, 4) BGL_RBIN(O, 5) BGL_RBIN(O, 6) BGL_RBIN(O, 7)     \
  BGL_RBIN(O, 8) BGL_RBIN(O, 9) BGL_RBIN(O, 10) BGL_RBIN(O, 11) BGL_RBIN(O, 12) BGL_RBIN(O, 13) \
  BGL_RBIN(O, 14) BGL_RBIN(O, 15) BGL_RBIN(O, 16)
        BGL_RBIN_ALL(B_ADD)
        BGL_RBIN_ALL(B_SUB)
        BGL_RBIN_ALL(B_MUL)
        BGL_RBIN_ALL(B_DIV)
        BGL_RBIN_ALL(B_RSUB)
        BGL_RBIN_ALL(B_RDIV)
#undef BGL_RBIN
#undef BGL_RBIN_ALL
        case H_UN + 0:
        case H_UN + 1:
        case H_UN + 2:
        case H_UN + 3:
        case H_UN + 4:
          g = g * dunary((w & 0xFFu) - H_UN, tget(t - 1), tget(t));
          break;
#define BGL_RFUSED(O)                                   \
  case H_FUSED + O: {                                   \
    float dA, dB;                                       \
    dbinop<O>(tget(t - 1), xl[arg * 64], dA, dB);   \
    g = g * dA;                                         \
    break;                                              \
  }                                                     \
  case H_FUSED + 6 + O: {                               \
    float dA, dB;                                       \
    dbinop<O>(tget(t - 1), W.cv(t), dA, dB);        \
    gc = g * dB;                                        \
    has_c = true;                                       \
    g = g * dA;                                         \
    break;                                              \
  }
        BGL_RFUSED(B_ADD)
        BGL_RFUSED(B_SUB)
        BGL_RFUSED(B_MUL)
        BGL_RFUSED(B_DIV)
        BGL_RFUSED(B_RSUB)
        BGL_RFUSED(B_RDIV)
#undef BGL_RFUSED
        default: break;
      }
      astk[xw >> 16] = wv;
      if (has_c) {  // wave-uniform
        const double v = valid ? double(gc) : 0.0;
        if (arg < uint32_t(LANE_SLOTS)) {
          lg[arg * 64] += v;
        } else {
          const double sv = wave_sum_d(v);
          if (lane == 0) wg[arg] += sv;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // ---- reductions (fixed order) and partial outputs
  s_mse = wave_sum_d(s_mse);
  if (lane == 0) a.part[int64_t(c) * a.n_programs + p] = s_mse;
  double* gp = a.gpart + int64_t(c) * a.n_consts + coff;
  const int nl = cc < LANE_SLOTS ? cc : LANE_SLOTS;
  for (int j = 0; j < nl; ++j) {
    const double v = wave_sum_d(lg[j * 64]);
    if (lane == 0) gp[j] = v;
  }
  __builtin_amdgcn_wave_barrier();
  for (int j = LANE_SLOTS + lane; j < cc; j += 64) gp[j] = wg[j];
  __builtin_amdgcn_wave_barrier();
}

template <bool LONG>
__global__ void __launch_bounds__(64) k_grad(GradArgs a) {
  extern __shared__ float lds[];
  const int32_t count = a.list_count[LONG ? 1 : 0];
  const int64_t items = int64_t(count) * a.n_chunks;
  const int32_t* list = a.list + (LONG ? int64_t(a.n_programs) : 0);
  for (;;) {
    unsigned long long it = 0;
    if (threadIdx.x == 0) it = atomicAdd(a.work + (LONG ? 1 : 0), 1ull);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(it));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(it >> 32));
    const int64_t item = int64_t((uint64_t(hi) << 32) | lo);
    if (item >= items) break;
    const int c = int(item / count);
    const int p = list[item % count];
    grad_item<LONG>(a, p, c, lds);
  }
}

__global__ void k_grad_finalize(GradFinalizeArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_programs) return;
  const ProgMeta m = a.meta[p];
  const double nan = __longlong_as_double(0x7FF8000000000000LL);
  const int64_t coff = a.const_offset[p];
  const int cc = a.const_count[p];
  if (m.status != BEAGLE_PROG_OK) {
    a.fitness[p] = nan;
    for (int j = 0; j < cc; ++j) a.grad[coff + j] = __int_as_float(0x7FC00000);
    return;
  }
  double s = 0.0;
  for (int c = 0; c < a.n_chunks; ++c) s += a.part[int64_t(c) * a.n_programs + p];
  a.fitness[p] = s / double(a.M);
  for (int j = 0; j < cc; ++j) {
    double g = 0.0;
    for (int c = 0; c < a.n_chunks; ++c) g += a.gpart[int64_t(c) * a.n_consts + coff + j];
    a.grad[coff + j] = float(g);
  }
}

static int grad_cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 1;
  }
  return n;
}

size_t grad_lds_bytes(int D, bool long_tape) {
  size_t b = size_t(D) * 64 * sizeof(float) + (size_t(LANE_SLOTS) * 64 + 256) * sizeof(double);
  if (long_tape) b += size_t(GRAD_LONG_WORDS) * 64 * sizeof(float);
  return b;
}

hipError_t launch_grad(const GradArgs& a, hipStream_t s) {
  const int cus = grad_cu_count();
  const size_t l0 = grad_lds_bytes(a.D, false), l1 = grad_lds_bytes(a.D, true);
  int nb0 = 0, nb1 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb0, k_grad<false>, 64, l0) != hipSuccess || nb0 < 1) nb0 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, k_grad<true>, 64, l1) != hipSuccess || nb1 < 1) nb1 = 1;
  hipLaunchKernelGGL(k_grad<false>, dim3(nb0 * cus), dim3(64), l0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad<true>, dim3(nb1 * cus), dim3(64), l1, s, a);
  return hipGetLastError();
}

}  // namespace bgl
