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
//  seed     g = dF/dyhat for the case (0 for padding): MSE 2 (yhat - y) / M,
//           CORR from the program's coefficients (see Seed);
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
constexpr int LANE_SLOTS = GRAD_LANE_SLOTS;  // constant slots accumulated per lane

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
    const float r = __builtin_amdgcn_rcpf(nz ? B : 1.0f);
    dA = nz ? r : 0.0f;
    dB = nz ? -A * r * r : 0.0f;
  }
  if constexpr (O == B_RSUB) { dA = -1.0f; dB = 1.0f; }
  if constexpr (O == B_RDIV) {
    const bool nz = A != 0.0f;
    const float r = __builtin_amdgcn_rcpf(nz ? A : 1.0f);
    dA = nz ? -B * r * r : 0.0f;
    dB = nz ? r : 0.0f;
  }
}

// binop<O> and its partial derivatives on G cases per lane: the protected
// quotients through div_tile_r, whose reciprocal the derivatives reuse
// (the same values dbinop gives)
template <uint32_t O, int G>
__device__ __forceinline__ void dbinop_tile(const float (&A)[G], const float (&B)[G], float (&q)[G], float (&dA)[G],
                                            float (&dB)[G]) {
  if constexpr (O == B_DIV || O == B_RDIV) {
    float r[G];
    if constexpr (O == B_DIV)
      div_tile_r<G>(A, B, q, r);
    else
      div_tile_r<G>(B, A, q, r);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if constexpr (O == B_DIV) {
        const bool nz = B[k] != 0.0f;
        dA[k] = nz ? r[k] : 0.0f;
        dB[k] = nz ? -A[k] * r[k] * r[k] : 0.0f;
      } else {
        const bool nz = A[k] != 0.0f;
        dA[k] = nz ? -B[k] * r[k] * r[k] : 0.0f;
        dB[k] = nz ? r[k] : 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < G; ++k) {
      q[k] = gbinop<O>(A[k], B[k]);
      dbinop<O>(A[k], B[k], dA[k], dB[k]);
    }
  }
}

// binop<O> on G cases per lane (values only)
template <uint32_t O, int G>
__device__ __forceinline__ void binop_tile_g(const float (&A)[G], const float (&B)[G], float (&q)[G]) {
  if constexpr (O == B_DIV) {
    div_tile<G>(A, B, q);
  } else if constexpr (O == B_RDIV) {
    div_tile<G>(B, A, q);
  } else {
#pragma unroll
    for (int k = 0; k < G; ++k) q[k] = gbinop<O>(A[k], B[k]);
  }
}

// sin (COS = false) or cos of one value per lane, the interpreter's functions
template <bool COS>
__device__ __forceinline__ float trig1(float x) {
  float v[1] = {x};
  trig_tile<COS, 1>(v);
  return v[0];
}

// d/dx of unary operator u at operand x with value y
__device__ __forceinline__ float dunary(uint32_t u, float x, float y) {
  switch (u) {
    case 0: return trig1<true>(x);
    case 1: return -trig1<false>(x);
    case 2: return (x > 80.0f || x < -80.0f) ? 0.0f : y;
    case 3: return x != 0.0f ? __builtin_amdgcn_rcpf(x) : 0.0f;
    case 4: return x != 0.0f ? copysignf(0.5f, x) * __builtin_amdgcn_rcpf(y) : 0.0f;
    case 5: return 2.0f * x;
    case 6: return -(y * y);
    case 7: return 1.0f + y * y;
    case 8: return rsqrtf((1.0f - x) * (1.0f + x));
    case 9: return -rsqrtf((1.0f - x) * (1.0f + x));
    case 10: return 1.0f / (1.0f + x * x);
    default: {
      // tanh: sech^2 x = 4e / (1 + e)^2 with e = exp(-2|x|) (1 - y^2 cancels
      // where tanh saturates)
      const float e = op_exp(-2.0f * __builtin_fabsf(x));
      const float ep = 1.0f + e;
      return (4.0f * e) / (ep * ep);
    }
  }
}

// An opaque copy: keeps two loaded values from being folded into one load
// through a selected address (which would force the arrays out of registers).
__device__ __forceinline__ float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ double wave_sum_d(double v) { return wave_sum(v); }

// dF/dyhat of one case: MSE 2 (yhat - y) / M (the binary64 difference
// rounded, then scaled); CORR alpha (y - ycen) + beta (yhat - mu) in
// binary64 with the program's coefficients from the evaluation pass
// (ycen = mean y + mean of y - mean y).
struct Seed {
  bool corr;
  float inv2m;
  double alpha, beta, mu, ycen;
  __device__ __forceinline__ Seed(const GradArgs& a, int p) {
    corr = a.kind == BEAGLE_FIT_CORR;
    inv2m = float(2.0 / double(a.M));
    alpha = beta = mu = ycen = 0.0;
    if (corr) {
      alpha = uniform(a.coef[3 * int64_t(p)]);
      beta = uniform(a.coef[3 * int64_t(p) + 1]);
      mu = uniform(a.coef[3 * int64_t(p) + 2]);
      ycen = uniform(a.stats[0] + a.stats[1] / double(a.M));
    }
  }
  // a wave-uniform value held in scalar registers
  __device__ static __forceinline__ double uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
  }
  __device__ __forceinline__ float operator()(float yhat, float y) const {
    if (corr) return float(alpha * (double(y) - ycen) + beta * (double(yhat) - mu));
    return float(double(yhat) - double(y)) * inv2m;
  }
};

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
  const Seed seed(a, p);
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
        case H_UN + 5: top = op_ext<5>(top); break;
        case H_UN + 6: top = op_ext<6>(top); break;
        case H_UN + 7: top = op_ext<7>(top); break;
        case H_UN + 8: top = op_ext<8>(top); break;
        case H_UN + 9: top = op_ext<9>(top); break;
        case H_UN + 10: top = op_ext<10>(top); break;
        case H_UN + 11: top = op_ext<11>(top); break;
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
    float g = valid ? seed(top, yk) : 0.0f;
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
        case H_UN + 5:
        case H_UN + 6:
        case H_UN + 7:
        case H_UN + 8:
        case H_UN + 9:
        case H_UN + 10:
        case H_UN + 11:
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
      astk[(xw >> 16) & 0xFu] = wv;
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
  // waves beyond the item batches leave at once (no atomic on a short list)
  if (int64_t(blockIdx.x) * GRAD_BATCH >= items) return;
  for (;;) {
    // as in k_grad_dtape: every lane in the atomic, a batch per atomic
    const unsigned long long it =
        atomicAdd(a.work + (LONG ? 1 : 0), threadIdx.x == 0 ? (unsigned long long)GRAD_BATCH : 0ull);
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(it), 0);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(it >> 32), 0);
    const int64_t first = int64_t((uint64_t(hi) << 32) | lo);
    if (first >= items) break;
    const int n = int(first + GRAD_BATCH < items ? GRAD_BATCH : items - first);
    int c = int(first / count), i = int(first - int64_t(c) * count);
    for (int k = 0; k < n; ++k) {
      const int p = __builtin_amdgcn_readfirstlane(list[i]);
      grad_item<LONG>(a, p, c, lds);
      if (++i == count) {
        i = 0;
        ++c;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The derivative-tape adjoint: programs of register need <= 4 and at most
// GRAD_LANE_SLOTS constant slots whose tape fits GRAD_DTAPE_SMALL (list 2, 4
// cases per lane), GRAD_DTAPE_MID (list 3, 2 cases per lane) or
// GRAD_DTAPE_LARGE (list 4, 2 cases per lane) entries per case.
//
// The forward sweep runs the small-stack handlers (stack size n known per
// handler: every stack slot is a register named at compile time) and each
// handler stores the local partial derivatives the reverse sweep will need,
// not its output: binary *, / and reversed / two entries (d/da, d/db), unary
// operators one (sin x takes cos x from its own reduction), fused VAR *, /
// one, fused CONST *, / one (d/dc) and reversed / two, every other word none.
// Entries are appended in word order, so the reverse sweep, walking the
// words backwards, takes them from the end with a wave-uniform counter.  The
// reverse handler of a word (aux bits 24..31) is a linear update of the
// adjoint stack A:
//   binary at n    A[n-1] = A[n-2] d/db,  A[n-2] = A[n-2] d/da
//   unary, fused   A[n-1] scaled by d/dtop
//   CONST          its slot's gradient gains A (times d/dc when fused)
// A subtree without CONST words adds to no gradient: its words store no
// entries (their own forward handlers), and the reverse sweep follows a
// per-word "next" index (aux bits 0..7) that skips such a subtree in one
// step, and skips the words whose reverse update is the identity.
// The tape is one register array per case (list 4: two, entries 0..31 and
// 32..63), each array a separate variable so that it stays in registers.
static_assert(GRAD_TILE_CASES % (4 * 64) == 0 && GRAD_TILE_CASES % (2 * 64) == 0,
              "adjoint chunks hold whole tiles");

// The tape of 2 cases per lane: entry e of case k in lk[e] (e < 32) or
// hk[e - 32] (H > 0).
template <int H>
struct Tape2 {
  static constexpr int HS = H > 0 ? H : 1;
  float (&l0)[32];
  float (&l1)[32];
  float (&h0)[HS];
  float (&h1)[HS];
  __device__ __forceinline__ void put(int e, const float (&v)[2]) {
    if (H == 0 || e < 32) {
      l0[e & 31] = v[0];
      l1[e & 31] = v[1];
    } else {
      h0[(e - 32) & (HS - 1)] = v[0];
      h1[(e - 32) & (HS - 1)] = v[1];
    }
  }
  __device__ __forceinline__ void get(int e, float (&v)[2]) const {
    if constexpr (H == 0) {
      v[0] = l0[e & 31];
      v[1] = l1[e & 31];
    } else {
      // both halves read and one selected (no branch on the entry index)
      const float x0 = opaque(l0[e & 31]), y0 = opaque(h0[(e - 32) & (HS - 1)]);
      const float x1 = opaque(l1[e & 31]), y1 = opaque(h1[(e - 32) & (HS - 1)]);
      v[0] = e < 32 ? x0 : y0;
      v[1] = e < 32 ? x1 : y1;
    }
  }
};

// The tape of 4 cases per lane, N entries per case.
template <int N>
struct Tape4 {
  float (&t0)[N];
  float (&t1)[N];
  float (&t2)[N];
  float (&t3)[N];
  __device__ __forceinline__ void put(int e, const float (&v)[4]) {
    t0[e & (N - 1)] = v[0];
    t1[e & (N - 1)] = v[1];
    t2[e & (N - 1)] = v[2];
    t3[e & (N - 1)] = v[3];
  }
  __device__ __forceinline__ void get(int e, float (&v)[4]) const {
    v[0] = t0[e & (N - 1)];
    v[1] = t1[e & (N - 1)];
    v[2] = t2[e & (N - 1)];
    v[3] = t3[e & (N - 1)];
  }
};

#define BGL_K(G) _Pragma("unroll") for (int k = 0; k < (G); ++k)

// one forward word (forward handler fid) for G cases; e = the next free tape
// entry
template <int G, class TP>
__device__ __forceinline__ void dt_fwd(uint32_t fid, float cv, const float (&x)[G], float (&st)[G][4], TP& tp,
                                       int& e) {
#define BGL_PUT(D) \
  tp.put(e, D);    \
  ++e;
  switch (fid) {
#define BGL_F_PUSH(N)                    \
  case I0_PUSH_VAR + N:                  \
    BGL_K(G) st[k][N] = x[k];            \
    break;                               \
  case I0_PUSH_CONST + N:                \
    BGL_K(G) st[k][N] = cv;              \
    break;
    BGL_F_PUSH(0) BGL_F_PUSH(1) BGL_F_PUSH(2) BGL_F_PUSH(3)
#undef BGL_F_PUSH
#define BGL_F_BIN(O, N)                                       \
  case I0_BIN + 3 * O + (N - 2): {                            \
    float a_[G], b_[G], q_[G], dA[G], dB[G];                  \
    BGL_K(G) {                                                \
      a_[k] = st[k][N - 2];                                   \
      b_[k] = st[k][N - 1];                                   \
    }                                                         \
    dbinop_tile<O, G>(a_, b_, q_, dA, dB);                    \
    BGL_K(G) st[k][N - 2] = q_[k];                            \
    if constexpr (O == B_MUL || O == B_DIV || O == B_RDIV) {  \
      BGL_PUT(dA)                                             \
      BGL_PUT(dB)                                             \
    }                                                         \
    break;                                                    \
  }
#define BGL_F_BIN3(O) BGL_F_BIN(O, 2) BGL_F_BIN(O, 3) BGL_F_BIN(O, 4)
    BGL_F_BIN3(B_ADD) BGL_F_BIN3(B_SUB) BGL_F_BIN3(B_MUL) BGL_F_BIN3(B_DIV) BGL_F_BIN3(B_RSUB) BGL_F_BIN3(B_RDIV)
#undef BGL_F_BIN3
#undef BGL_F_BIN
#define BGL_F_UN(N)                                            \
  case I0_UN + 0 * 4 + (N - 1): {                              \
    float s[G], c[G];                                          \
    BGL_K(G) s[k] = st[k][N - 1];                              \
    sincos_tile<G>(s, c);                                      \
    BGL_K(G) st[k][N - 1] = s[k];                              \
    BGL_PUT(c)                                                 \
    break;                                                     \
  }                                                            \
  case I0_UN + 1 * 4 + (N - 1): {                              \
    float v[G], d[G];                                          \
    BGL_K(G) v[k] = st[k][N - 1];                              \
    cos_nsin_tile<G>(v, d);                                    \
    BGL_K(G) st[k][N - 1] = v[k];                              \
    BGL_PUT(d)                                                 \
    break;                                                     \
  }                                                            \
  case I0_UN + 2 * 4 + (N - 1): {                              \
    float u[G], v[G], d[G];                                    \
    BGL_K(G) u[k] = v[k] = st[k][N - 1];                       \
    exp_tile<G>(v);                                            \
    BGL_K(G) {                                                 \
      st[k][N - 1] = v[k];                                     \
      d[k] = dunary(2u, u[k], v[k]);                           \
    }                                                          \
    BGL_PUT(d)                                                 \
    break;                                                     \
  }                                                            \
  case I0_UN + 3 * 4 + (N - 1): {                              \
    float u[G], v[G], d[G];                                    \
    BGL_K(G) u[k] = v[k] = st[k][N - 1];                       \
    log_tile<G>(v);                                            \
    BGL_K(G) {                                                 \
      st[k][N - 1] = v[k];                                     \
      d[k] = dunary(3u, u[k], 0.0f);                           \
    }                                                          \
    BGL_PUT(d)                                                 \
    break;                                                     \
  }                                                            \
  case I0_UN + 4 * 4 + (N - 1): {                              \
    float u[G], v[G], d[G];                                    \
    BGL_K(G) u[k] = v[k] = st[k][N - 1];                       \
    sqrt_tile<G>(v);                                           \
    BGL_K(G) {                                                 \
      st[k][N - 1] = v[k];                                     \
      d[k] = dunary(4u, u[k], v[k]);                           \
    }                                                          \
    BGL_PUT(d)                                                 \
    break;                                                     \
  }
    BGL_F_UN(1) BGL_F_UN(2) BGL_F_UN(3) BGL_F_UN(4)
#undef BGL_F_UN
#define BGL_F_FUSED(O, N)                                     \
  case I0_FUSED + 3 * O + (N - 1): {                          \
    float a_[G], q_[G], dA[G], dB[G];                         \
    BGL_K(G) a_[k] = st[k][N - 1];                            \
    dbinop_tile<O, G>(a_, x, q_, dA, dB);                     \
    BGL_K(G) st[k][N - 1] = q_[k];                            \
    if constexpr (O == B_MUL || O == B_DIV || O == B_RDIV) {  \
      BGL_PUT(dA)                                             \
    }                                                         \
    break;                                                    \
  }                                                           \
  case I0_FUSED + 3 * (6 + O) + (N - 1): {                    \
    float a_[G], c_[G], q_[G], dA[G], dB[G];                  \
    BGL_K(G) {                                                \
      a_[k] = st[k][N - 1];                                   \
      c_[k] = cv;                                             \
    }                                                         \
    dbinop_tile<O, G>(a_, c_, q_, dA, dB);                    \
    BGL_K(G) st[k][N - 1] = q_[k];                            \
    if constexpr (O == B_RDIV) {                              \
      BGL_PUT(dA)                                             \
    }                                                         \
    if constexpr (O == B_MUL || O == B_DIV || O == B_RDIV) {  \
      BGL_PUT(dB)                                             \
    }                                                         \
    break;                                                    \
  }
#define BGL_F_FUSED3(O) BGL_F_FUSED(O, 1) BGL_F_FUSED(O, 2) BGL_F_FUSED(O, 3)
    BGL_F_FUSED3(B_ADD) BGL_F_FUSED3(B_SUB) BGL_F_FUSED3(B_MUL) BGL_F_FUSED3(B_DIV) BGL_F_FUSED3(B_RSUB)
    BGL_F_FUSED3(B_RDIV)
#undef BGL_F_FUSED3
#undef BGL_F_FUSED
    // constant-free words: values only
#define BGL_N_BIN(J, O, N)                                         \
  case F_BIN_NT + 3 * J + (N - 2): {                               \
    float a_[G], b_[G], q_[G];                                     \
    BGL_K(G) {                                                     \
      a_[k] = st[k][N - 2];                                        \
      b_[k] = st[k][N - 1];                                        \
    }                                                              \
    binop_tile_g<O, G>(a_, b_, q_);                                \
    BGL_K(G) st[k][N - 2] = q_[k];                                 \
    break;                                                         \
  }
#define BGL_N_BIN3(J, O) BGL_N_BIN(J, O, 2) BGL_N_BIN(J, O, 3) BGL_N_BIN(J, O, 4)
    BGL_N_BIN3(0, B_MUL) BGL_N_BIN3(1, B_DIV) BGL_N_BIN3(2, B_RDIV)
#undef BGL_N_BIN3
#undef BGL_N_BIN
#define BGL_N_UN(N)                                  \
  case F_UN_NT + 0 * 4 + (N - 1): {                  \
    float v[G];                                      \
    BGL_K(G) v[k] = st[k][N - 1];                    \
    trig_tile<false, G>(v);                          \
    BGL_K(G) st[k][N - 1] = v[k];                    \
    break;                                           \
  }                                                  \
  case F_UN_NT + 1 * 4 + (N - 1): {                  \
    float v[G];                                      \
    BGL_K(G) v[k] = st[k][N - 1];                    \
    trig_tile<true, G>(v);                           \
    BGL_K(G) st[k][N - 1] = v[k];                    \
    break;                                           \
  }                                                  \
  case F_UN_NT + 2 * 4 + (N - 1): {                  \
    float v[G];                                      \
    BGL_K(G) v[k] = st[k][N - 1];                    \
    exp_tile<G>(v);                                  \
    BGL_K(G) st[k][N - 1] = v[k];                    \
    break;                                           \
  }                                                  \
  case F_UN_NT + 3 * 4 + (N - 1): {                  \
    float v[G];                                      \
    BGL_K(G) v[k] = st[k][N - 1];                    \
    log_tile<G>(v);                                  \
    BGL_K(G) st[k][N - 1] = v[k];                    \
    break;                                           \
  }                                                  \
  case F_UN_NT + 4 * 4 + (N - 1): {                  \
    float v[G];                                      \
    BGL_K(G) v[k] = st[k][N - 1];                    \
    sqrt_tile<G>(v);                                 \
    BGL_K(G) st[k][N - 1] = v[k];                    \
    break;                                           \
  }
    BGL_N_UN(1) BGL_N_UN(2) BGL_N_UN(3) BGL_N_UN(4)
#undef BGL_N_UN
#define BGL_N_FV(J, O, N)                                 \
  case F_FV_NT + 3 * J + (N - 1): {                       \
    float a_[G], q_[G];                                   \
    BGL_K(G) a_[k] = st[k][N - 1];                        \
    binop_tile_g<O, G>(a_, x, q_);                        \
    BGL_K(G) st[k][N - 1] = q_[k];                        \
    break;                                                \
  }
#define BGL_N_FV3(J, O) BGL_N_FV(J, O, 1) BGL_N_FV(J, O, 2) BGL_N_FV(J, O, 3)
    BGL_N_FV3(0, B_MUL) BGL_N_FV3(1, B_DIV) BGL_N_FV3(2, B_RDIV)
#undef BGL_N_FV3
#undef BGL_N_FV
    default:
      break;
  }
#undef BGL_PUT
}

// slot arg (< GRAD_LANE_SLOTS) of the lane's gradient sums gains the cases'
// contributions g[k] (valid cases only): an LDS add without a returned value,
// so nothing waits for it, and the adds of one lane reach its slot in
// program order
template <int G>
__device__ __forceinline__ void add_const_grad(uint32_t arg, const float (&g)[G], const bool (&valid)[G],
                                               double* lg) {
  double v = 0.0;
  BGL_K(G) v += valid[k] ? double(g[k]) : 0.0;
  __hip_atomic_fetch_add(lg + arg * 64, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// one program on one chunk of cases, G cases per lane (case base + 64 k +
// lane of each tile of 64 G cases)
template <int G, class TP>
__device__ __forceinline__ void dtape_item(const GradArgs& a, int p, int c, float* lds, TP tp) {
  const int lane = threadIdx.x;
  const ProgMeta m = a.meta[p];
  const int L = m.len;
  const int64_t off = a.tok_offset[p];
  const int64_t coff = a.const_offset[p];
  const int cc = a.const_count[p];
  const uint32_t vmask = uint32_t(__builtin_amdgcn_readfirstlane(int(m.vmask)));
  const uint32_t dmax = uint32_t(a.D - 1);
  // x: the word's aux entry, (next + 1) | fid << 8 | arg << 16 | rid << 24
  auto xrow = [dmax](uint32_t x) -> uint32_t {
    const uint32_t r = (x >> 16) & 0xFFu;
    return r < dmax ? r : dmax;
  };
  const uint32_t va = lane < L ? a.aux[off + lane] : 0u;
  const float vv = lane < L ? a.cval[off + lane] : 0.0f;
  // LDS: input tile [D][G][64] | lane gradients [LANE_SLOTS][64] doubles
  // (the program has at most LANE_SLOTS constant slots)
  double* lg = reinterpret_cast<double*>(lds + a.D * G * 64) + lane;
  for (int j = 0; j < LANE_SLOTS; ++j) lg[j * 64] = 0.0;
  __builtin_amdgcn_wave_barrier();
  double s_mse = 0.0;
  const Seed seed(a, p);
  const int64_t c0 = int64_t(c) * a.chunk;
  const int64_t c1 = c0 + a.chunk < a.M ? c0 + a.chunk : a.M;
  for (int64_t base = c0; base < c1; base += G * 64) {
    bool valid[G];
    float yv[G];
    BGL_K(G) valid[k] = base + 64 * k + lane < a.M;
    // the tile's inputs go straight from global memory to LDS (64 cases per
    // instruction), every variable's loads issued before one wait
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the last tile's LDS reads are done
    for (int d = 0; d < a.D; ++d) {
      if (!((vmask >> d) & 1u)) continue;
      BGL_K(G) __builtin_amdgcn_global_load_lds(a.Xt + int64_t(d) * a.Mp + base + 64 * k + lane,
                                                lds + (d * G + k) * 64, 4, 0, 0);
    }
    BGL_K(G) yv[k] = a.yp[base + 64 * k + lane];
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the tile is in LDS
    __builtin_amdgcn_wave_barrier();
    // ---- forward: values on the stack, partial derivatives on the tape
    float st[G][4];
    BGL_K(G) for (int j = 0; j < 4; ++j) st[k][j] = 0.0f;
    // The input row a word reads is loaded at the end of the previous word,
    // into the registers the handler reads (no copies), so that the LDS
    // latency overlaps the dispatch; words that read no input load row
    // min(arg, D - 1), which is in the tile and unused.
    const float* xt = lds + lane;
    int e = 0;
    uint32_t w = __builtin_amdgcn_readlane(va, 0);
    float xa[G];
    BGL_K(G) xa[k] = xt[xrow(w) * (G * 64) + 64 * k];
    for (int t = 0; t < L; ++t) {
      const float cv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t));
      dt_fwd<G>((w >> 8) & 0xFFu, cv, xa, st, tp, e);
      w = t + 1 < L ? __builtin_amdgcn_readlane(va, t + 1) : 0u;
      BGL_K(G) xa[k] = xt[xrow(w) * (G * 64) + 64 * k];
    }
    // ---- seed and fitness terms
    float A[G][4];
    BGL_K(G) {
      const double ek = double(st[k][0]) - double(yv[k]);
      s_mse += valid[k] ? ek * ek : 0.0;
      for (int j = 0; j < 4; ++j) A[k][j] = 0.0f;
      A[k][0] = valid[k] ? seed(st[k][0], yv[k]) : 0.0f;
    }
    // ---- reverse: linear updates of the adjoint stack, visiting only the
    // words that are neither constant-free nor NOP (the root always)
    for (int t = L - 1; t >= 0;) {
      const uint32_t x = __builtin_amdgcn_readlane(va, t);
      const uint32_t rid = x >> 24;
      const uint32_t arg = (x >> 16) & 0xFFu;
      const float cv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t));
      t = int(x & 0xFFu) - 1;
      float g[G], d0[G], d1[G];
      switch (rid) {
#define BGL_R_PUSH(N)                             \
  case R_PUSH_CONST + N:                          \
    BGL_K(G) g[k] = A[k][N];                      \
    add_const_grad<G>(arg, g, valid, lg);         \
    break;
        BGL_R_PUSH(0) BGL_R_PUSH(1) BGL_R_PUSH(2) BGL_R_PUSH(3)
#undef BGL_R_PUSH
#define BGL_R_BIN(N)                                    \
  case R_BIN_ADD + (N - 2):                             \
    BGL_K(G) A[k][N - 1] = A[k][N - 2];                 \
    break;                                              \
  case R_BIN_SUB + (N - 2):                             \
    BGL_K(G) A[k][N - 1] = -A[k][N - 2];                \
    break;                                              \
  case R_BIN_RSUB + (N - 2):                            \
    BGL_K(G) {                                          \
      A[k][N - 1] = A[k][N - 2];                        \
      A[k][N - 2] = -A[k][N - 2];                       \
    }                                                   \
    break;                                              \
  case R_BIN_GEN + (N - 2):                             \
    e -= 2;                                             \
    tp.get(e, d0);                                      \
    tp.get(e + 1, d1);                                  \
    BGL_K(G) {                                          \
      A[k][N - 1] = A[k][N - 2] * d1[k];                \
      A[k][N - 2] *= d0[k];                             \
    }                                                   \
    break;
        BGL_R_BIN(2) BGL_R_BIN(3) BGL_R_BIN(4)
#undef BGL_R_BIN
#define BGL_R_UN(N)                       \
  case R_UN + (N - 1):                    \
    e -= 1;                               \
    tp.get(e, d0);                        \
    BGL_K(G) A[k][N - 1] *= d0[k];        \
    break;
        BGL_R_UN(1) BGL_R_UN(2) BGL_R_UN(3) BGL_R_UN(4)
#undef BGL_R_UN
#define BGL_R_FUSED(N)                                             \
  case R_FV_RSUB + (N - 1):                                        \
    BGL_K(G) A[k][N - 1] = -A[k][N - 1];                           \
    break;                                                         \
  case R_FV_GEN + (N - 1):                                         \
    e -= 1;                                                        \
    tp.get(e, d0);                                                 \
    BGL_K(G) A[k][N - 1] *= d0[k];                                 \
    break;                                                         \
  case R_FC_ADD + (N - 1):                                         \
    BGL_K(G) g[k] = A[k][N - 1];                                   \
    add_const_grad<G>(arg, g, valid, lg);                          \
    break;                                                         \
  case R_FC_SUB + (N - 1):                                         \
    BGL_K(G) g[k] = -A[k][N - 1];                                  \
    add_const_grad<G>(arg, g, valid, lg);                          \
    break;                                                         \
  case R_FC_RSUB + (N - 1):                                        \
    BGL_K(G) {                                                     \
      g[k] = A[k][N - 1];                                          \
      A[k][N - 1] = -A[k][N - 1];                                  \
    }                                                              \
    add_const_grad<G>(arg, g, valid, lg);                          \
    break;                                                         \
  case R_FC_MUL + (N - 1):                                         \
    e -= 1;                                                        \
    tp.get(e, d0);                                                 \
    BGL_K(G) {                                                     \
      g[k] = A[k][N - 1] * d0[k];                                  \
      A[k][N - 1] *= cv;                                           \
    }                                                              \
    add_const_grad<G>(arg, g, valid, lg);                          \
    break;                                                         \
  case R_FC_DIV + (N - 1): {                                       \
    e -= 1;                                                        \
    tp.get(e, d0);                                                 \
    float dA, dB;                                                  \
    dbinop<B_DIV>(0.0f, cv, dA, dB);                               \
    BGL_K(G) {                                                     \
      g[k] = A[k][N - 1] * d0[k];                                  \
      A[k][N - 1] *= dA;                                           \
    }                                                              \
    add_const_grad<G>(arg, g, valid, lg);                          \
    break;                                                         \
  }                                                                \
  case R_FC_RDIV + (N - 1):                                        \
    e -= 2;                                                        \
    tp.get(e, d0);                                                 \
    tp.get(e + 1, d1);                                             \
    BGL_K(G) {                                                     \
      g[k] = A[k][N - 1] * d1[k];                                  \
      A[k][N - 1] *= d0[k];                                        \
    }                                                              \
    add_const_grad<G>(arg, g, valid, lg);                          \
    break;
        BGL_R_FUSED(1) BGL_R_FUSED(2) BGL_R_FUSED(3)
#undef BGL_R_FUSED
        default:
          break;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // ---- reductions (fixed order) and partial outputs
  s_mse = wave_sum_d(s_mse);
  if (lane == 0) a.part[int64_t(c) * a.n_programs + p] = s_mse;
  double* gp = a.gpart + int64_t(c) * a.n_consts + coff;
  for (int j = 0; j < cc; ++j) {
    const double v = wave_sum_d(lg[j * 64]);
    if (lane == 0) gp[j] = v;
  }
  __builtin_amdgcn_wave_barrier();
}

// cases per lane of list 2, 3, 4
__host__ __device__ constexpr int dtape_cases(int list) { return list == 2 ? 4 : 2; }

template <int LIST>
__device__ __forceinline__ void dtape_list_item(const GradArgs& a, int p, int c, float* lds) {
  if constexpr (LIST == 2) {
    constexpr int N = GRAD_DTAPE_SMALL;
    float t0[N], t1[N], t2[N], t3[N];
    dtape_item<4>(a, p, c, lds, Tape4<N>{t0, t1, t2, t3});
  } else {
    constexpr int H = (LIST == 3 ? GRAD_DTAPE_MID : GRAD_DTAPE_LARGE) - 32;
    constexpr int HS = H > 0 ? H : 1;
    float l0[32], l1[32], h0[HS], h1[HS];
    dtape_item<2>(a, p, c, lds, Tape2<H>{l0, l1, h0, h1});
  }
}

// LIST 2, 3, 4: at most GRAD_DTAPE_SMALL (4 cases per lane), MID, LARGE
// entries per case (2 cases per lane, upper tape 0 or 32 entries).
template <int LIST>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LIST == 3 || LIST == 2 ? 4 : 1))) k_grad_dtape(GradArgs a) {
  extern __shared__ float lds[];
  const int32_t count = a.list_count[LIST];
  const int64_t items = int64_t(count) * a.n_chunks;
  const int32_t* list = a.list + LIST * int64_t(a.n_programs);
  if (int64_t(blockIdx.x) * GRAD_BATCH >= items) return;  // (as in k_grad)
  for (;;) {
    // every lane takes part (lane 0 adds GRAD_BATCH): no divergent branch in
    // the persistent loop, the first item read from lane 0 explicitly; a
    // batch of items per atomic (one same-address atomic per item would
    // serialise at the counter)
    const unsigned long long it = atomicAdd(a.work + LIST, threadIdx.x == 0 ? (unsigned long long)GRAD_BATCH : 0ull);
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(it), 0);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(it >> 32), 0);
    const int64_t first = int64_t((uint64_t(hi) << 32) | lo);
    if (first >= items) break;
    const int n = int(first + GRAD_BATCH < items ? GRAD_BATCH : items - first);
    // item = c * count + i, stepped without a division per item
    int c = int(first / count), i = int(first - int64_t(c) * count);
    for (int k = 0; k < n; ++k) {
      const int p = __builtin_amdgcn_readfirstlane(list[i]);
      dtape_list_item<LIST>(a, p, c, lds);
      if (++i == count) {
        i = 0;
        ++c;
      }
    }
  }
}
#undef BGL_K

// One wave per program: lane 0 sums the fitness partials, lane j the
// gradient partials of constant slot j (and j + 64, ...), each over the
// chunks in chunk order.
__global__ void __launch_bounds__(64) k_grad_finalize(GradFinalizeArgs a) {
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const ProgMeta m = a.meta[p];
  const double nan = __longlong_as_double(0x7FF8000000000000LL);
  const int64_t coff = a.const_offset[p];
  const int cc = a.const_count[p];
  if (m.status != BEAGLE_PROG_OK) {
    if (a.kind == BEAGLE_FIT_MSE && lane == 0) a.fitness[p] = nan;
    for (int j = lane; j < cc; j += 64) a.grad[coff + j] = __int_as_float(0x7FC00000);
    return;
  }
  if (a.kind == BEAGLE_FIT_MSE && lane == 0) {
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < a.n_chunks; ++c) s += a.part[int64_t(c) * a.n_programs + p];
    a.fitness[p] = s / double(a.M);
  }
  for (int j = lane; j < cc; j += 64) {
    double g = 0.0;
#pragma unroll 8
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
  const size_t l2 = size_t(a.D) * dtape_cases(2) * 64 * sizeof(float) + size_t(LANE_SLOTS) * 64 * sizeof(double);
  const size_t l3 = size_t(a.D) * dtape_cases(3) * 64 * sizeof(float) + size_t(LANE_SLOTS) * 64 * sizeof(double);
  int nb0 = 0, nb1 = 0, nb2 = 0, nb3 = 0, nb4 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb0, k_grad<false>, 64, l0) != hipSuccess || nb0 < 1) nb0 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, k_grad<true>, 64, l1) != hipSuccess || nb1 < 1) nb1 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, k_grad_dtape<2>, 64, l2) != hipSuccess || nb2 < 1) nb2 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb3, k_grad_dtape<3>, 64, l3) != hipSuccess || nb3 < 1) nb3 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb4, k_grad_dtape<4>, 64, l3) != hipSuccess || nb4 < 1) nb4 = 1;
  hipLaunchKernelGGL(k_grad_dtape<2>, dim3(nb2 * cus), dim3(64), l2, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_dtape<3>, dim3(nb3 * cus), dim3(64), l3, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_dtape<4>, dim3(nb4 * cus), dim3(64), l3, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad<false>, dim3(nb0 * cus), dim3(64), l0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad<true>, dim3(nb1 * cus), dim3(64), l1, s, a);
  return hipGetLastError();
}

}  // namespace bgl
