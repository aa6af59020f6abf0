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
    case 3: return x != 0.0f ? __builtin_amdgcn_rcpf(x) : 0.0f;
    default: return x != 0.0f ? copysignf(0.5f, x) * __builtin_amdgcn_rcpf(y) : 0.0f;
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

// ---------------------------------------------------------------------------
// The derivative-tape adjoint: programs of register need <= 4 whose tape
// fits GRAD_DTAPE_SMALL (list 2) or GRAD_DTAPE_LARGE (list 3) entries per
// case, GK cases per lane.
//
// The forward sweep runs the small-stack handlers (word bits 24..31, stack
// size n known per handler: every stack slot is a register named at compile
// time) and each handler stores the local partial derivatives the reverse
// sweep will need, not its output: binary *, / and reversed / two entries
// (d/da, d/db), unary operators one (sin x takes cos x from its own
// reduction), fused VAR *, / one, fused CONST *, / one (d/dc) and reversed /
// two, every other word none.  Entries are appended in word order, so the
// reverse sweep, walking the words backwards, takes them from the end with a
// wave-uniform counter.  The reverse handler of a word (aux bits 24..31) is a
// linear update of the adjoint stack A:
//   binary at n    A[n-1] = A[n-2] d/db,  A[n-2] = A[n-2] d/da
//   unary, fused   A[n-1] scaled by d/dtop
//   CONST          its slot's gradient gains A (times d/dc when fused)
// A subtree without CONST words adds to no gradient: its words store no
// entries (their own forward handlers), and the reverse sweep follows a
// per-word "next" index (aux bits 0..7) that skips such a subtree in one
// step, and skips the words whose reverse update is the identity.
// The tape is one register array per case (list 3: two, entries 0..31 and
// 32..63; an index addresses at most a 32-entry array).
constexpr int GK = 2;
static_assert(GRAD_TILE_CASES % (GK * 64) == 0, "adjoint chunks hold whole tiles");

template <bool COS>
__device__ __forceinline__ void trig2(float& a, float& b) {
  float v[GK] = {a, b};
  trig_tile<COS, GK>(v);
  a = v[0];
  b = v[1];
}

// entry e of case k's tape: lo[e] for e < 32, hi[e - 32] above (HI = 0: no
// upper part)
template <int HI>
struct DTape {
  static constexpr int HS = HI > 0 ? HI : 1;
};

template <int HI>
__device__ __forceinline__ void dt_put(float (&lo0)[32], float (&lo1)[32], float (&hi0)[DTape<HI>::HS],
                                       float (&hi1)[DTape<HI>::HS], int e, float v0, float v1) {
  if (HI == 0 || e < 32) {
    lo0[e & 31] = v0;
    lo1[e & 31] = v1;
  } else {
    hi0[(e - 32) & (DTape<HI>::HS - 1)] = v0;
    hi1[(e - 32) & (DTape<HI>::HS - 1)] = v1;
  }
}

template <int HI>
__device__ __forceinline__ float dt_get(const float (&lo)[32], const float (&hi)[DTape<HI>::HS], int e) {
  if constexpr (HI == 0) {
    return lo[e & 31];
  } else {
    const float x = opaque(lo[e & 31]);
    const float y = opaque(hi[(e - 32) & (HI - 1)]);
    return e < 32 ? x : y;
  }
}

// one forward word (forward handler fid); e = the next free tape entry
template <int HI>
__device__ __forceinline__ void dt_fwd(uint32_t fid, float cv, float x0, float x1, float (&st)[GK][4],
                                       float (&lo0)[32], float (&lo1)[32], float (&hi0)[DTape<HI>::HS],
                                       float (&hi1)[DTape<HI>::HS], int& e) {
#define BGL_PUT(V0, V1)                        \
  dt_put<HI>(lo0, lo1, hi0, hi1, e, V0, V1);   \
  ++e;
  switch (fid) {
#define BGL_F_PUSH(N)     \
  case I0_PUSH_VAR + N:   \
    st[0][N] = x0;        \
    st[1][N] = x1;        \
    break;                \
  case I0_PUSH_CONST + N: \
    st[0][N] = cv;        \
    st[1][N] = cv;        \
    break;
    BGL_F_PUSH(0) BGL_F_PUSH(1) BGL_F_PUSH(2) BGL_F_PUSH(3)
#undef BGL_F_PUSH
#define BGL_F_BIN(O, N)                                                   \
  case I0_BIN + 3 * O + (N - 2): {                                        \
    const float a0 = st[0][N - 2], b0 = st[0][N - 1];                     \
    const float a1 = st[1][N - 2], b1 = st[1][N - 1];                     \
    st[0][N - 2] = gbinop<O>(a0, b0);                                     \
    st[1][N - 2] = gbinop<O>(a1, b1);                                     \
    if constexpr (O == B_MUL || O == B_DIV || O == B_RDIV) {              \
      float dA0, dB0, dA1, dB1;                                           \
      dbinop<O>(a0, b0, dA0, dB0);                                        \
      dbinop<O>(a1, b1, dA1, dB1);                                        \
      BGL_PUT(dA0, dA1)                                                   \
      BGL_PUT(dB0, dB1)                                                   \
    }                                                                     \
    break;                                                                \
  }
#define BGL_F_BIN3(O) BGL_F_BIN(O, 2) BGL_F_BIN(O, 3) BGL_F_BIN(O, 4)
    BGL_F_BIN3(B_ADD) BGL_F_BIN3(B_SUB) BGL_F_BIN3(B_MUL) BGL_F_BIN3(B_DIV) BGL_F_BIN3(B_RSUB) BGL_F_BIN3(B_RDIV)
#undef BGL_F_BIN3
#undef BGL_F_BIN
#define BGL_F_UN(N)                                                           \
  case I0_UN + 0 * 4 + (N - 1): {                                             \
    float s[GK] = {st[0][N - 1], st[1][N - 1]}, c[GK];                        \
    sincos_tile<GK>(s, c);                                                    \
    st[0][N - 1] = s[0];                                                      \
    st[1][N - 1] = s[1];                                                      \
    BGL_PUT(c[0], c[1])                                                       \
    break;                                                                    \
  }                                                                           \
  case I0_UN + 1 * 4 + (N - 1): {                                             \
    float d0 = st[0][N - 1], d1 = st[1][N - 1];                               \
    trig2<true>(st[0][N - 1], st[1][N - 1]);                                  \
    trig2<false>(d0, d1);                                                     \
    BGL_PUT(-d0, -d1)                                                         \
    break;                                                                    \
  }                                                                           \
  case I0_UN + 2 * 4 + (N - 1): {                                             \
    const float u0 = st[0][N - 1], u1 = st[1][N - 1];                         \
    st[0][N - 1] = op_exp(u0);                                                \
    st[1][N - 1] = op_exp(u1);                                                \
    BGL_PUT(dunary(2u, u0, st[0][N - 1]), dunary(2u, u1, st[1][N - 1]))       \
    break;                                                                    \
  }                                                                           \
  case I0_UN + 3 * 4 + (N - 1): {                                             \
    const float u0 = st[0][N - 1], u1 = st[1][N - 1];                         \
    st[0][N - 1] = op_log(u0);                                                \
    st[1][N - 1] = op_log(u1);                                                \
    BGL_PUT(dunary(3u, u0, 0.0f), dunary(3u, u1, 0.0f))                       \
    break;                                                                    \
  }                                                                           \
  case I0_UN + 4 * 4 + (N - 1): {                                             \
    const float u0 = st[0][N - 1], u1 = st[1][N - 1];                         \
    st[0][N - 1] = op_sqrt(u0);                                               \
    st[1][N - 1] = op_sqrt(u1);                                               \
    BGL_PUT(dunary(4u, u0, st[0][N - 1]), dunary(4u, u1, st[1][N - 1]))       \
    break;                                                                    \
  }
    BGL_F_UN(1) BGL_F_UN(2) BGL_F_UN(3) BGL_F_UN(4)
#undef BGL_F_UN
#define BGL_F_FUSED(O, N)                                                 \
  case I0_FUSED + 3 * O + (N - 1): {                                      \
    const float a0 = st[0][N - 1], a1 = st[1][N - 1];                     \
    st[0][N - 1] = gbinop<O>(a0, x0);                                     \
    st[1][N - 1] = gbinop<O>(a1, x1);                                     \
    if constexpr (O == B_MUL || O == B_DIV || O == B_RDIV) {              \
      float dA0, dB0, dA1, dB1;                                           \
      dbinop<O>(a0, x0, dA0, dB0);                                        \
      dbinop<O>(a1, x1, dA1, dB1);                                        \
      BGL_PUT(dA0, dA1)                                                   \
    }                                                                     \
    break;                                                                \
  }                                                                       \
  case I0_FUSED + 3 * (6 + O) + (N - 1): {                                \
    const float a0 = st[0][N - 1], a1 = st[1][N - 1];                     \
    st[0][N - 1] = gbinop<O>(a0, cv);                                     \
    st[1][N - 1] = gbinop<O>(a1, cv);                                     \
    if constexpr (O == B_MUL || O == B_DIV || O == B_RDIV) {              \
      float dA0, dB0, dA1, dB1;                                           \
      dbinop<O>(a0, cv, dA0, dB0);                                        \
      dbinop<O>(a1, cv, dA1, dB1);                                        \
      if constexpr (O == B_RDIV) {                                        \
        BGL_PUT(dA0, dA1)                                                 \
      }                                                                   \
      BGL_PUT(dB0, dB1)                                                   \
    }                                                                     \
    break;                                                                \
  }
#define BGL_F_FUSED3(O) BGL_F_FUSED(O, 1) BGL_F_FUSED(O, 2) BGL_F_FUSED(O, 3)
    BGL_F_FUSED3(B_ADD) BGL_F_FUSED3(B_SUB) BGL_F_FUSED3(B_MUL) BGL_F_FUSED3(B_DIV) BGL_F_FUSED3(B_RSUB)
    BGL_F_FUSED3(B_RDIV)
#undef BGL_F_FUSED3
#undef BGL_F_FUSED
    // constant-free words: values only
#define BGL_N_BIN(J, O, N)                                \
  case F_BIN_NT + 3 * J + (N - 2):                        \
    st[0][N - 2] = gbinop<O>(st[0][N - 2], st[0][N - 1]); \
    st[1][N - 2] = gbinop<O>(st[1][N - 2], st[1][N - 1]); \
    break;
#define BGL_N_BIN3(J, O) BGL_N_BIN(J, O, 2) BGL_N_BIN(J, O, 3) BGL_N_BIN(J, O, 4)
    BGL_N_BIN3(0, B_MUL) BGL_N_BIN3(1, B_DIV) BGL_N_BIN3(2, B_RDIV)
#undef BGL_N_BIN3
#undef BGL_N_BIN
#define BGL_N_UN(N)                                         \
  case F_UN_NT + 0 * 4 + (N - 1):                           \
    trig2<false>(st[0][N - 1], st[1][N - 1]);               \
    break;                                                  \
  case F_UN_NT + 1 * 4 + (N - 1):                           \
    trig2<true>(st[0][N - 1], st[1][N - 1]);                \
    break;                                                  \
  case F_UN_NT + 2 * 4 + (N - 1):                           \
    st[0][N - 1] = op_exp(st[0][N - 1]);                    \
    st[1][N - 1] = op_exp(st[1][N - 1]);                    \
    break;                                                  \
  case F_UN_NT + 3 * 4 + (N - 1):                           \
    st[0][N - 1] = op_log(st[0][N - 1]);                    \
    st[1][N - 1] = op_log(st[1][N - 1]);                    \
    break;                                                  \
  case F_UN_NT + 4 * 4 + (N - 1):                           \
    st[0][N - 1] = op_sqrt(st[0][N - 1]);                   \
    st[1][N - 1] = op_sqrt(st[1][N - 1]);                   \
    break;
    BGL_N_UN(1) BGL_N_UN(2) BGL_N_UN(3) BGL_N_UN(4)
#undef BGL_N_UN
#define BGL_N_FV(J, O, N)                                 \
  case F_FV_NT + 3 * J + (N - 1):                         \
    st[0][N - 1] = gbinop<O>(st[0][N - 1], x0);           \
    st[1][N - 1] = gbinop<O>(st[1][N - 1], x1);           \
    break;
#define BGL_N_FV3(J, O) BGL_N_FV(J, O, 1) BGL_N_FV(J, O, 2) BGL_N_FV(J, O, 3)
    BGL_N_FV3(0, B_MUL) BGL_N_FV3(1, B_DIV) BGL_N_FV3(2, B_RDIV)
#undef BGL_N_FV3
#undef BGL_N_FV
    default:
      break;
  }
#undef BGL_PUT
}

// slot arg (< GRAD_LANE_SLOTS) of the lane's gradient sums gains the two
// cases' contributions: an LDS add without a returned value, so nothing waits
// for it, and the adds of one lane reach its slot in program order
__device__ __forceinline__ void add_const_grad(uint32_t arg, float g0, float g1, bool v0, bool v1, double* lg) {
  const double v = (v0 ? double(g0) : 0.0) + (v1 ? double(g1) : 0.0);
  __hip_atomic_fetch_add(lg + arg * 64, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <int HI>  // upper tape entries per case (0: at most 32 entries)
__device__ void dtape_item(const GradArgs& a, int p, int c, float* lds) {
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
  // LDS: input tile [D][GK][64] | lane gradients [LANE_SLOTS][64] doubles
  // (the program has at most LANE_SLOTS constant slots)
  float* xl = lds + lane;
  double* lg = reinterpret_cast<double*>(lds + a.D * GK * 64) + lane;
  float lo0[32], lo1[32], hi0[DTape<HI>::HS], hi1[DTape<HI>::HS];
  for (int j = 0; j < LANE_SLOTS; ++j) lg[j * 64] = 0.0;
  __builtin_amdgcn_wave_barrier();
  double s_mse = 0.0;
  const float inv2m = float(2.0 / double(a.M));
  const int64_t c0 = int64_t(c) * a.chunk;
  const int64_t c1 = c0 + a.chunk < a.M ? c0 + a.chunk : a.M;
  for (int64_t base = c0; base < c1; base += GK * 64) {
    const int64_t i0 = base + lane, i1 = base + 64 + lane;
    const bool v0 = i0 < a.M, v1 = i1 < a.M;
    for (int d = 0; d < a.D; ++d) {
      if (!((vmask >> d) & 1u)) continue;
      const float x0 = a.Xt[int64_t(d) * a.Mp + i0];
      const float x1 = a.Xt[int64_t(d) * a.Mp + i1];
      xl[(d * GK) * 64] = x0;
      xl[(d * GK + 1) * 64] = x1;
    }
    const float y0 = a.yp[i0], y1 = a.yp[i1];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the tile is in LDS
    // ---- forward: values on the stack, partial derivatives on the tape
    float st[GK][4];
#pragma unroll
    for (int k = 0; k < GK; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) st[k][j] = 0.0f;
    // The input row a word reads is loaded one word ahead, so that the LDS
    // latency overlaps the previous word; words that read no input load row
    // min(arg, D - 1), which is in the tile and unused.
    const float* xt = lds + lane;
    int e = 0;
    uint32_t w = __builtin_amdgcn_readlane(va, 0);
    float xa0 = xt[xrow(w) * (GK * 64)], xa1 = xt[xrow(w) * (GK * 64) + 64];
    for (int t = 0; t < L; ++t) {
      const uint32_t wn = t + 1 < L ? __builtin_amdgcn_readlane(va, t + 1) : 0u;
      const float xb0 = xt[xrow(wn) * (GK * 64)], xb1 = xt[xrow(wn) * (GK * 64) + 64];
      const float cv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t));
      dt_fwd<HI>((w >> 8) & 0xFFu, cv, xa0, xa1, st, lo0, lo1, hi0, hi1, e);
      w = wn;
      xa0 = xb0;
      xa1 = xb1;
    }
    // ---- seed and fitness terms
    const double e0 = double(st[0][0]) - double(y0), e1 = double(st[1][0]) - double(y1);
    s_mse += (v0 ? e0 * e0 : 0.0) + (v1 ? e1 * e1 : 0.0);
    float A[GK][4];
#pragma unroll
    for (int k = 0; k < GK; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) A[k][j] = 0.0f;
    A[0][0] = v0 ? float(e0) * inv2m : 0.0f;
    A[1][0] = v1 ? float(e1) * inv2m : 0.0f;
    // ---- reverse: linear updates of the adjoint stack, visiting only the
    // words that are neither constant-free nor NOP (the root always)
    auto T0 = [&](int i) { return dt_get<HI>(lo0, hi0, i); };
    auto T1 = [&](int i) { return dt_get<HI>(lo1, hi1, i); };
    for (int t = L - 1; t >= 0;) {
      const uint32_t x = __builtin_amdgcn_readlane(va, t);
      const uint32_t rid = x >> 24;
      const uint32_t arg = (x >> 16) & 0xFFu;
      const float cv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), t));
      t = int(x & 0xFFu) - 1;
#define BGL_CG(G0, G1) add_const_grad(arg, G0, G1, v0, v1, lg);
      switch (rid) {
#define BGL_R_PUSH(N)             \
  case R_PUSH_CONST + N:          \
    BGL_CG(A[0][N], A[1][N]) break;
        BGL_R_PUSH(0) BGL_R_PUSH(1) BGL_R_PUSH(2) BGL_R_PUSH(3)
#undef BGL_R_PUSH
#define BGL_R_BIN(N)                              \
  case R_BIN_ADD + (N - 2):                       \
    A[0][N - 1] = A[0][N - 2];                    \
    A[1][N - 1] = A[1][N - 2];                    \
    break;                                        \
  case R_BIN_SUB + (N - 2):                       \
    A[0][N - 1] = -A[0][N - 2];                   \
    A[1][N - 1] = -A[1][N - 2];                   \
    break;                                        \
  case R_BIN_RSUB + (N - 2):                      \
    A[0][N - 1] = A[0][N - 2];                    \
    A[1][N - 1] = A[1][N - 2];                    \
    A[0][N - 2] = -A[0][N - 2];                   \
    A[1][N - 2] = -A[1][N - 2];                   \
    break;                                        \
  case R_BIN_GEN + (N - 2):                       \
    e -= 2;                                       \
    A[0][N - 1] = A[0][N - 2] * T0(e + 1);        \
    A[1][N - 1] = A[1][N - 2] * T1(e + 1);        \
    A[0][N - 2] *= T0(e);                         \
    A[1][N - 2] *= T1(e);                         \
    break;
        BGL_R_BIN(2) BGL_R_BIN(3) BGL_R_BIN(4)
#undef BGL_R_BIN
#define BGL_R_UN(N)       \
  case R_UN + (N - 1):    \
    e -= 1;               \
    A[0][N - 1] *= T0(e); \
    A[1][N - 1] *= T1(e); \
    break;
        BGL_R_UN(1) BGL_R_UN(2) BGL_R_UN(3) BGL_R_UN(4)
#undef BGL_R_UN
#define BGL_R_FUSED(N)                                             \
  case R_FV_RSUB + (N - 1):                                        \
    A[0][N - 1] = -A[0][N - 1];                                    \
    A[1][N - 1] = -A[1][N - 1];                                    \
    break;                                                         \
  case R_FV_GEN + (N - 1):                                         \
    e -= 1;                                                        \
    A[0][N - 1] *= T0(e);                                          \
    A[1][N - 1] *= T1(e);                                          \
    break;                                                         \
  case R_FC_ADD + (N - 1):                                         \
    BGL_CG(A[0][N - 1], A[1][N - 1]) break;                        \
  case R_FC_SUB + (N - 1):                                         \
    BGL_CG(-A[0][N - 1], -A[1][N - 1]) break;                      \
  case R_FC_RSUB + (N - 1):                                        \
    BGL_CG(A[0][N - 1], A[1][N - 1])                               \
    A[0][N - 1] = -A[0][N - 1];                                    \
    A[1][N - 1] = -A[1][N - 1];                                    \
    break;                                                         \
  case R_FC_MUL + (N - 1):                                         \
    e -= 1;                                                        \
    BGL_CG(A[0][N - 1] * T0(e), A[1][N - 1] * T1(e))               \
    A[0][N - 1] *= cv;                                             \
    A[1][N - 1] *= cv;                                             \
    break;                                                         \
  case R_FC_DIV + (N - 1): {                                       \
    e -= 1;                                                        \
    BGL_CG(A[0][N - 1] * T0(e), A[1][N - 1] * T1(e))               \
    float dA, dB;                                                  \
    dbinop<B_DIV>(0.0f, cv, dA, dB);                               \
    A[0][N - 1] *= dA;                                             \
    A[1][N - 1] *= dA;                                             \
    break;                                                         \
  }                                                                \
  case R_FC_RDIV + (N - 1):                                        \
    e -= 2;                                                        \
    BGL_CG(A[0][N - 1] * T0(e + 1), A[1][N - 1] * T1(e + 1))       \
    A[0][N - 1] *= T0(e);                                          \
    A[1][N - 1] *= T1(e);                                          \
    break;
        BGL_R_FUSED(1) BGL_R_FUSED(2) BGL_R_FUSED(3)
#undef BGL_R_FUSED
#undef BGL_CG
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

// LIST 2, 3, 4: at most GRAD_DTAPE_SMALL, MID, LARGE entries per case (upper
// tape 0, 16, 32 entries; 128, <= 168 and <= 256 VGPRs: 4, 3, 2 waves per
// SIMD).
template <int LIST>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LIST == 2 ? 4 : 1)))
k_grad_dtape(GradArgs a) {
  extern __shared__ float lds[];
  constexpr int HI = (LIST == 2 ? GRAD_DTAPE_SMALL : LIST == 3 ? GRAD_DTAPE_MID : GRAD_DTAPE_LARGE) - 32;
  const int32_t count = a.list_count[LIST];
  const int64_t items = int64_t(count) * a.n_chunks;
  const int32_t* list = a.list + LIST * int64_t(a.n_programs);
  for (;;) {
    unsigned long long it = 0;
    if (threadIdx.x == 0) it = atomicAdd(a.work + LIST, 1ull);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(it));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(it >> 32));
    const int64_t item = int64_t((uint64_t(hi) << 32) | lo);
    if (item >= items) break;
    const int c = int(item / count);
    const int p = list[item % count];
    dtape_item<HI>(a, p, c, lds);
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
  const size_t l2 = size_t(a.D) * GK * 64 * sizeof(float) + size_t(LANE_SLOTS) * 64 * sizeof(double);
  int nb0 = 0, nb1 = 0, nb2 = 0, nb3 = 0, nb4 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb0, k_grad<false>, 64, l0) != hipSuccess || nb0 < 1) nb0 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, k_grad<true>, 64, l1) != hipSuccess || nb1 < 1) nb1 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, k_grad_dtape<2>, 64, l2) != hipSuccess || nb2 < 1) nb2 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb3, k_grad_dtape<3>, 64, l2) != hipSuccess || nb3 < 1) nb3 = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb4, k_grad_dtape<4>, 64, l2) != hipSuccess || nb4 < 1) nb4 = 1;
  hipLaunchKernelGGL(k_grad_dtape<2>, dim3(nb2 * cus), dim3(64), l2, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_dtape<3>, dim3(nb3 * cus), dim3(64), l2, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_dtape<4>, dim3(nb4 * cus), dim3(64), l2, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad<false>, dim3(nb0 * cus), dim3(64), l0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad<true>, dim3(nb1 * cus), dim3(64), l1, s, a);
  return hipGetLastError();
}

}  // namespace bgl
