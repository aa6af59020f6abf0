// Generation step on the device: ramped half-and-half initialisation,
// tournament selection, subtree crossover and point mutation on postfix
// programs, driven by the Philox4x32-10 counter-based generator.
//
// One thread per child.  Child c's random words come from Philox with key =
// seed and counter (c, generation, block, tag); word j of the child's stream
// is word j % 4 of block j / 4, so every draw has a fixed position whatever
// operator the child ends up using, and children are independent of the
// order in which threads run.
#include "beagle_device.h"
#include "gen.h"

namespace bgl {

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------------
struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // round multipliers
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // key schedule (Weyl) increments
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint32_t hi0 = __umulhi(kM0, c0), lo0 = kM0 * c0;
    const uint32_t hi1 = __umulhi(kM1, c2), lo1 = kM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

struct Stream {
  uint32_t k0, k1, index, gen, tag;
  int blk = -1;
  U4 words;
  __device__ Stream(uint64_t seed, uint32_t index_, uint32_t gen_, uint32_t tag_)
      : k0(uint32_t(seed)), k1(uint32_t(seed >> 32)), index(index_), gen(gen_), tag(tag_) {}
  __device__ uint32_t draw(int j) {
    const int b = j >> 2;
    if (b != blk) {
      words = philox4x32_10(index, gen, uint32_t(b), tag, k0, k1);
      blk = b;
    }
    return words.v[j & 3];
  }
};

// integer in [0, n): multiply-high; unit float: 24 high bits
__device__ __forceinline__ uint32_t below(uint32_t u, uint32_t n) { return __umulhi(u, n); }
__device__ __forceinline__ double unit01(uint32_t u) { return double(u >> 8) * (1.0 / 16777216.0); }

// fp32(lo + (hi - lo) * unit), every step rounded in binary64 (no contraction)
__device__ __noinline__ float const_value(uint32_t u, float lo, float hi) {
#pragma clang fp contract(off)
  const double span = double(hi) - double(lo);
  const double prod = span * unit01(u);
  return float(double(lo) + prod);
}

// Zeroes elements [from, to) of a child slot: element stores up to the first
// 16-byte boundary, then 16-byte stores, then the tail (one thread writes a
// whole slot, so element-wide stores would each touch another cache line
// across the wave).
template <class T>
__device__ __forceinline__ void zero_fill(T* base, int from, int to) {
  constexpr int PER = 16 / int(sizeof(T));
  int i = from;
  while (i < to && (reinterpret_cast<uintptr_t>(base + i) & 15u) != 0) base[i++] = T(0);
  for (; i + PER <= to; i += PER) *reinterpret_cast<uint4*>(base + i) = make_uint4(0u, 0u, 0u, 0u);
  for (; i < to; ++i) base[i] = T(0);
}

// opcode of unary index u (0..4: SIN..SQRT, 5..11: SQUARE..TANH)
__device__ __forceinline__ uint32_t unary_opcode(uint32_t u) { return u < 5u ? OP_SIN + u : OP_SQUARE + (u - 5u); }

__device__ __forceinline__ int subtree_start(const uint16_t* tok, int i) {
  int need = 1;
  for (int j = i; j >= 0; --j) {
    need += arity(tok[j] & 0xFFu) - 1;
    if (need == 0) return j;
  }
  return 0;  // malformed parent: clamp (documented: parents must be valid)
}

// Appends parent tokens [from, to) to the child, renumbering constants.
struct ChildWriter {
  uint16_t* tok;
  float* cst;
  int len = 0;
  int ncst = 0;
  int max_consts;
  __device__ ChildWriter(uint16_t* t, float* c, int mc) : tok(t), cst(c), max_consts(mc) {}
  __device__ void put(uint32_t t, float cval) {
    if ((t & 0xFFu) == OP_CONST) {
      if (ncst < max_consts) {
        tok[len++] = uint16_t(OP_CONST | (uint32_t(ncst) << 8));
        cst[ncst++] = cval;
      } else {
        tok[len++] = uint16_t(OP_VAR);
      }
    } else {
      tok[len++] = uint16_t(t);
    }
  }
  __device__ void copy(const uint16_t* ptok, const float* pcst, int pcc, int from, int to) {
    for (int i = from; i < to; ++i) {
      const uint32_t t = ptok[i];
      const uint32_t a = t >> 8;
      put(t, ((t & 0xFFu) == OP_CONST && int(a) < pcc) ? pcst[a] : 0.0f);
    }
  }
};

__device__ __forceinline__ bool better(double fa, int ia, double fb, int ib) {
  // lower fitness wins; NaN loses to everything; ties -> lower index
  const bool na = isnan(fa), nb = isnan(fb);
  if (na != nb) return nb;
  if (!na && fa != fb) return fa < fb;
  return ia < ib;
}

__device__ __forceinline__ int tournament(Stream& s, int first_draw, int t, const double* fit, uint32_t N) {
  int best = int(below(s.draw(first_draw), N));
  double fb = fit[best];
  for (int k = 1; k < t; ++k) {
    const int e = int(below(s.draw(first_draw + k), N));
    const double fe = fit[e];
    if (better(fe, e, fb, best)) {
      best = e;
      fb = fe;
    }
  }
  return best;
}

__global__ void k_generation(GenStepArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  const int t = a.tournament;
  Stream s(a.seed, uint32_t(c), a.generation, a.tag);
  const double choice = unit01(s.draw(0));
  const uint32_t N = uint32_t(a.n_parents);
  int ia, ib;
  if (a.surv) {
    const int S = *a.n_surv;
    const uint32_t ua = below(s.draw(1), uint32_t(S > 0 ? S : N));
    const uint32_t ub = below(s.draw(1 + t), uint32_t(S > 0 ? S : N));
    ia = S > 0 ? a.surv[ua] : int(ua);
    ib = S > 0 ? a.surv[ub] : int(ub);
  } else {
    ia = tournament(s, 1, t, a.fitness, N);
    ib = tournament(s, 1 + t, t, a.fitness, N);
  }
  // (a regular layout gives the offsets without reading them)
  const bool reg = a.slots && a.slots[0] != 0;
  const int64_t oa = reg ? a.slots[1] + int64_t(ia) * a.slots[2] : a.tok_offset[ia];
  const int64_t ob = reg ? a.slots[1] + int64_t(ib) * a.slots[2] : a.tok_offset[ib];
  const int64_t coa = reg ? a.slots[3] + int64_t(ia) * a.slots[4] : a.const_offset[ia];
  const int64_t cob = reg ? a.slots[3] + int64_t(ib) * a.slots[4] : a.const_offset[ib];
  const int LA = a.tok_len[ia], LB = a.tok_len[ib];
  const int ca = a.const_count[ia], cb = a.const_count[ib];
  // a parent outside its arrays, empty or longer than a child slot gives an
  // empty child (parents are meant to be valid programs)
  auto usable = [&](int64_t o, int L, int64_t co, int cc) {
    return L > 0 && L <= a.max_len && o >= 0 && o + L <= a.n_tokens && cc >= 0 &&
           (cc == 0 || (co >= 0 && co + cc <= a.n_consts));
  };
  const bool okA = usable(oa, LA, coa, ca), okB = usable(ob, LB, cob, cb);
  const uint16_t* A = a.tokens + (okA ? oa : 0);
  const uint16_t* B = a.tokens + (okB ? ob : 0);
  const float* Ac = a.consts + (okA && ca > 0 ? coa : 0);
  const float* Bc = a.consts + (okB && cb > 0 ? cob : 0);
  const int xa = int(below(s.draw(2 * t + 1), uint32_t(okA ? LA : 0)));
  const int xb = int(below(s.draw(2 * t + 2), uint32_t(okB ? LB : 0)));
  const int mpos = int(below(s.draw(2 * t + 3), uint32_t(okA ? LA : 0)));
  const uint32_t msym = s.draw(2 * t + 4);
  const uint32_t mconst = s.draw(2 * t + 5);
  uint16_t* out = a.child_tokens + int64_t(c) * a.max_len;
  float* outc = a.child_consts + int64_t(c) * a.max_consts;
  ChildWriter w(out, outc, a.max_consts);
  const bool cross = choice < double(a.t_cross);
  if (!okA || (cross && !okB)) {
    // empty child
  } else if (cross) {
    const int sa = subtree_start(A, xa);
    const int sb = subtree_start(B, xb);
    const int len = LA - (xa - sa + 1) + (xb - sb + 1);
    if (len > a.max_len) {
      w.copy(A, Ac, ca, 0, LA);
    } else {
      w.copy(A, Ac, ca, 0, sa);
      w.copy(B, Bc, cb, sb, xb + 1);
      w.copy(A, Ac, ca, xa + 1, LA);
    }
  } else if (choice < double(a.t_mut)) {
    const uint32_t old = A[mpos] & 0xFFu;
    const int ar = arity(old);
    uint32_t repl;
    float rval = 0.0f;
    if (ar == 2) {
      repl = below(msym, 4);  // ADD, SUB, MUL, DIV
    } else if (ar == 1) {
      repl = unary_opcode(below(msym, uint32_t(a.n_unary)));
    } else {
      const uint32_t sym = below(msym, uint32_t(a.D + 1));
      if (int(sym) < a.D) {
        repl = OP_VAR | (sym << 8);
      } else {
        int others = 0;
        for (int i = 0; i < LA; ++i) others += (i != mpos && (A[i] & 0xFFu) == OP_CONST) ? 1 : 0;
        if (others < a.max_consts) {
          repl = OP_CONST;
          rval = const_value(mconst, a.const_lo, a.const_hi);
        } else {
          repl = OP_VAR;
        }
      }
    }
    w.copy(A, Ac, ca, 0, mpos);
    w.put(repl, rval);
    w.copy(A, Ac, ca, mpos + 1, LA);
  } else {
    w.copy(A, Ac, ca, 0, LA);
  }
  zero_fill(out, w.len, a.max_len);
  zero_fill(outc, w.ncst, a.max_consts);
  a.child_len[c] = w.len;
  a.child_const_count[c] = w.ncst;
}

// ---- microcosm selection ----------------------------------------------------
// A random sample of the population, ranked in one workgroup, gives the
// fitness threshold at the keep quantile; every individual at least that
// good survives, compacted in index order (per-block counts, one scan, a
// scatter), and the children draw their parents uniformly from the
// survivors.  Sort order of the sample: lower fitness first, NaN last, ties
// by draw position; survival: fitness not NaN and <= tau (every non-NaN
// individual when tau is NaN).

__device__ __forceinline__ bool survives(double f, double tau) { return !isnan(f) && (isnan(tau) || f <= tau); }

// blockDim.x == MICRO_MAX_SAMPLE, one workgroup
__global__ void __launch_bounds__(MICRO_MAX_SAMPLE) k_micro_threshold(MicroArgs a) {
  __shared__ double f[MICRO_MAX_SAMPLE];
  const int j = threadIdx.x;
  if (j == 0 && a.slots) {
    // the layout of parents 0 and 1, tested on every parent by k_micro_count
    const int64_t t0 = a.tok_offset[0], c0 = a.const_offset[0];
    a.slots[0] = 1;
    a.slots[1] = t0;
    a.slots[2] = a.n > 1 ? a.tok_offset[1] - t0 : 0;
    a.slots[3] = c0;
    a.slots[4] = a.n > 1 ? a.const_offset[1] - c0 : 0;
  }
  if (j < a.sample) {
    Stream s(a.seed, MICRO_INDEX, a.generation, a.tag);
    f[j] = a.fitness[below(s.draw(j), uint32_t(a.n))];
  }
  __syncthreads();
  if (j >= a.sample) return;
  const double fj = f[j];
  const bool nj = isnan(fj);
  int rank = 0;
  for (int i = 0; i < a.sample; ++i) {
    const double fi = f[i];
    const bool ni = isnan(fi);
    const bool less = ni != nj ? nj : (!ni && fi != fj ? fi < fj : i < j);
    rank += less ? 1 : 0;
  }
  if (rank == a.k) *a.tau = fj;  // ranks are a permutation: exactly one writer
}

// survivors of block b (MICRO_BLOCK consecutive individuals), MICRO_BLOCK threads
__global__ void __launch_bounds__(MICRO_BLOCK) k_micro_count(MicroArgs a) {
  __shared__ int wave_n[MICRO_BLOCK / 64];
  const int64_t i = int64_t(blockIdx.x) * MICRO_BLOCK + threadIdx.x;
  const double tau = *a.tau;
  const bool keep = i < a.n && survives(a.fitness[i], tau);
  if (a.slots && i < a.n &&
      (a.tok_offset[i] != a.slots[1] + i * a.slots[2] || a.const_offset[i] != a.slots[3] + i * a.slots[4]))
    a.slots[0] = 0;  // (every writer stores the same value)
  const int n = __popcll(__builtin_amdgcn_ballot_w64(keep));
  if ((threadIdx.x & 63) == 0) wave_n[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < MICRO_BLOCK / 64; ++w) t += wave_n[w];
    a.block_off[blockIdx.x] = t;
  }
}

// exclusive prefix sums of the block counts in place, and the total; one
// workgroup of 1024 threads walking the counts 1024 at a time
__global__ void __launch_bounds__(1024) k_micro_scan(MicroArgs a) {
  __shared__ int wave_tot[16];
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int base = 0; base < a.n_blocks; base += 1024) {
    const int b = base + int(threadIdx.x);
    const int v = b < a.n_blocks ? a.block_off[b] : 0;
    // inclusive scan inside the wave
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wave_tot[w] = x;
    __syncthreads();
    const int carry = carry_s;
    int before = 0;
    for (int q = 0; q < w; ++q) before += wave_tot[q];
    if (b < a.n_blocks) a.block_off[b] = carry + before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = carry + before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.n_surv = carry_s;
}

__global__ void __launch_bounds__(MICRO_BLOCK) k_micro_scatter(MicroArgs a) {
  __shared__ int wave_n[MICRO_BLOCK / 64];
  const int64_t i = int64_t(blockIdx.x) * MICRO_BLOCK + threadIdx.x;
  const double tau = *a.tau;
  const bool keep = i < a.n && survives(a.fitness[i], tau);
  if (a.slots && i < a.n &&
      (a.tok_offset[i] != a.slots[1] + i * a.slots[2] || a.const_offset[i] != a.slots[3] + i * a.slots[4]))
    a.slots[0] = 0;  // (every writer stores the same value)
  const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
  if ((threadIdx.x & 63) == 0) wave_n[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  int at = a.block_off[blockIdx.x];
  for (int w = 0; w < int(threadIdx.x >> 6); ++w) at += wave_n[w];
  at += __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
  if (keep) a.surv[at] = int32_t(i);
}

__global__ void k_init_population(InitArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  const int n_depths = a.depth_max - a.depth_min + 1;
  const int depth = a.depth_min + c % n_depths;
  const bool full = ((c / n_depths) % 2) == 0;
  Stream s(a.seed, uint32_t(c), 0u, a.tag);
  int cursor = 0;
  uint16_t* out = a.tokens + int64_t(c) * a.max_len;
  float* outc = a.consts + int64_t(c) * a.max_consts;
  int len = 0, ncst = 0;
  // pre-order generation, post-order emission: frames of open functions
  struct Frame {
    uint8_t op, left, level;
  };
  Frame fr[MAX_INIT_DEPTH + 1];
  int sp = 0;
  int level = 0;
  const uint32_t n_fun = 4u + uint32_t(a.n_unary);
  for (;;) {
    bool term;
    uint32_t sym;
    if (level == depth) {
      term = true;
      sym = below(s.draw(cursor++), uint32_t(a.D + 1));
    } else if (full) {
      term = false;
      sym = below(s.draw(cursor++), n_fun);
    } else {
      const uint32_t v = below(s.draw(cursor++), n_fun + uint32_t(a.D + 1));
      term = v >= n_fun;
      sym = term ? v - n_fun : v;
    }
    if (!term) {
      // functions in the order ADD SUB MUL DIV, then the unary ones
      fr[sp].op = uint8_t(sym < 4u ? sym : unary_opcode(sym - 4u));
      fr[sp].left = uint8_t(arity(fr[sp].op));
      fr[sp].level = uint8_t(level);
      ++sp;
      ++level;
      continue;
    }
    if (int(sym) < a.D) {
      out[len++] = uint16_t(OP_VAR | (sym << 8));
    } else if (ncst < a.max_consts) {
      out[len++] = uint16_t(OP_CONST | (uint32_t(ncst) << 8));
      outc[ncst++] = const_value(s.draw(cursor++), a.const_lo, a.const_hi);
    } else {
      out[len++] = uint16_t(OP_VAR);
    }
    while (sp > 0) {
      Frame& f = fr[sp - 1];
      if (--f.left > 0) break;
      out[len++] = uint16_t(f.op);
      --sp;
    }
    if (sp == 0) break;
    level = fr[sp - 1].level + 1;
  }
  zero_fill(out, len, a.max_len);
  zero_fill(outc, ncst, a.max_consts);
  a.len[c] = len;
  a.const_count[c] = ncst;
}

}  // namespace bgl
