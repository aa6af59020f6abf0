// Program preparation (validation, Sethi-Ullman re-serialisation, decoding)
// and fitness-case staging.
#include <type_traits>

#include "beagle_device.h"
#include "grad.h"
#include "kernels.h"

namespace bgl {

// Per-token scratch of one program: an array of T with a stride (LDS
// arrays are interleaved across the workgroup's threads, so that
// neighbouring threads hit neighbouring banks).
template <class T, int STRIDE>
struct Scratch {
  T* p;
  __device__ __forceinline__ int get(int i) const { return int(p[i * STRIDE]); }
  __device__ __forceinline__ void set(int i, int v) const { p[i * STRIDE] = T(v); }
};

// One thread per program.  Three passes over the tokens, with per-token
// scratch (`stack`, `start`, `need`, the re-ordered program `ord` and a copy
// of the tokens `tok`):
//  1. forward: validate, and for every token record the start of its
//     subtree and its register need (Strahler number),
//  2. backward from the root: place every subtree in the output order
//     (operand with the larger need first) and write the re-ordered
//     (opcode, arg) at its output position,
//  3. forward over the output: track the stack size n before each token and
//     write the handler word; CONST values go to the side table cval.
// The forward handler of a word that stores no tape entries (a constant-free
// subtree's word) in the derivative-tape adjoint's numbering.
__device__ static uint32_t fwd_notape(uint32_t i0) {
  auto gen = [](uint32_t o) -> int { return o == B_MUL ? 0 : o == B_DIV ? 1 : o == B_RDIV ? 2 : -1; };
  if (i0 >= I0_UN && i0 < I0_FUSED) return F_UN_NT + (i0 - I0_UN);
  if (i0 >= I0_BIN && i0 < I0_UN) {
    const uint32_t q = i0 - I0_BIN;
    const int j = gen(q / 3u);
    return j >= 0 ? F_BIN_NT + 3u * uint32_t(j) + q % 3u : i0;
  }
  if (i0 >= I0_FUSED && i0 < I0_FUSED + 18u) {  // fused VAR words
    const uint32_t q = i0 - I0_FUSED;
    const int j = gen(q / 3u);
    return j >= 0 ? F_FV_NT + 3u * uint32_t(j) + q % 3u : i0;
  }
  return i0;
}

// Rewrites aux of a program of the derivative-tape adjoint (at most 64
// words; none of the value-tape kernels reads it) as
//   (next + 1) | (fid << 8) | (arg << 16) | (rid << 24):
// fid its forward handler (fwd_notape for constant-free words), arg its
// variable or constant slot, next the word the reverse sweep visits after
// it: the reverse sweep visits only words that are not constant-free and not
// NOP, and steps over a constant-free subtree in one jump.  wfirst holds,
// per word, the first word of its subtree (bit 15: constant-free); vis is
// scratch (the word to visit when the sweep arrives at word u, plus one).
template <class S>
__device__ static void dtape_words(const uint32_t* code, uint32_t* aux, int L, S vis, S wfirst) {
  for (int u = 0; u < L; ++u) {
    const int fw = wfirst.get(u);
    const bool wcf = (fw & 0x8000) != 0;
    const int sk = wcf ? (fw & 0x7FFF) - 1 : u - 1;
    const bool real = !wcf && (aux[u] >> 24) != R_NOP;
    vis.set(u, real ? u + 1 : (sk >= 0 ? vis.get(sk) : 0));
  }
  for (int u = 0; u < L; ++u) {
    const uint32_t c = code[u];
    const int fw = wfirst.get(u);
    const bool wcf = (fw & 0x8000) != 0;
    const int sk = wcf ? (fw & 0x7FFF) - 1 : u - 1;
    const uint32_t next1 = sk >= 0 ? uint32_t(vis.get(sk)) : 0u;
    const uint32_t fid = wcf ? fwd_notape(c >> 24) : (c >> 24);
    aux[u] = next1 | (fid << 8) | (((c >> 8) & 0xFFu) << 16) | (aux[u] & 0xFF000000u);
  }
}

// The lists a valid program joins: its register-need class and its adjoint
// list (-1: an invalid program joins none).
struct ListIds {
  int cls = -1, lc = -1;
  // the wave decoders' program header fields (ProgMeta): status | need << 8
  // | len << 16, and the variable mask (shift is 0 after decoding)
  int32_t head = 0;
  uint32_t vmask = 0u;
};

// Whether program p holds its token range (and, for the adjoint, its
// constant range) alone: always when the ranges are sorted and disjoint,
// else when every slot of its ranges carries its own index as the lowest
// covering one (see PrepareArgs::layout).
__device__ static bool owns_ranges(const PrepareArgs& a, int p, int64_t off, int32_t L, int64_t coff, int32_t cc) {
  if (!a.layout) return true;
  if (a.layout[0])
    for (int32_t i = 0; i < L; ++i)
      if (a.owner[off + i] != p) return false;
  if (a.adjoint && a.layout[1])
    for (int32_t j = 0; j < cc; ++j)
      if (a.cowner[coff + j] != p) return false;
  return true;
}

template <class ST, class S, class SO>
__device__ static ListIds prepare_program(const PrepareArgs& a, int p, ST tok, S stack, S start, S need, SO ord) {
  const int64_t off = a.tok_offset[p];
  const int32_t L = a.tok_len[p];
  const int64_t coff = a.const_offset[p];
  const int32_t cc = a.const_count[p];
  int status = BEAGLE_PROG_OK;
  int need_root = 0;
  int L_dec = 0;
  int n_ent = 0;  // derivative-tape entries per case (adjoint)
  uint32_t vmask = 0;
  bool ext = false;  // uses one of the further operators (SQUARE .. TANH)
  if (L <= 0) {
    status = L == 0 ? BEAGLE_PROG_EMPTY : BEAGLE_PROG_BAD_LAYOUT;
  } else if (L > MAX_LEN) {
    status = BEAGLE_PROG_TOO_LONG;
  } else if (off < 0 || off + L > a.n_tokens || cc < 0 ||
             (cc > 0 && (coff < 0 || coff + cc > a.n_consts))) {
    status = BEAGLE_PROG_BAD_LAYOUT;
  } else if (!owns_ranges(a, p, off, L, coff, cc)) {
    status = BEAGLE_PROG_BAD_LAYOUT;  // overlaps a lower-indexed program's range
  }
  if (status == BEAGLE_PROG_OK) {
    // stack: node stack in pass 1, output starts in pass 2
    int depth = 0;
    for (int i = 0; i < L; ++i) {
      const uint32_t t = uint32_t(tok.get(i));
      const uint32_t op = t & 0xFFu, arg = t >> 8;
      if (op >= N_OPCODES) { status = BEAGLE_PROG_BAD_OPCODE; break; }
      if (op == OP_VAR && int(arg) >= a.D) { status = BEAGLE_PROG_BAD_VAR; break; }
      if (op == OP_VAR) vmask |= 1u << arg;
      ext |= is_extended(op);
      if (op == OP_CONST && int(arg) >= cc) { status = BEAGLE_PROG_BAD_CONST; break; }
      const int ar = arity(op);
      if (depth < ar) { status = BEAGLE_PROG_UNDERFLOW; break; }
      if (ar == 0) {
        start.set(i, i);
        need.set(i, 1);
      } else if (ar == 1) {
        const int c = stack.get(depth - 1);
        start.set(i, start.get(c));
        need.set(i, need.get(c));
      } else {
        const int r = stack.get(depth - 1), l = stack.get(depth - 2);
        start.set(i, start.get(l));
        const int nl = need.get(l), nr = need.get(r);
        need.set(i, nl == nr ? nl + 1 : (nl > nr ? nl : nr));
      }
      depth += 1 - ar;
      stack.set(depth - 1, i);
    }
    if (status == BEAGLE_PROG_OK && depth != 1) status = BEAGLE_PROG_BAD_FINAL_DEPTH;
    if (status == BEAGLE_PROG_OK) {
      need_root = need.get(L - 1);
      uint32_t* code = a.code + off;
      // pass 2: output start of every subtree, root first
      const S ostart = stack;
      ostart.set(L - 1, 0);
      for (int i = L - 1; i >= 0; --i) {
        const uint32_t t = uint32_t(tok.get(i));
        uint32_t op = t & 0xFFu;
        const uint32_t arg = t >> 8;
        const int o = ostart.get(i);
        const int size = i - start.get(i) + 1;
        const int ar = arity(op);
        if (ar == 1) {
          ostart.set(i - 1, o);
        } else if (ar == 2) {
          const int r = i - 1, l = start.get(r) - 1;
          const int size_l = l - start.get(l) + 1;
          const int size_r = r - start.get(r) + 1;
          if (need.get(r) > need.get(l)) {
            ostart.set(r, o);
            ostart.set(l, o + size_r);
            op = op == OP_SUB ? 100u + B_RSUB : (op == OP_DIV ? 100u + B_RDIV : op);
          } else {
            ostart.set(l, o);
            ostart.set(r, o + size_l);
          }
        }
        ord.set(o + size - 1, int(op | (arg << 8)));
      }
      // pass 3: handler words, fusing "terminal, binary operator" pairs;
      // decoded words go to `code` (out <= i always, so `ord` may alias it).
      // Alongside, for the adjoint: aux[out] = pa | (rws << 16) | (rid << 24),
      // pa = the decoded word that produced the value below the top (binary
      // words), rws = the adjoint-stack slot the reverse sweep writes, rid =
      // the word's reverse handler in the derivative-tape adjoint, whose tape
      // entries per case are counted in n_ent (see grad.hip).  A word whose
      // subtree holds no CONST ("constant-free") needs no adjoint: it has no
      // entries and its rid is NOP.  `start` is free after pass 2 and holds
      // the producer of each stack slot, `need` the first decoded word of
      // each slot's subtree, `stack` per word the first word of its subtree
      // with bit 15 set when constant-free; cfm bit j: slot j constant-free.
      float* cv = a.cval + off;
      uint32_t* aux = a.aux + off;
      const S prod = start;
      const S pfirst = need;
      const S wfirst = stack;
      uint32_t cfm = 0u;
      int n = 0, nmax = 0, out = 0;
      for (int i = 0; i < L; ++i) {
        const uint32_t w = uint32_t(ord.get(i));
        const uint32_t op = w & 0xFFu, arg = (w >> 8) & 0xFFu;
        const uint32_t wslot = n > 0 ? uint32_t(n - 1) : 0u;
        uint32_t h, i0, pa = 0u, rws, rid;
        bool wcf;   // constant-free subtree
        int wfst;   // first word of the subtree
        int ent;    // derivative-tape entries when not constant-free
        const bool term = op == OP_VAR || op == OP_CONST;
        const uint32_t nxt = i + 1 < L ? (uint32_t(ord.get(i + 1)) & 0xFFu) : 0xFFu;
        const bool next_bin = nxt < 4u || (nxt >= 100u && nxt < 106u);
        if (term && n >= 1 && next_bin) {
          // the pushed value is the right operand of the next operator and
          // the current top its left one: top = top op value
          const uint32_t o = nxt >= 100u ? nxt - 100u : nxt;
          h = H_FUSED + 6u * (op == OP_CONST ? 1u : 0u) + o;
          i0 = n <= 3 ? I0_FUSED + 3u * (6u * (op == OP_CONST ? 1u : 0u) + o) + uint32_t(n - 1) : I0_NONE;
          if (op == OP_CONST) cv[out] = a.consts[coff + arg];
          nmax = n + 1 > nmax ? n + 1 : nmax;
          rws = uint32_t(n - 1);
          const bool gen = o == B_MUL || o == B_DIV || o == B_RDIV;
          if (op == OP_VAR) {
            rid = o == B_RSUB ? R_FV_RSUB : (gen ? R_FV_GEN : R_NOP);
            ent = gen ? 1 : 0;
          } else {
            const uint32_t fc[6] = {R_FC_ADD, R_FC_SUB, R_FC_MUL, R_FC_DIV, R_FC_RSUB, R_FC_RDIV};
            rid = fc[o];
            ent = o == B_RDIV ? 2 : (gen ? 1 : 0);
          }
          if (rid != R_NOP) rid = n <= 3 ? rid + uint32_t(n - 1) : R_NONE;
          wcf = op == OP_VAR && ((cfm >> (n - 1)) & 1u);
          wfst = pfirst.get(n - 1);
          cfm = wcf ? (cfm | (1u << (n - 1))) : (cfm & ~(1u << (n - 1)));
          prod.set(n - 1, out);
          ++i;  // the operator is consumed; stack size unchanged
        } else if (term) {
          h = op == OP_VAR ? H_VAR : H_CONST;
          i0 = n <= 3 ? (op == OP_VAR ? I0_PUSH_VAR : I0_PUSH_CONST) + uint32_t(n) : I0_NONE;
          if (op == OP_CONST) cv[out] = a.consts[coff + arg];
          rws = uint32_t(n);
          rid = op == OP_VAR ? R_NOP : (n <= 3 ? R_PUSH_CONST + uint32_t(n) : R_NONE);
          ent = 0;
          wcf = op == OP_VAR;
          wfst = out;
          if (n < 32) cfm = wcf ? (cfm | (1u << n)) : (cfm & ~(1u << n));
          if (n < MAX_STACK) pfirst.set(n, out);
          prod.set(n, out);
          ++n;
        } else if (op >= 100u || op < 4) {
          h = op >= 100u ? h_bin(op - 100u, n) : h_bin(op, n);  // ADD..DIV: BinIdx == opcode
          i0 = n <= 4 ? I0_BIN + 3u * (op >= 100u ? op - 100u : op) + uint32_t(n - 2) : I0_NONE;
          pa = uint32_t(prod.get(n - 2));
          rws = uint32_t(n - 2);
          const uint32_t bo = op >= 100u ? op - 100u : op;
          const uint32_t rb[6] = {R_BIN_ADD, R_BIN_SUB, R_BIN_GEN, R_BIN_GEN, R_BIN_RSUB, R_BIN_GEN};
          rid = n <= 4 ? rb[bo] + uint32_t(n - 2) : R_NONE;
          ent = rb[bo] == R_BIN_GEN ? 2 : 0;
          wcf = ((cfm >> (n - 2)) & 1u) && ((cfm >> (n - 1)) & 1u);
          wfst = pfirst.get(n - 2);
          cfm = wcf ? (cfm | (1u << (n - 2))) : (cfm & ~(1u << (n - 2)));
          --n;
          prod.set(n - 1, out);
        } else {
          const uint32_t u = unary_index(op);
          h = H_UN + u;
          i0 = n <= 4 && u < U_FIRST_EXT ? I0_UN + 4u * u + uint32_t(n - 1) : I0_NONE;
          rws = uint32_t(n - 1);
          rid = n <= 4 ? R_UN + uint32_t(n - 1) : R_NONE;
          ent = 1;
          wcf = (cfm >> (n - 1)) & 1u;
          wfst = pfirst.get(n - 1);
          prod.set(n - 1, out);
        }
        nmax = n > nmax ? n : nmax;
        // arg: variable index (VAR words), constant slot (CONST words), 0 otherwise
        const uint32_t warg = term ? arg : 0u;
        code[out] = h | (warg << 8) | (wslot << 16) | (i0 << 24);
        if (wcf)
          rid = R_NOP;
        else
          n_ent += ent;
        wfirst.set(out, wfst | (wcf ? 0x8000 : 0));
        if (a.adjoint) aux[out] = pa | (rws << 16) | (rid << 24);
        ++out;
      }
      // nmax == need_root by construction; the larger one is kept defensively
      need_root = nmax > need_root ? nmax : need_root;
      if (need_root > MAX_STACK || out > a.max_words) status = BEAGLE_PROG_TOO_LONG;
      L_dec = out;
    }
  }
  ProgMeta m;
  m.status = status;
  m.need = need_root;
  m.len = status == BEAGLE_PROG_OK ? L_dec : 0;
  m.shift = 0.0f;
  m.vmask = status == BEAGLE_PROG_OK ? vmask : 0u;
  a.meta[p] = m;
  if (a.status_out) a.status_out[p] = int8_t(status);
  ListIds ids;
  if (status == BEAGLE_PROG_OK) {
    // the list of its register-need class (list order does not affect any
    // result: every (program, chunk) partial has its own slot)
    ids.cls = need_class(need_root);
    // the further operators are compiled into the general-stack kernels only
    if (ext && ids.cls == 0) ids.cls = 1;
    // and by tape size (the adjoint keeps short tapes in registers)
    // adjoint lists: 0 short value tape, 1 long value tape; register need
    // <= 4 and at most GRAD_LANE_SLOTS constant slots: 2, 3, 4 at most
    // GRAD_DTAPE_SMALL, MID, LARGE derivative-tape entries
    const int lc = L_dec > a.short_words                          ? 1
                   : need_root > 4 || cc > GRAD_LANE_SLOTS || ext  ? 0
                   : n_ent <= GRAD_DTAPE_SMALL ? 2
                   : n_ent <= GRAD_DTAPE_MID   ? 3
                   : n_ent <= GRAD_DTAPE_LARGE ? 4
                                               : 0;
    if (a.adjoint && lc >= 2) dtape_words(a.code + off, a.aux + off, L_dec, need, stack);
    ids.lc = lc;
  }
  return ids;
}

// Appends every active lane's program p to list `which` (< NL) of
// count/list (lists `stride` apart), one atomic per list and wave: the lanes
// of one list take consecutive slots in lane order.  Every lane of the wave
// calls it.
template <int NL>
__device__ static void wave_append(int which, int p, int32_t* count, int32_t* list, int64_t stride) {
  const int lane = threadIdx.x & 63;
  for (int l = 0; l < NL; ++l) {
    const uint64_t m = __ballot(which == l);
    if (m == 0) continue;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    int base = 0;
    if (lane == leader) base = atomicAdd(count + l, __popcll(m));
    base = __shfl(base, leader, 64);
    if (which == l) list[int64_t(l) * stride + base + rank] = p;
  }
}

// The same appends for a whole workgroup of WAVES waves, one atomic per
// list and workgroup: a list's slots go to the waves in wave order and,
// within a wave, to the lanes in lane order.  Every thread of the
// workgroup calls it (it synchronises the workgroup twice).
template <int NL, int WAVES>
__device__ static void block_append(int which, int p, int32_t* count, int32_t* list, int64_t stride,
                                    int32_t (&cnt)[WAVES][8], int32_t (&base)[8]) {
  static_assert(NL <= 8, "at most 8 lists");
  const int lane = threadIdx.x & 63, w = int(threadIdx.x >> 6);
  int rank = 0;
  for (int l = 0; l < NL; ++l) {
    const uint64_t m = __ballot(which == l);
    if (which == l)
      rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    if (lane == 0) cnt[w][l] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < NL) {
    int total = 0;
    for (int v = 0; v < WAVES; ++v) total += cnt[v][threadIdx.x];
    base[threadIdx.x] = total > 0 ? atomicAdd(count + threadIdx.x, total) : 0;
  }
  __syncthreads();
  if (which >= 0 && which < NL) {
    int slot = base[which] + rank;
    for (int v = 0; v < w; ++v) slot += cnt[v][which];
    list[int64_t(which) * stride + slot] = p;
  }
}

// One program's list appends with one atomic each (the batched kernel:
// neighbouring lanes belong to different problems).
__device__ static void append_one(const PrepareArgs& a, int p, ListIds ids) {
  if (ids.cls < 0) return;
  const int slot = atomicAdd(a.class_count + ids.cls, 1);
  a.class_list[int64_t(ids.cls) * a.n_programs + slot] = p;
  if (!a.adjoint) return;
  const int ls = atomicAdd(a.len_count + ids.lc, 1);
  a.len_list[int64_t(ids.lc) * a.n_programs + ls] = p;
}

// The second decoding pass (k_prepare_long, and the batched kernel): programs
// of at most PREP_SHORT tokens keep their scratch in LDS (16-bit entries:
// token indices, needs and tokens all fit), longer ones in the global scratch
// arrays.  The first pass uses the narrow scratch below.
constexpr int PREP_BLOCK = 64;
constexpr int PREP_SHORT = 128;

struct PrepLds {
  static constexpr int SHORT = PREP_SHORT;
  using Index = Scratch<uint16_t, PREP_BLOCK>;
  uint16_t tok[PREP_SHORT * PREP_BLOCK];
  uint16_t stack[PREP_SHORT * PREP_BLOCK];
  uint16_t start[PREP_SHORT * PREP_BLOCK];
  uint16_t need[PREP_SHORT * PREP_BLOCK];
  uint16_t ord[PREP_SHORT * PREP_BLOCK];
};

// 8-bit index scratch for programs of at most PREP_NARROW tokens: every value
// the passes store is an index or count below 128, or such an index with the
// constant-free flag (bit 15), which is kept in bit 7 here.
template <int STRIDE>
struct Scratch8 {
  uint8_t* p;
  __device__ __forceinline__ int get(int i) const {
    const int b = p[i * STRIDE];
    return (b & 0x7F) | ((b & 0x80) << 8);
  }
  __device__ __forceinline__ void set(int i, int v) const { p[i * STRIDE] = uint8_t((v & 0x7F) | ((v >> 8) & 0x80)); }
};

// The scratch of the first decoding pass: 28 KB per workgroup instead of
// 80 KB, so five workgroups share a compute unit instead of two (the passes
// are latency-bound); longer programs go to k_prepare_long.
constexpr int PREP_NARROW = 64;
struct PrepLdsNarrow {
  static constexpr int SHORT = PREP_NARROW;
  using Index = Scratch8<PREP_BLOCK>;
  uint16_t tok[PREP_NARROW * PREP_BLOCK];
  uint8_t stack[PREP_NARROW * PREP_BLOCK];
  uint8_t start[PREP_NARROW * PREP_BLOCK];
  uint8_t need[PREP_NARROW * PREP_BLOCK];
  uint16_t ord[PREP_NARROW * PREP_BLOCK];
};

template <class LDS>
__device__ static ListIds prepare_one(const PrepareArgs& a, int p, LDS& lds) {
  const int64_t off = a.tok_offset[p];
  const int32_t L = a.tok_len[p];
  if (L >= 1 && L <= LDS::SHORT && off >= 0 && off + L <= a.n_tokens) {
    using SL = Scratch<uint16_t, PREP_BLOCK>;
    using SI = typename LDS::Index;
    const int t = threadIdx.x;
    // the tokens first, eight independent loads at a time
    const uint16_t* src = a.tokens + off;
    uint16_t* dst = lds.tok + t;
    int i = 0;
    for (; i + 8 <= L; i += 8) {
      uint16_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = src[i + j];
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[(i + j) * PREP_BLOCK] = v[j];
    }
    for (; i < L; ++i) dst[i * PREP_BLOCK] = src[i];
    return prepare_program(a, p, SL{lds.tok + t}, SI{lds.stack + t}, SI{lds.start + t}, SI{lds.need + t},
                           SL{lds.ord + t});
  } else {
    // (an invalid layout is reported before any scratch access)
    const int64_t o = off >= 0 && off < a.n_tokens ? off : 0;
    using SG = Scratch<int32_t, 1>;
    return prepare_program(a, p, Scratch<const uint16_t, 1>{a.tokens + o}, SG{a.scr_stack + o}, SG{a.scr_start + o},
                    SG{a.scr_need + o}, Scratch<uint32_t, 1>{a.code + o});
  }
}

// One thread per program, with the narrow LDS scratch; a program longer than
// PREP_NARROW tokens is not decoded here but appended to the long list for
// k_prepare_long (list order does not affect any result).
__global__ void __launch_bounds__(PREP_BLOCK) k_prepare(PrepareArgs a) {
  __shared__ PrepLdsNarrow lds;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  ListIds ids;
  bool defer = false;
  if (p < a.n_programs) {
    defer = a.tok_len[p] > PREP_NARROW;
    if (!defer) ids = prepare_one(a, p, lds);
  }
  // list appends aggregated per wave (per-program atomics on a handful of
  // counters serialise when the population is large)
  wave_append<1>(defer ? 0 : -1, p, a.long_count, a.long_list, 0);
  wave_append<N_CLASSES>(ids.cls, p, a.class_count, a.class_list, a.n_programs);
  if (a.adjoint) wave_append<GRAD_LISTS>(ids.lc, p, a.len_count, a.len_list, a.n_programs);
}

// The programs k_prepare deferred: a fixed grid striding over the long list
// with the wide LDS scratch (programs above PREP_SHORT tokens use the global
// scratch).  Exits at once when the list is empty.
__global__ void __launch_bounds__(PREP_BLOCK) k_prepare_long(PrepareArgs a) {
  __shared__ PrepLds lds;
  const int32_t n = *a.long_count;
  for (int32_t base = blockIdx.x * PREP_BLOCK; base < n; base += gridDim.x * PREP_BLOCK) {
    const int32_t item = base + int32_t(threadIdx.x);
    ListIds ids;
    int p = 0;
    if (item < n) {
      p = a.long_list[item];
      ids = prepare_one(a, p, lds);
    }
    wave_append<N_CLASSES>(ids.cls, p, a.class_count, a.class_list, a.n_programs);
    if (a.adjoint) wave_append<GRAD_LISTS>(ids.lc, p, a.len_count, a.len_list, a.n_programs);
  }
}

// ---- wave-per-program decoding ---------------------------------------------
// The same decoding (statuses, words, side tables, metadata, list
// membership -- bit for bit) for a program of at most 64 tokens, with the
// program's tokens spread over one wave's lanes (lane i holds token i) and
// every sequential pass replaced by prefix sums and pointer chasing across
// lanes, so a program costs a few hundred wave instructions whatever its
// shape and no lane waits on another program's length.
//  - depth after each token: a prefix sum of (1 - arity); the first faulty
//    token (in token order) decides the status, as in the serial passes;
//  - subtree start s_i of each token: one past the last earlier position
//    whose depth is below token i's (found by a binary descent over the
//    minima of power-of-two windows);
//  - register need: repeated bottom-up relaxation (one round per tree
//    level);
//  - output position: each child learns from its parent (through LDS)
//    whether it is placed second and behind how many tokens; the offsets
//    are summed to the root by pointer jumping;
//  - words: the re-ordered tokens are gathered through LDS; stack sizes,
//    fused pairs and word indices are prefix sums; a word's producer and
//    first word, and whether its subtree is constant-free, are read at its
//    subtree's bounds.
namespace wdec {

__device__ __forceinline__ int lane_id() { return int(threadIdx.x & 63u); }
// v of lane src (0 <= src < 64 where the result is used)
__device__ __forceinline__ int from(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
// v of the lane CTRL names (a DPP row shift or broadcast), 0 where that
// lane is outside the row or the row is outside ROW_MASK
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, true); }
// Inclusive prefix sum over the 64 lanes (all active), register to
// register: row shifts by 1, 2, 4, 8 give each row of 16 its own prefix
// sums, then lane 15's total is added into rows 1 and 3 and lane 31's into
// rows 2 and 3.
__device__ __forceinline__ int scan_add(int v) {
  v += dpp<0x111, 0xF>(v);
  v += dpp<0x112, 0xF>(v);
  v += dpp<0x114, 0xF>(v);
  v += dpp<0x118, 0xF>(v);
  v += dpp<0x142, 0xA>(v);
  v += dpp<0x143, 0xC>(v);
  return v;
}
// Inclusive prefix maximum of non-negative values, the same pattern (zero
// never changes a result).
__device__ __forceinline__ int scan_max(int v) {
  v = max(v, dpp<0x111, 0xF>(v));
  v = max(v, dpp<0x112, 0xF>(v));
  v = max(v, dpp<0x114, 0xF>(v));
  v = max(v, dpp<0x118, 0xF>(v));
  v = max(v, dpp<0x142, 0xA>(v));
  v = max(v, dpp<0x143, 0xC>(v));
  return v;
}
// Bitwise OR over the 64 lanes, the same pattern, read from lane 63
// (uniform).
__device__ __forceinline__ uint32_t wave_or(uint32_t u) {
  int v = int(u);
  v |= dpp<0x111, 0xF>(v);
  v |= dpp<0x112, 0xF>(v);
  v |= dpp<0x114, 0xF>(v);
  v |= dpp<0x118, 0xF>(v);
  v |= dpp<0x142, 0xA>(v);
  v |= dpp<0x143, 0xC>(v);
  return uint32_t(__builtin_amdgcn_readlane(v, 63));
}
__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
// selections whose operands are evaluated first (a conditional expression
// with computed operands can become a lane-divergent branch)
template <class T>
__device__ __forceinline__ T sel(bool c, T a, T b) { return c ? a : b; }
template <class T>
__device__ __forceinline__ T pick4(int k, T a, T b, T c, T d) { return sel(k == 0, a, sel(k == 1, b, sel(k == 2, c, d))); }
__device__ __forceinline__ int lane_value(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

}  // namespace wdec

// Handlers of a decoded word by its kind.  Key k: a binary operator word
// (k = 0..3 and 18, 19 for ADD..DIV, RSUB, RDIV), a unary operator word (k =
// its opcode), a VAR or CONST push (9, 10), a fused pair (20 + 6 * [CONST] +
// the pair's binary operator).  Entry: the handler (bits 0..7, plus the stack
// size when bit 8 is set), the small-stack handler (bits 9..16 plus the stack
// size) for stack sizes below bits 17..19 (I0_NONE from there on).
__device__ static uint32_t word_entry(uint32_t k) {
  uint32_t h, step, i0, lim;
  if (k < 4u || k == 18u || k == 19u) {
    const uint32_t bo = k < 4u ? k : k - 14u;
    h = H_BIN + 15u * bo - 2u, step = 1u, i0 = I0_BIN + 3u * bo - 2u, lim = 5u;
  } else if (k == OP_VAR || k == OP_CONST) {
    h = k == OP_VAR ? H_VAR : H_CONST, step = 0u, i0 = k == OP_VAR ? I0_PUSH_VAR : I0_PUSH_CONST, lim = 4u;
  } else if (k < 20u) {
    const uint32_t u = unary_index(k);
    h = H_UN + u, step = 0u, i0 = I0_UN + 4u * u - 1u, lim = u < U_FIRST_EXT ? 5u : 0u;
  } else {
    const uint32_t f = k - 20u;  // 6 * [CONST] + operator
    h = H_FUSED + f, step = 0u, i0 = I0_FUSED + 3u * f - 1u, lim = 4u;
  }
  return h | (step << 8) | (i0 << 9) | (lim << 17);
}
// The word of an output token from its table key and the stack size n
// before it (the handler fields; operand and slot are added by the caller).
__device__ __forceinline__ uint32_t word_handlers(const uint32_t* wt, uint32_t key, uint32_t n) {
  const uint32_t te = wt[key & 31u];
  const uint32_t h = (te & 0xFFu) + ((te & 0x100u) ? n : 0u);
  const uint32_t i0 = n < (te >> 17) ? ((te >> 9) & 0xFFu) + n : I0_NONE;
  return h | (i0 << 24);
}

// Per-wave LDS of the wave decoder.
struct WaveDecLds {
  uint32_t a[64];
  uint32_t b[64];
  int32_t nd[68];  // register needs by lane; nd[NEED_ZERO] = 0
};
constexpr int NEED_ZERO = 64;

// Decodes program p (at most 64 tokens, its header fields given, uniform)
// with the calling wave; `tok` is the lane's token (lane < L, when the
// token range lies within the array; 0 otherwise).  Returns its lists
// (wave-uniform).
template <bool ADJ>
__device__ static ListIds decode_wave(const PrepareArgs& a, int p, int64_t off, int32_t L, int64_t coff, int32_t cc,
                                      int hstat, uint32_t tok, int lay_tok, int lay_const, WaveDecLds& sh,
                                      const uint32_t* wt) {
  using namespace wdec;
  const int lane = lane_id();
  // (hstat: the header's own checks, made before the call)
  int status = hstat;
  int need_root = 0, L_dec = 0;
  uint32_t vmask = 0;
  bool ext = false;
  if (status == BEAGLE_PROG_OK && (lay_tok | lay_const)) {
    // ranges not sorted and disjoint: every slot must carry p as its owner
    bool mine = true;
    if (lay_tok) mine = __builtin_amdgcn_ballot_w64(lane < L && a.owner[off + lane] != p) == 0;
    if (ADJ && mine && lay_const)
      for (int32_t j0 = 0; j0 < cc && mine; j0 += 64)
        mine = __builtin_amdgcn_ballot_w64(j0 + lane < cc && a.cowner[coff + j0 + lane] != p) == 0;
    if (!mine) status = BEAGLE_PROG_BAD_LAYOUT;
  }
  if (status == BEAGLE_PROG_OK) {
    const bool act = lane < L;
    const uint32_t t = act ? tok : 0u;
    const uint32_t op = t & 0xFFu, arg = t >> 8;
    const bool opok = op < N_OPCODES;
    // arity per opcode, 2 bits each (ADD..DIV 2, SIN..SQRT 1, VAR, CONST 0,
    // SQUARE..TANH 1)
    constexpr uint64_t ARITY = 0x5554155AAull;
    const int ar = opok ? int((ARITY >> (2u * op)) & 3u) : 0;
    // depth after each token
    const int d = scan_add(act ? 1 - ar : 0);
    // lanes holding a token (L <= 64 here); ballots of lane conditions are
    // masked with it and combined on the scalar side
    const uint64_t actm = L >= 64 ? ~0ull : (1ull << L) - 1ull;
    // faulty tokens: bad opcode, variable or constant slot out of range,
    // depth before < arity (underflow); the first one's code is decided from
    // its token on the scalar side, in that order of precedence
    const uint64_t em = (__builtin_amdgcn_ballot_w64(!opok) |
                         (__builtin_amdgcn_ballot_w64(op == OP_VAR) & __builtin_amdgcn_ballot_w64(int(arg) >= a.D)) |
                         (__builtin_amdgcn_ballot_w64(op == OP_CONST) & __builtin_amdgcn_ballot_w64(int(arg) >= cc)) |
                         __builtin_amdgcn_ballot_w64(d < 1)) &
                        actm;
    if (em) {
      const uint32_t tj = uint32_t(lane_value(int(t), first_lane(em)));
      const uint32_t opj = tj & 0xFFu, argj = tj >> 8;
      status = opj >= uint32_t(N_OPCODES)                  ? BEAGLE_PROG_BAD_OPCODE
               : (opj == OP_VAR) & (int(argj) >= a.D)      ? BEAGLE_PROG_BAD_VAR
               : (opj == OP_CONST) & (int(argj) >= cc)     ? BEAGLE_PROG_BAD_CONST
                                                           : BEAGLE_PROG_UNDERFLOW;
    } else if (lane_value(d, L - 1) != 1) {
      status = BEAGLE_PROG_BAD_FINAL_DEPTH;
    }
    if (status == BEAGLE_PROG_OK) {
      vmask = wave_or(act & (op == OP_VAR) ? 1u << arg : 0u);
      ext = (__builtin_amdgcn_ballot_w64(op - uint32_t(OP_SQUARE) < uint32_t(N_OPCODES - OP_SQUARE)) & actm) != 0;
      // ---- subtree starts: s = 1 + the last j < lane with d_j < d (d_{-1} = 0)
      int mn[6];
      mn[0] = d;
#pragma unroll
      for (int k = 1; k < 6; ++k) {
        // min over [max(0, lane - 2^k + 1), lane]: lanes below w read their
        // own value
        const int w = 1 << (k - 1);
        mn[k] = min(mn[k - 1], from(mn[k - 1], lane >= w ? lane - w : lane));
      }
      // descent: r moves down past windows [r - 2^k, r - 1] holding no
      // smaller depth; a window cut off at position 0 (mn[k] then covers
      // [0, r - 1]) leaves no earlier position, and r saturates at 0 (at r
      // = 0 the read lane is unused: any step leaves 0)
      uint32_t r = uint32_t(lane);
#pragma unroll
      for (int k = 5; k >= 0; --k) {
        const int v = __builtin_amdgcn_ds_bpermute(int(r << 2) - 4, mn[k]);
        r = __builtin_elementwise_sub_sat(r, sel(v >= d, 1u << k, 0u));
      }
      const int st = int(r);
      // ---- register need, bottom-up: leaves 1; unary: the child's;
      // binary: the larger child's, plus one when both are equal.  A need
      // not yet known is NEED_UNKNOWN or more (known ones are at most 7):
      // the larger-child rule then keeps it unknown without a test
      const int s_prev = from(st, lane > 0 ? lane - 1 : 0);  // start of the right operand
      const int lch = s_prev - 1;                              // left child (binary)
      constexpr int NEED_UNKNOWN = 1024;
      const bool is_un = ar == 1;
      // A unary operator's need is its operand's, and a run of unary
      // operators stands on consecutive tokens (postfix), so a child's need
      // is read at the bottom of its run: the last non-unary token at or
      // before it (bot: that token + 1).  The relaxation then steps over
      // binary levels only.
      const int bot = scan_max(is_un ? 0 : lane + 1);
      const int bot_r = max(from(bot, lane > 0 ? lane - 1 : 0) - 1, 0);
      const int bot_l = max(from(bot, lch > 0 ? lch : 0) - 1, 0);
      // The operands' needs are read from LDS, where slot NEED_ZERO holds 0:
      // a leaf reads (0, 0) and keeps 1, a unary operator (its operand's, 0)
      // and takes its operand's need -- one rule for every token, no
      // selection per round.
      const int src_r = sel(ar == 0, NEED_ZERO, bot_r);
      const int src_l = sel(ar == 2, bot_l, NEED_ZERO);
      if (lane == 0) sh.nd[NEED_ZERO] = 0;
      int need = ar == 0 ? 1 : NEED_UNKNOWN;
      int nr = 0, nl = 0;
      for (;;) {
        sh.nd[lane] = need;
        __builtin_amdgcn_wave_barrier();
        nr = sh.nd[src_r];
        nl = sh.nd[src_l];
        __builtin_amdgcn_wave_barrier();
        need = max(nl, nr) + int(nl == nr);
        if ((__builtin_amdgcn_ballot_w64(need >= 64) & actm) == 0) break;
      }
      need_root = lane_value(need, L - 1);
      // ---- output order: parents tell children their offset within the
      // parent's output range; the root's range starts at 0
      const bool swap = (ar == 2) & (nr > nl);
      const int size_r = lane - s_prev;  // binary: the right operand's size
      const int st_l = from(st, lch > 0 ? lch : 0);
      const int size_l = lch - st_l + 1;
      // (the parent's lane times 4 in bits 2..7: the byte address of a
      // lane read, with the offset from bit 8)
      if (act && ar >= 1) sh.a[lane - 1] = uint32_t(lane << 2) | (uint32_t(ar == 2 && !swap ? size_l : 0) << 8);
      if (act && ar == 2) sh.a[lch] = uint32_t(lane << 2) | (uint32_t(swap ? size_r : 0) << 8);
      if (lane == L - 1) sh.a[lane] = uint32_t(lane << 2);
      __builtin_amdgcn_wave_barrier();
      int pk = act ? int(sh.a[lane]) : lane << 2;  // parent * 4 | offset << 8
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        // (before the fifth and sixth rounds: done once every token's
        // pointer has reached the root -- trees under 16 or 32 levels)
        if (r >= 4 && (__builtin_amdgcn_ballot_w64((pk & 0xFC) != ((L - 1) << 2)) & actm) == 0) break;
        const int v = __builtin_amdgcn_ds_bpermute(pk & 0xFC, pk);
        pk = (pk & ~0xFC) + v;  // offsets add up, the parent pointer jumps
      }
      const int ostart = pk >> 8;
      const int oend = ostart + (lane - st);
      const uint32_t op2 = sel(swap & (op == OP_SUB), 100u + B_RSUB, sel(swap & (op == OP_DIV), 100u + B_RDIV, op));
      // (the token's arity rides along in bits 24..25)
      if (act) sh.b[oend] = op2 | (arg << 8) | (uint32_t(ostart) << 16) | (uint32_t(ar) << 24);
      __builtin_amdgcn_wave_barrier();
      const uint32_t e = act ? sh.b[lane] : 0x010000FFu;  // (no token: arity 1, stack unchanged)
      __builtin_amdgcn_wave_barrier();
      // ---- words, in output order (lane o holds output token o)
      const uint32_t o_op = e & 0xFFu, o_arg = (e >> 8) & 0xFFu;
      // a CONST word's value, loaded as soon as the slot is known (its
      // latency then overlaps the word's assembly; stored with the word)
      float cvv = 0.0f;
      if (o_op == OP_CONST) cvv = a.consts[coff + o_arg];
      const int o_st = int((e >> 16) & 0xFFu);  // start of its subtree
      const uint32_t o_ar = e >> 24;
      const bool o_bin = o_ar == 2u;
      const bool o_term = o_ar == 0u;  // VAR or CONST
      const int o_delta = 1 - int(o_ar);
      const int n_after = scan_add(o_delta);
      const int n = n_after - o_delta;  // stack size before the token
      const uint32_t nxt = uint32_t(from(int(o_op), lane < 63 ? lane + 1 : 63));
      // fused pairs: a terminal on a non-empty stack followed by a binary
      // operator; words: every token but such a terminal -- lane masks
      // combined on the scalar side, turned back into lane conditions by
      // inverse ballots (no VALU work)
      const uint64_t fm = __builtin_amdgcn_ballot_w64(o_term) & __builtin_amdgcn_ballot_w64(n >= 1) &
                          (__builtin_amdgcn_ballot_w64(nxt < 4u) | __builtin_amdgcn_ballot_w64(nxt - 100u < 6u)) &
                          (actm >> 1);
      const bool fused = __builtin_amdgcn_inverse_ballot_w64(fm);
      const uint64_t wm = actm & ~(fm << 1);
      const bool ws = __builtin_amdgcn_inverse_ballot_w64(wm);
      const int E = int(__builtin_amdgcn_mbcnt_hi(uint32_t(wm >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(wm), 0u)));
      const int widx = ws ? E : E - 1;  // word of each token (a fused pair's operator: the pair's word)
      L_dec = __popcll(wm);
      // the word's handler and small-stack handler: fused pair, terminal
      // push, binary operator, unary operator (all four computed, one
      // selection each: no branch per kind)
      const uint32_t un = uint32_t(n);
      const uint32_t ob = nxt >= 100u ? nxt - 100u : nxt;     // the fused pair's operator
      const uint32_t bo = o_op >= 100u ? o_op - 100u : o_op;  // a binary word's operator
      const bool isc = o_op == OP_CONST, isv = o_op == OP_VAR;
      const uint32_t u = unary_index(o_op);
      const uint32_t isc1 = isc ? 1u : 0u;
      const int kind = fused ? 0 : o_term ? 1 : o_bin ? 2 : 3;
      const uint32_t key = fused ? 20u + 6u * isc1 + ob : o_op >= 100u ? o_op - 86u : o_op;
      const uint32_t wslot = n > 0 ? un - 1u : 0u;
      const uint32_t warg = o_term ? o_arg : 0u;
      const uint32_t word = word_handlers(wt, key, un) | (warg << 8) | (wslot << 16);
      // (the largest stack size in output order equals need_root: the
      // larger operand first reaches max(a, b + 1) for needs a >= b)
      if (need_root > MAX_STACK || L_dec > a.max_words) status = BEAGLE_PROG_TOO_LONG;
      if (ws) {
        a.code[off + widx] = word;
        if (isc) a.cval[off + widx] = cvv;
      }
      int lc_short = -1;
      if constexpr (ADJ) {
        const int cst = scan_add(act & isc ? 1 : 0);  // CONST tokens up to here
        // the token whose subtree the word produces, and that subtree's start
        // (every cross-lane read runs on all lanes: inside a lane-dependent
        // branch its source lane may be inactive)
        const int last = sel(fused, lane + 1, lane);
        const int st_next = from(o_st, lane < 63 ? lane + 1 : 63);
        const int last_st = sel(fused, st_next, o_st);
        const int c_hi = from(cst, last < 64 ? last : 63);
        const int c_lo = from(cst, last_st > 0 ? last_st - 1 : 0);
        const bool sub_cf = c_hi - (last_st > 0 ? c_lo : 0) == 0;  // no CONST in the subtree
        const int wfst = from(widx, last_st);
        // binary words: the producer of the left operand ends just before the
        // right operand's subtree
        const int r_st = from(o_st, lane > 0 ? lane - 1 : 0);
        const int pa_w = from(widx, r_st > 0 ? r_st - 1 : 0);
        // per operator (B_ADD .. B_RDIV, 8 bits each): reverse handler and
        // derivative-tape entries of fused VAR words, fused CONST words and
        // binary words
        constexpr uint64_t RID_FV = uint64_t(R_FV_GEN) << 40 | uint64_t(R_FV_RSUB) << 32 | uint64_t(R_FV_GEN) << 24 |
                                    uint64_t(R_FV_GEN) << 16 | uint64_t(R_NOP) << 8 | uint64_t(R_NOP);
        constexpr uint64_t RID_FC = uint64_t(R_FC_RDIV) << 40 | uint64_t(R_FC_RSUB) << 32 | uint64_t(R_FC_DIV) << 24 |
                                    uint64_t(R_FC_MUL) << 16 | uint64_t(R_FC_SUB) << 8 | uint64_t(R_FC_ADD);
        constexpr uint64_t RID_BIN = uint64_t(R_BIN_GEN) << 40 | uint64_t(R_BIN_RSUB) << 32 |
                                     uint64_t(R_BIN_GEN) << 24 | uint64_t(R_BIN_GEN) << 16 |
                                     uint64_t(R_BIN_SUB) << 8 | uint64_t(R_BIN_ADD);
        constexpr uint32_t ENT_FV = 0x101100u, ENT_FC = 0x201100u, ENT_BIN = 0x202200u;  // 4 bits each
        const uint32_t rid_f = uint32_t(((isc ? RID_FC : RID_FV) >> (8u * ob)) & 0xFFu);
        const uint32_t rid_b = uint32_t((RID_BIN >> (8u * bo)) & 0xFFu);
        const int ent_f = int(((isc ? ENT_FC : ENT_FV) >> (4u * ob)) & 0xFu);
        const int ent_b = int((ENT_BIN >> (4u * bo)) & 0xFu);
        // the slot the reverse sweep writes, also the offset of the handler
        const uint32_t rws = pick4(kind, un - 1u, un, un - 2u, un - 1u);
        const uint32_t rid0 = pick4(kind, rid_f, isv ? R_NOP : R_PUSH_CONST, rid_b, R_UN);
        const int rlim = kind <= 1 ? 3 : 4;
        const int ent = pick4(kind, ent_f, 0, ent_b, 1);
        const bool wcf = pick4<bool>(kind, (!isc) & sub_cf, isv, sub_cf, sub_cf);
        const uint32_t pa = sel(kind == 2, uint32_t(pa_w), 0u);
        const uint32_t rid = sel(wcf | (rid0 == R_NOP), R_NOP, sel(n <= rlim, rid0 + rws, R_NONE));
        const int n_ent = lane_value(scan_add(ws & !wcf ? ent : 0), 63);
        lc_short = L_dec > a.short_words ? 1
                   : need_root > 4 || cc > GRAD_LANE_SLOTS || ext ? 0
                   : n_ent <= GRAD_DTAPE_SMALL ? 2 : n_ent <= GRAD_DTAPE_MID ? 3
                   : n_ent <= GRAD_DTAPE_LARGE ? 4 : 0;
        const bool dtape = status == BEAGLE_PROG_OK && lc_short >= 2;
        if (ws && !dtape) a.aux[off + widx] = pa | (rws << 16) | (rid << 24);
        // ---- the derivative-tape adjoint's words (see dtape_words)
        if (dtape) {
          // per word u (lane u): first word of its subtree with the
          // constant-free flag, its reverse handler, its code word
          if (ws) {
            sh.a[widx] = uint32_t(wfst) | (wcf ? 0x8000u : 0u) | (rid << 16);
            sh.b[widx] = word;
          }
          __builtin_amdgcn_wave_barrier();
          const bool wact = lane < L_dec;
          const uint32_t fw = wact ? sh.a[lane] : 0u;
          const uint32_t c = wact ? sh.b[lane] : 0u;
          __builtin_amdgcn_wave_barrier();
          const bool ucf = (fw & 0x8000u) != 0;
          const uint32_t urid = (fw >> 16) & 0xFFu;
          const int sk = ucf ? int(fw & 0x7FFFu) - 1 : lane - 1;
          const bool real = (!ucf) & (urid != R_NOP);
          // vis(u) = u + 1 if real, vis(sk) if sk >= 0, else 0: pointer
          // jumping over the skip links (state: the value | 0x100 once known,
          // else the link)
          int stv = sel(real, (lane + 1) | 0x100, sel(sk < 0, 0x100, sk));
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            const int v = from(stv, stv & 0xFF);
            stv = sel((stv & 0x100) != 0, stv, v);
          }
          const int vis = stv & 0xFF;
          const int next1 = from(vis, sk > 0 ? sk : 0);
          const uint32_t fid = ucf ? fwd_notape(c >> 24) : (c >> 24);
          if (wact)
            a.aux[off + lane] = uint32_t(sk >= 0 ? next1 : 0) | (fid << 8) | (((c >> 8) & 0xFFu) << 16) | (urid << 24);
        }
      }
      L_dec = status == BEAGLE_PROG_OK ? L_dec : 0;
      ListIds ids;
      if (status == BEAGLE_PROG_OK) {
        ids.cls = need_class(need_root);
        if (ext && ids.cls == 0) ids.cls = 1;
        ids.lc = lc_short;
      }
      ids.head = status | (need_root << 8) | (L_dec << 16);
      ids.vmask = status == BEAGLE_PROG_OK ? vmask : 0u;
      return ids;
    }
  }
  ListIds ids;
  ids.head = status;
  return ids;
}

// ---- several short programs per wave (evaluation only) -------------------
// The same decoding, bit for bit, for 64 / SEG programs of at most SEG tokens
// at once, program s in lanes s * SEG .. s * SEG + SEG - 1 (lane sb + i holds
// its token i).  Every cross-lane step stays inside the segment: prefix sums
// and maxima stop before the row broadcasts that would cross it, lane reads
// add the segment's base, ballots are cut to the segment's bits, word
// indices subtract the words of the segments below.  The program fields
// (header, status, register need) are per lane, equal within a segment.
namespace wdec {

template <int SEG>
__device__ __forceinline__ int seg_scan_add(int v) {
  v += dpp<0x111, 0xF>(v);
  v += dpp<0x112, 0xF>(v);
  v += dpp<0x114, 0xF>(v);
  v += dpp<0x118, 0xF>(v);
  if constexpr (SEG >= 32) v += dpp<0x142, 0xA>(v);
  return v;
}
template <int SEG>
__device__ __forceinline__ int seg_scan_max(int v) {
  v = max(v, dpp<0x111, 0xF>(v));
  v = max(v, dpp<0x112, 0xF>(v));
  v = max(v, dpp<0x114, 0xF>(v));
  v = max(v, dpp<0x118, 0xF>(v));
  if constexpr (SEG >= 32) v = max(v, dpp<0x142, 0xA>(v));
  return v;
}
// OR over the segment, on every lane
template <int SEG>
__device__ __forceinline__ uint32_t seg_or(uint32_t u, int last_lane) {
  int v = int(u);
  v |= dpp<0x111, 0xF>(v);
  v |= dpp<0x112, 0xF>(v);
  v |= dpp<0x114, 0xF>(v);
  v |= dpp<0x118, 0xF>(v);
  if constexpr (SEG >= 32) v |= dpp<0x142, 0xA>(v);
  return uint32_t(from(v, last_lane));
}

}  // namespace wdec

template <int SEG>
__device__ static ListIds decode_seg(const PrepareArgs& a, int p, int64_t off, int32_t L, int64_t coff, int32_t cc,
                                     int hstat, uint32_t tok, int lay_tok, WaveDecLds& sh, const uint32_t* wt) {
  using namespace wdec;
  static_assert(SEG == 16 || SEG == 32, "segments of 16 or 32 lanes");
  constexpr int LOG = SEG == 16 ? 4 : 5;
  constexpr uint64_t SEGMASK = (1ull << SEG) - 1ull;
  const int lane = lane_id();
  const int sb = lane & ~(SEG - 1);  // the segment's first lane
  const int sl = lane - sb;          // position in the segment
  // v of position i of this lane's segment (0 <= i < SEG where used)
  auto sfrom = [&](int v, int i) { return from(v, sb + i); };
  auto segbits = [&](uint64_t m) { return (m >> sb) & SEGMASK; };
  int status = hstat;
  if (lay_tok) {
    // ranges not sorted and disjoint: every slot must carry p as its owner
    const bool bad = status == BEAGLE_PROG_OK && sl < L && a.owner[off + sl] != p;
    if (segbits(__builtin_amdgcn_ballot_w64(bad)) != 0) status = BEAGLE_PROG_BAD_LAYOUT;
  }
  const bool ok0 = status == BEAGLE_PROG_OK;
  const bool act = ok0 & (sl < L);
  // lane masks of lane conditions, combined on the scalar side
  const uint64_t ltm = __builtin_amdgcn_ballot_w64(sl < L);
  const uint64_t actm = __builtin_amdgcn_ballot_w64(ok0) & ltm;
  const uint32_t t = act ? tok : 0u;
  const uint32_t op = t & 0xFFu, arg = t >> 8;
  const bool opok = op < N_OPCODES;
  constexpr uint64_t ARITY = 0x5554155AAull;  // as in decode_wave
  const int ar = opok ? int((ARITY >> (2u * op)) & 3u) : 0;
  const int d = seg_scan_add<SEG>(act ? 1 - ar : 0);
  const int err = !opok                              ? BEAGLE_PROG_BAD_OPCODE
                  : (op == OP_VAR) & (int(arg) >= a.D)  ? BEAGLE_PROG_BAD_VAR
                  : (op == OP_CONST) & (int(arg) >= cc) ? BEAGLE_PROG_BAD_CONST
                  : d < 1                             ? BEAGLE_PROG_UNDERFLOW
                                                      : 0;
  const uint64_t em = segbits(actm & __builtin_amdgcn_ballot_w64(err != 0));
  const int first_err = em ? __ffsll((unsigned long long)em) - 1 : 0;
  const int err_first = sfrom(err, first_err);
  const int d_last = sfrom(d, L >= 1 ? L - 1 : 0);
  if (ok0) status = em ? err_first : (d_last != 1 ? BEAGLE_PROG_BAD_FINAL_DEPTH : BEAGLE_PROG_OK);
  const bool ok = status == BEAGLE_PROG_OK;  // the structural pass ran
  const bool live = ok & (sl < L);
  const uint64_t livem = __builtin_amdgcn_ballot_w64(ok) & ltm;
  const uint32_t vmask = seg_or<SEG>(live & (op == OP_VAR) ? 1u << arg : 0u, sb + SEG - 1);
  const bool ext =
      segbits(livem & __builtin_amdgcn_ballot_w64(op - uint32_t(OP_SQUARE) < uint32_t(N_OPCODES - OP_SQUARE))) != 0;
  // ---- subtree starts (descent over minima of power-of-two windows)
  int mn[LOG];
  mn[0] = d;
#pragma unroll
  for (int k = 1; k < LOG; ++k) {
    const int w = 1 << (k - 1);
    mn[k] = min(mn[k - 1], sfrom(mn[k - 1], sl >= w ? sl - w : sl));
  }
  uint32_t r = uint32_t(sl);  // (as in decode_wave)
#pragma unroll
  for (int k = LOG - 1; k >= 0; --k) {
    const int v = __builtin_amdgcn_ds_bpermute(int((uint32_t(sb) + r) << 2) - 4, mn[k]);
    r = __builtin_elementwise_sub_sat(r, sel(v >= d, 1u << k, 0u));
  }
  const int st = int(r);
  // ---- register need (as in decode_wave)
  const int s_prev = sfrom(st, sl > 0 ? sl - 1 : 0);
  const int lch = s_prev - 1;
  constexpr int NEED_UNKNOWN = 1024;
  const bool is_un = ar == 1;
  // children's needs read at the bottom of their runs of unary operators
  const int bot = seg_scan_max<SEG>(is_un ? 0 : sl + 1);
  const int bot_r = sb + max(sfrom(bot, sl > 0 ? sl - 1 : 0) - 1, 0);
  const int bot_l = sb + max(sfrom(bot, lch > 0 ? lch : 0) - 1, 0);
  // (one rule for every token through the zero slot, as in decode_wave)
  const int src_r = sel(ar == 0, NEED_ZERO, bot_r);
  const int src_l = sel(ar == 2, bot_l, NEED_ZERO);
  if (lane == 0) sh.nd[NEED_ZERO] = 0;
  int need = ar == 0 ? 1 : NEED_UNKNOWN;
  int nr = 0, nl = 0;
  for (;;) {
    sh.nd[lane] = need;
    __builtin_amdgcn_wave_barrier();
    nr = sh.nd[src_r];
    nl = sh.nd[src_l];
    __builtin_amdgcn_wave_barrier();
    need = max(nl, nr) + int(nl == nr);
    if ((__builtin_amdgcn_ballot_w64(need >= 64) & livem) == 0) break;
  }
  int need_root = sfrom(need, L >= 1 ? L - 1 : 0);
  // ---- output order (parents' lanes as byte addresses)
  const bool swap = (ar == 2) & (nr > nl);
  const int size_r = sl - s_prev;
  const int st_l = sfrom(st, lch > 0 ? lch : 0);
  const int size_l = lch - st_l + 1;
  if (live && ar >= 1) sh.a[lane - 1] = uint32_t(lane << 2) | (uint32_t(ar == 2 && !swap ? size_l : 0) << 8);
  if (live && ar == 2) sh.a[sb + lch] = uint32_t(lane << 2) | (uint32_t(swap ? size_r : 0) << 8);
  if (ok && sl == L - 1) sh.a[lane] = uint32_t(lane << 2);
  __builtin_amdgcn_wave_barrier();
  int pk = live ? int(sh.a[lane]) : lane << 2;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < LOG; ++r) {
    const int v = __builtin_amdgcn_ds_bpermute(pk & 0xFC, pk);
    pk = (pk & ~0xFC) + v;
  }
  const int ostart = pk >> 8;
  const int oend = ostart + (sl - st);
  const uint32_t op2 = sel(swap & (op == OP_SUB), 100u + B_RSUB, sel(swap & (op == OP_DIV), 100u + B_RDIV, op));
  if (live) sh.b[sb + oend] = op2 | (arg << 8) | (uint32_t(ostart) << 16) | (uint32_t(ar) << 24);
  __builtin_amdgcn_wave_barrier();
  const uint32_t e = live ? sh.b[lane] : 0x010000FFu;  // (as in decode_wave)
  __builtin_amdgcn_wave_barrier();
  // ---- words, in output order (position sl holds output token sl)
  const uint32_t o_op = e & 0xFFu, o_arg = (e >> 8) & 0xFFu;
  float cvv = 0.0f;  // (loaded early, as in decode_wave)
  if (o_op == OP_CONST) cvv = a.consts[coff + o_arg];
  const uint32_t o_ar = e >> 24;
  const bool o_term = o_ar == 0u;
  const int o_delta = 1 - int(o_ar);
  const int n_after = seg_scan_add<SEG>(o_delta);
  const int n = n_after - o_delta;
  const uint32_t nxt = uint32_t(sfrom(int(o_op), sl < SEG - 1 ? sl + 1 : SEG - 1));
  // (as in decode_wave; the next token must be in the same segment, and a
  // segment's first token absorbs nothing)
  constexpr uint64_t SEGFIRST = SEG == 16 ? 0x0001000100010001ull : 0x0000000100000001ull;
  constexpr uint64_t SEGLAST = SEGFIRST << (SEG - 1);
  const uint64_t fm = __builtin_amdgcn_ballot_w64(o_term) & __builtin_amdgcn_ballot_w64(n >= 1) &
                      (__builtin_amdgcn_ballot_w64(nxt < 4u) | __builtin_amdgcn_ballot_w64(nxt - 100u < 6u)) &
                      (livem >> 1) & ~SEGLAST & livem;
  const bool fused = __builtin_amdgcn_inverse_ballot_w64(fm);
  const uint64_t wm = livem & ~((fm << 1) & ~SEGFIRST);
  const bool ws = __builtin_amdgcn_inverse_ballot_w64(wm);
  const uint64_t below = sb == 0 ? 0ull : wm & ((1ull << sb) - 1ull);  // words of the segments below
  const int E = int(__builtin_amdgcn_mbcnt_hi(uint32_t(wm >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(wm), 0u))) -
                __popcll(below);
  const int widx = ws ? E : E - 1;
  int L_dec = __popcll(segbits(wm));
  const uint32_t un = uint32_t(n);
  const uint32_t ob = nxt >= 100u ? nxt - 100u : nxt;
  const bool isc = o_op == OP_CONST;
  const uint32_t key = fused ? 20u + 6u * (isc ? 1u : 0u) + ob : o_op >= 100u ? o_op - 86u : o_op;
  const uint32_t wslot = n > 0 ? un - 1u : 0u;
  const uint32_t warg = o_term ? o_arg : 0u;
  const uint32_t word = word_handlers(wt, key, un) | (warg << 8) | (wslot << 16);
  if (ok && (need_root > MAX_STACK || L_dec > a.max_words)) status = BEAGLE_PROG_TOO_LONG;
  if (ws) {
    a.code[off + widx] = word;
    if (isc) a.cval[off + widx] = cvv;
  }
  ListIds ids;
  if (status == BEAGLE_PROG_OK) {
    ids.cls = need_class(need_root);
    if (ext && ids.cls == 0) ids.cls = 1;
  }
  // (a program stopped by its length keeps its need)
  ids.head = status | ((ok ? need_root : 0) << 8) | ((status == BEAGLE_PROG_OK ? L_dec : 0) << 16);
  ids.vmask = status == BEAGLE_PROG_OK ? vmask : 0u;
  return ids;
}

// Four waves per workgroup, a.wave_programs (1..64) consecutive programs per
// wave decoded one at a time (few per wave when the population is small, so
// that the grid still fills the chip); a program longer than 64 tokens is
// appended to the long list for k_prepare_long.  List appends: one atomic
// per list and workgroup.  The program headers of a
// wave's programs are loaded once (lane j: program j), and each program's
// tokens are loaded while the previous program is decoded.
__device__ __forceinline__ int64_t lane64(int64_t v, int j) {
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(uint64_t(v)), j);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(uint64_t(v) >> 32), j);
  return int64_t((uint64_t(hi) << 32) | lo);
}
// v of lane src (any lane's own choice)
__device__ __forceinline__ int64_t from64(int64_t v, int src) {
  const uint32_t lo = uint32_t(wdec::from(int(uint32_t(uint64_t(v))), src));
  const uint32_t hi = uint32_t(wdec::from(int(uint32_t(uint64_t(v) >> 32)), src));
  return int64_t((uint64_t(hi) << 32) | lo);
}

#ifndef PREP_WAVE_WPE
#define PREP_WAVE_WPE 8
#endif
template <bool ADJ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ADJ ? 1 : PREP_WAVE_WPE))) k_prepare_wave(PrepareArgs a) {
  __shared__ WaveDecLds lds[4];
  __shared__ uint32_t wt[32];
  if (threadIdx.x < 32) wt[threadIdx.x] = word_entry(threadIdx.x);
  __syncthreads();
  const int lane = int(threadIdx.x & 63u), w = int(threadIdx.x >> 6);
  const int ppw = a.wave_programs;
  const int64_t base = (int64_t(blockIdx.x) * 4 + w) * ppw;
  const int64_t pl = base + lane;
  const bool have = lane < ppw && pl < a.n_programs;
  const int32_t hL = have ? a.tok_len[pl] : 0;
  const int64_t hoff = have ? a.tok_offset[pl] : 0;
  const int64_t hcoff = have ? a.const_offset[pl] : 0;
  const int32_t hcc = have ? a.const_count[pl] : 0;
  const int nb = base < a.n_programs ? int(a.n_programs - base < ppw ? a.n_programs - base : ppw) : 0;
  // the header's own checks (lane j: program j): no tokens, or token or
  // constant range outside its array
  const int hst = hL == 0 ? BEAGLE_PROG_EMPTY
                  : hL < 0 || hoff < 0 || hoff + hL > a.n_tokens || hcc < 0 ||
                            (hcc > 0 && (hcoff < 0 || hcoff + hcc > a.n_consts))
                      ? BEAGLE_PROG_BAD_LAYOUT
                      : BEAGLE_PROG_OK;
  const uint64_t fetch_ok = __builtin_amdgcn_ballot_w64(hst == BEAGLE_PROG_OK && hL <= PREP_NARROW);
  // the lane's token of program j, where program j is decoded here and its
  // header passed (else 0: the decoder reports the header's status)
  auto fetch = [&](int j) -> uint32_t {
    const int32_t L = __builtin_amdgcn_readlane(hL, j);
    const bool ok = ((fetch_ok >> j) & 1u) && lane < L;
    return ok ? uint32_t(a.tokens[lane64(hoff, j) + lane]) : 0u;
  };
  // the disjoint-ranges flags (set before this kernel)
  const int lay_tok = a.layout ? a.layout[0] : 0;
  const int lay_const = a.layout && ADJ ? a.layout[1] : 0;
  int cls = -1, lc = -1;
  // program j's header fields, held by lane j and stored together at the end
  int32_t head = 0;
  uint32_t vmask = 0u;
  bool defer = false;
  if constexpr (ADJ) {
    uint32_t t_next = nb > 0 ? fetch(0) : 0u;
    for (int j = 0; j < nb; ++j) {
      const uint32_t t = t_next;
      if (j + 1 < nb) t_next = fetch(j + 1);
      const int32_t L = __builtin_amdgcn_readlane(hL, j);
      if (L > PREP_NARROW) {
        defer |= lane == j;
        continue;
      }
      const ListIds ids = decode_wave<ADJ>(a, int(base + j), lane64(hoff, j), L, lane64(hcoff, j),
                                           __builtin_amdgcn_readlane(hcc, j), __builtin_amdgcn_readlane(hst, j), t,
                                           lay_tok, lay_const, lds[w], wt);
      cls = wdec::sel(lane == j, ids.cls, cls);
      lc = wdec::sel(lane == j, ids.lc, lc);
      head = wdec::sel(lane == j, ids.head, head);
      vmask = wdec::sel(lane == j, ids.vmask, vmask);
    }
  } else {
    // Programs of at most 16 tokens four to a wave, then (with those left
    // over) programs of at most 32 tokens two to a wave, then the rest one at
    // a time -- three loops one after another, so that the register needs
    // of the two decoders do not add up.
    const bool hold = lane < nb;
    uint64_t m16 = __builtin_amdgcn_ballot_w64(hold && hL <= 16);
    uint64_t m32 = __builtin_amdgcn_ballot_w64(hold && hL > 16 && hL <= 32);
    uint64_t rest = __builtin_amdgcn_ballot_w64(hold) & ~(m16 | m32);
    auto take = [](uint64_t& m) -> int {
      const int j = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      return j;
    };
    // tokens of program jj (this lane's segment) at position sl (the
    // lane reads run on every lane, before the lane-dependent load: a read
    // from a lane outside the active ones returns 0)
    auto fetch_seg = [&](int jj, int sl) -> uint32_t {
      const int hs = wdec::from(hst, jj), Lp = wdec::from(hL, jj);
      const int64_t offp = from64(hoff, jj);
      return (hs == BEAGLE_PROG_OK) & (sl < Lp) ? uint32_t(a.tokens[offp + sl]) : 0u;
    };
    while (__popcll(m16) >= 4) {
      const int j0 = take(m16), j1 = take(m16), j2 = take(m16), j3 = take(m16);
      const int jj = wdec::pick4(lane >> 4, j0, j1, j2, j3);
      const uint32_t t = fetch_seg(jj, lane & 15);
      const ListIds ids = decode_seg<16>(a, int(base + jj), from64(hoff, jj), wdec::from(hL, jj), from64(hcoff, jj),
                                         wdec::from(hcc, jj), wdec::from(hst, jj), t, lay_tok, lds[w], wt);
      // program j_s's lists and header come from its segment's first lane
      const int s = wdec::sel(lane == j0, 0, wdec::sel(lane == j1, 1, wdec::sel(lane == j2, 2, 3)));
      const bool mine = (lane == j0) | (lane == j1) | (lane == j2) | (lane == j3);
      cls = wdec::sel(mine, wdec::from(ids.cls, s * 16), cls);
      head = wdec::sel(mine, wdec::from(ids.head, s * 16), head);
      vmask = wdec::sel(mine, uint32_t(wdec::from(int(ids.vmask), s * 16)), vmask);
    }
    m32 |= m16;
    while (__popcll(m32) >= 2) {
      const int j0 = take(m32), j1 = take(m32);
      const int jj = lane < 32 ? j0 : j1;
      const uint32_t t = fetch_seg(jj, lane & 31);
      const ListIds ids = decode_seg<32>(a, int(base + jj), from64(hoff, jj), wdec::from(hL, jj), from64(hcoff, jj),
                                         wdec::from(hcc, jj), wdec::from(hst, jj), t, lay_tok, lds[w], wt);
      const int src = lane == j0 ? 0 : 32;
      const bool mine = (lane == j0) | (lane == j1);
      cls = wdec::sel(mine, wdec::from(ids.cls, src), cls);
      head = wdec::sel(mine, wdec::from(ids.head, src), head);
      vmask = wdec::sel(mine, uint32_t(wdec::from(int(ids.vmask), src)), vmask);
    }
    rest |= m32;
    // one at a time
    int j = rest ? take(rest) : -1;
    uint32_t t_next = j >= 0 ? fetch(j) : 0u;
    while (j >= 0) {
      const uint32_t t = t_next;
      const int jn = rest ? take(rest) : -1;
      if (jn >= 0) t_next = fetch(jn);
      const int32_t L = __builtin_amdgcn_readlane(hL, j);
      if (L > PREP_NARROW) {
        defer |= lane == j;
      } else {
        const ListIds ids = decode_wave<false>(a, int(base + j), lane64(hoff, j), L, lane64(hcoff, j),
                                               __builtin_amdgcn_readlane(hcc, j), __builtin_amdgcn_readlane(hst, j),
                                               t, lay_tok, 0, lds[w], wt);
        cls = wdec::sel(lane == j, ids.cls, cls);
        head = wdec::sel(lane == j, ids.head, head);
        vmask = wdec::sel(lane == j, ids.vmask, vmask);
      }
      j = jn;
    }
  }
  const int p = int(base + lane);  // (lanes without a program append nothing)
  // the headers of the programs decoded here (a long program's header is
  // written by k_prepare_long)
  if (lane < nb && !defer) {
    ProgMeta m;
    m.status = head & 0xFF;
    m.need = (head >> 8) & 0xFF;
    m.len = head >> 16;
    m.shift = 0.0f;
    m.vmask = vmask;
    a.meta[p] = m;
    if (a.status_out) a.status_out[p] = int8_t(m.status);
  }
  __shared__ int32_t cnt[4][8], lbase[8];
  block_append<1, 4>(defer ? 0 : -1, p, a.long_count, a.long_list, 0, cnt, lbase);
  __syncthreads();
  block_append<N_CLASSES, 4>(cls, p, a.class_count, a.class_list, a.n_programs, cnt, lbase);
  if (ADJ) {
    __syncthreads();
    block_append<GRAD_LISTS, 4>(lc, p, a.len_count, a.len_list, a.n_programs, cnt, lbase);
  }
}

template __global__ void k_prepare_wave<false>(PrepareArgs a);
template __global__ void k_prepare_wave<true>(PrepareArgs a);

// ---- disjoint-ranges check -------------------------------------------------
// Token range of program p when it lies within the token array (else
// false: the program is rejected by the layout checks of the decoder).
__device__ static bool tok_range(const PrepareArgs& a, int p, int64_t& off, int32_t& L) {
  off = a.tok_offset[p];
  L = a.tok_len[p];
  return L >= 0 && L <= MAX_LEN && off >= 0 && off + L <= a.n_tokens;
}

__device__ static bool const_range(const PrepareArgs& a, int p, int64_t& off, int32_t& n) {
  off = a.const_offset[p];
  n = a.const_count[p];
  return n >= 0 && (n == 0 || (off >= 0 && off + n <= a.n_consts));
}

// Program p against program p + 1: ranges out of order, overlapping, or out
// of bounds (conservatively) set the flag.
__device__ static void layout_pair(const PrepareArgs& a, int p) {
  if (p + 1 >= a.n_programs) return;
  int64_t o0, o1;
  int32_t n0, n1;
  const bool v0 = tok_range(a, p, o0, n0), v1 = tok_range(a, p + 1, o1, n1);
  if (!(v0 && v1 && o0 + n0 <= o1)) atomicOr(a.layout, 1);
  if (a.adjoint) {
    const bool c0 = const_range(a, p, o0, n0), c1 = const_range(a, p + 1, o1, n1);
    if (!(c0 && c1 && (n0 == 0 || n1 == 0 || o0 + n0 <= o1))) atomicOr(a.layout + 1, 1);
  }
}

// grid-stride fill of the owner arrays with the largest index (only after a
// flagged layout)
__device__ static void layout_fill(const PrepareArgs& a, int64_t i0, int64_t stride) {
  if (a.layout[0])
    for (int64_t i = i0; i < a.n_tokens; i += stride) a.owner[i] = 0x7FFFFFFF;
  if (a.adjoint && a.layout[1])
    for (int64_t i = i0; i < a.n_consts; i += stride) a.cowner[i] = 0x7FFFFFFF;
}

// program p marks its ranges with its index (the lowest index wins)
__device__ static void layout_mark(const PrepareArgs& a, int p) {
  int64_t off;
  int32_t n;
  if (a.layout[0] && tok_range(a, p, off, n))
    for (int32_t i = 0; i < n; ++i) atomicMin(a.owner + off + i, p);
  if (a.adjoint && a.layout[1] && const_range(a, p, off, n))
    for (int32_t i = 0; i < n; ++i) atomicMin(a.cowner + off + i, p);
}

__global__ void k_layout_fill(PrepareArgs a) {
  layout_fill(a, int64_t(blockIdx.x) * blockDim.x + threadIdx.x, int64_t(gridDim.x) * blockDim.x);
}

__global__ void k_layout_mark(PrepareArgs a) {
  if (!a.layout[0] && !(a.adjoint && a.layout[1])) return;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < a.n_programs;
       p += int64_t(gridDim.x) * blockDim.x)
    layout_mark(a, int(p));
}

__global__ void k_layout_check_batch(BatchArgs b) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= b.n_programs) return;
  const int q = batch_find(b, g, [](const BatchProblem& t) { return t.prog_begin; });
  layout_pair(b.table[q].prep, int(g - b.table[q].prog_begin));
}

// blockIdx.y: the problem
__global__ void k_layout_fill_batch(BatchArgs b) {
  layout_fill(b.table[blockIdx.y].prep, int64_t(blockIdx.x) * blockDim.x + threadIdx.x,
              int64_t(gridDim.x) * blockDim.x);
}

__global__ void k_layout_mark_batch(BatchArgs b) {
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < b.n_programs;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int q = batch_find(b, g, [](const BatchProblem& t) { return t.prog_begin; });
    const PrepareArgs& a = b.table[q].prep;
    if (a.layout[0] || (a.adjoint && a.layout[1])) layout_mark(a, int(g - b.table[q].prog_begin));
  }
}

// One thread per program of every problem of the table.
__global__ void __launch_bounds__(PREP_BLOCK) k_prepare_batch(BatchArgs b) {
  __shared__ PrepLds lds;
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= b.n_programs) return;
  const int q = batch_find(b, g, [](const BatchProblem& t) { return t.prog_begin; });
  const PrepareArgs& a = b.table[q].prep;
  const int p = int(g - b.table[q].prog_begin);
  append_one(a, p, prepare_one(a, p, lds));
}

// X [M x D] row-major -> Xt [D x Mp] (case index fastest), y -> yp [Mp];
// cases M..Mp-1 repeat case 0 (their outputs are masked out of every sum).
__device__ static void stage_case(const StageArgs& a, int64_t i) {
  const int64_t src = i < a.M ? i : 0;
  for (int d = 0; d < a.D; ++d) a.Xt[int64_t(d) * a.Mp + i] = a.X[src * a.D + d];
  a.yp[i] = a.y[src];
}

// Staging and the disjoint-ranges check in one launch (neither reads what
// the other writes): the first stage_blocks workgroups stage cases, the
// rest check program pairs.
__global__ void k_stage_and_check(StageArgs sa, PrepareArgs pa, uint32_t stage_blocks) {
  if (blockIdx.x < stage_blocks) {
    // (grid-stride: the staging part of the grid is capped)
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < sa.Mp;
         i += int64_t(stage_blocks) * blockDim.x)
      stage_case(sa, i);
  } else {
    const int64_t p = int64_t(blockIdx.x - stage_blocks) * blockDim.x + threadIdx.x;
    if (p < pa.n_programs) layout_pair(pa, int(p));
  }
}

// One thread per padded case of every problem of the table.
__global__ void k_stage_batch(BatchArgs b) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= b.n_cases) return;
  const int q = batch_find(b, g, [](const BatchProblem& t) { return t.case_begin; });
  const BatchProblem& P = b.table[q];
  StageArgs a;
  a.X = P.X;
  a.y = P.y;
  a.M = P.M;
  a.Mp = P.Mp;
  a.D = P.prep.D;
  a.Xt = P.Xt;
  a.yp = P.yp;
  stage_case(a, g - P.case_begin);
}

// Target statistics for the correlation fitness and the paper's r^4 score,
// one workgroup, fixed order, over the valid (finite) targets only (every
// target of a correlation fitness is valid): with n of them,
//   ybar = y0 + sum(y - y0) / n  (y0 = y[0], or 0 when y[0] is invalid),
//   w_i = y_i - ybar (binary64), stats = {ybar, sum w, sum w^2 - (sum w)^2 / n}.
constexpr int STATS_UNROLL = 8;

__device__ static void target_stats_block(const float* __restrict__ y, int64_t M, double* __restrict__ stats,
                                          double (&red)[2][1024]) {
  const int t = threadIdx.x;
  const double y0 = isfinite(y[0]) ? double(y[0]) : 0.0;
  double s = 0.0, cnt = 0.0;
  // each thread sums i = t, t + 1024, ... in that order; STATS_UNROLL of its
  // loads are issued before the first of their additions
  for (int64_t i0 = t; i0 < M; i0 += STATS_UNROLL * 1024) {
    float v[STATS_UNROLL];
#pragma unroll
    for (int u = 0; u < STATS_UNROLL; ++u) v[u] = i0 + u * 1024 < M ? y[i0 + u * 1024] : __builtin_nanf("");
#pragma unroll
    for (int u = 0; u < STATS_UNROLL; ++u) {
      const bool ok = isfinite(v[u]);
      s += ok ? double(v[u]) - y0 : 0.0;
      cnt += ok ? 1.0 : 0.0;
    }
  }
  red[0][t] = s;
  red[1][t] = cnt;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  const double n = red[1][0];
  const double ybar = n > 0.0 ? y0 + red[0][0] / n : y0;
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i0 = t; i0 < M; i0 += STATS_UNROLL * 1024) {
    float v[STATS_UNROLL];
#pragma unroll
    for (int u = 0; u < STATS_UNROLL; ++u) v[u] = i0 + u * 1024 < M ? y[i0 + u * 1024] : __builtin_nanf("");
#pragma unroll
    for (int u = 0; u < STATS_UNROLL; ++u) {
      const bool ok = isfinite(v[u]);
      const double w = ok ? double(v[u]) - ybar : 0.0;
      s1 += w;
      s2 += w * w;
    }
  }
  red[0][t] = s1;
  red[1][t] = s2;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    stats[0] = ybar;
    stats[1] = red[0][0];
    stats[2] = red[1][0] - red[0][0] * red[0][0] / (n > 0.0 ? n : 1.0);
  }
}

__global__ void __launch_bounds__(1024) k_target_stats(const float* __restrict__ y, int64_t M,
                                                       double* __restrict__ stats) {
  __shared__ double red[2][1024];
  target_stats_block(y, M, stats, red);
}

// One workgroup per problem of the table.
__global__ void __launch_bounds__(1024) k_target_stats_batch(BatchArgs b) {
  __shared__ double red[2][1024];
  const BatchProblem& P = b.table[blockIdx.x];
  target_stats_block(P.y, P.M, P.stats, red);
}

}  // namespace bgl
