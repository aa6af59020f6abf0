// Argument blocks and launchers of the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/beagle.h"
#include "beagle_device.h"

namespace bgl {

constexpr int GRAD_SHORT_WORDS = 64;   // tape in registers up to this many decoded words
constexpr int GRAD_LONG_WORDS = 256;   // tape in LDS up to this many (longer: TOO_LONG)
// the derivative-tape adjoint (register need <= 4): tape entries per case of
// its three kernels (4, 2 and 2 cases per lane)
constexpr int GRAD_DTAPE_SMALL = 16;
constexpr int GRAD_DTAPE_MID = 32;
constexpr int GRAD_DTAPE_LARGE = 64;
// adjoint program lists: 0 short value tape, 1 long value tape, 2..4
// derivative tape of at most GRAD_DTAPE_SMALL / MID / LARGE entries
constexpr int GRAD_LISTS = 5;
// constant slots whose gradients are summed per lane (the derivative-tape
// kernels take only programs with at most this many slots)
constexpr int GRAD_LANE_SLOTS = 8;
// cases per work item of the adjoint (at most), a multiple of the cases one
// tile of every adjoint kernel covers
constexpr int64_t GRAD_CHUNK_CASES = 1024;
constexpr int64_t GRAD_TILE_CASES = 256;
// work items a wave claims per atomic in the adjoint kernels
constexpr int GRAD_BATCH = 4;

// Reverse handler of a decoded word in the derivative-tape adjoint (bits
// 24..31 of the word's aux entry).  n is the stack size before the word in
// the forward sweep; the offsets below add n (pushes), n - 2 (binary
// operators) or n - 1 (unary operators and fused words).
//   NOP        VAR pushes; fused VAR + and -: the adjoint is unchanged
//   PUSH_CONST the pushed constant's gradient gains the slot's adjoint
//   BIN_ADD/SUB/RSUB  binary operators with constant partial derivatives
//   BIN_GEN    binary operators with two tape entries (d/da, d/db)
//   UN         unary operators: one tape entry (the derivative)
//   FV_RSUB    fused "x - top": the adjoint changes sign
//   FV_GEN     fused VAR *, /, reversed /: one entry (d/dtop)
//   FC_*       fused CONST words: the constant's gradient gains
//              adjoint * d/dc (ADD/SUB/RSUB: +-1; MUL, DIV: one entry;
//              RDIV: two entries, d/dtop then d/dc); the adjoint is scaled
//              by d/dtop (MUL: c; DIV: 1/c, 0 when c == 0)
constexpr uint32_t R_NOP = 0;
constexpr uint32_t R_PUSH_CONST = 1;  // + n, n 0..3
constexpr uint32_t R_BIN_ADD = 5;     // + n - 2, n 2..4
constexpr uint32_t R_BIN_SUB = 8;
constexpr uint32_t R_BIN_RSUB = 11;
constexpr uint32_t R_BIN_GEN = 14;
constexpr uint32_t R_UN = 17;         // + n - 1, n 1..4
constexpr uint32_t R_FV_RSUB = 21;    // + n - 1, n 1..3
constexpr uint32_t R_FV_GEN = 24;
constexpr uint32_t R_FC_ADD = 27;
constexpr uint32_t R_FC_SUB = 30;
constexpr uint32_t R_FC_RSUB = 33;
constexpr uint32_t R_FC_MUL = 36;
constexpr uint32_t R_FC_DIV = 39;
constexpr uint32_t R_FC_RDIV = 42;
constexpr uint32_t R_NONE = 255;

// Forward handlers of the derivative-tape adjoint: the small-stack handler
// numbers (I0_*) for words that store their entries, and for the words of
// constant-free subtrees (no entries) of the operators that would store some:
constexpr uint32_t F_BIN_NT = 82;  // + 3 j + n - 2, j: *, /, reversed /
constexpr uint32_t F_UN_NT = 91;   // + 4 u + n - 1
constexpr uint32_t F_FV_NT = 111;  // fused VAR: + 3 j + n - 1

struct GradArgs {
  const uint32_t* code;
  const uint32_t* aux;
  const float* cval;
  const int64_t* tok_offset;
  const ProgMeta* meta;
  const int64_t* const_offset;
  const int32_t* const_count;
  const float* Xt;  // [D x Mp]
  const float* yp;  // [Mp]
  int64_t M, Mp;
  int32_t D;
  int32_t n_programs;
  int32_t n_chunks;
  int64_t chunk;
  double* part;        // [n_chunks][n_programs] sums of squared errors
  double* gpart;       // [n_chunks][n_consts] gradient partials
  int64_t n_consts;
  int32_t kind;               // BEAGLE_FIT_MSE or BEAGLE_FIT_CORR
  const double* coef;         // CORR: per program (alpha, beta, mu) of the seed
  const double* stats;        // CORR: target statistics (mean, sum of w = y - mean, Syy)
  const int32_t* list_count;  // [GRAD_LISTS] program counts of the adjoint lists
  const int32_t* list;        // [GRAD_LISTS][n_programs]
  unsigned long long* work;   // [GRAD_LISTS] work-item counters, zero at launch
};

struct GradFinalizeArgs {
  const ProgMeta* meta;
  const double* part;
  const double* gpart;
  const int64_t* const_offset;
  const int32_t* const_count;
  int64_t M;
  int64_t n_consts;
  int32_t n_programs;
  int32_t n_chunks;
  int32_t kind;     // CORR: the fitness comes from the evaluation pass
  double* fitness;
  float* grad;
};

__global__ void k_grad_finalize(GradFinalizeArgs a);
size_t grad_lds_bytes(int D, bool long_tape);
hipError_t launch_grad(const GradArgs& a, hipStream_t s);

}  // namespace bgl
