// Kernel argument blocks and host-side launchers of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/beagle.h"
#include "beagle_device.h"

namespace bgl {

struct PrepareArgs {
  const uint16_t* tokens;
  int64_t n_tokens;
  const int64_t* tok_offset;
  const int32_t* tok_len;
  const float* consts;
  int64_t n_consts;
  const int64_t* const_offset;
  const int32_t* const_count;
  int32_t n_programs;
  int32_t D;
  uint32_t* code;      // [n_tokens] decoded words
  uint32_t* aux;       // [n_tokens] adjoint operands per decoded word
  float* cval;         // [n_tokens] CONST values by output position
  int32_t max_words;   // decoded words allowed (longer -> BEAGLE_PROG_TOO_LONG)
  int32_t* scr_stack;  // [n_tokens] scratch
  int32_t* scr_start;  // [n_tokens] scratch
  int32_t* scr_need;   // [n_tokens] scratch
  ProgMeta* meta;      // [n_programs]
  int8_t* status_out;  // [n_programs] or null
  int32_t* class_count;  // [N_CLASSES] programs per register-need class
  int32_t* class_list;   // [N_CLASSES][n_programs] program indices per class
  int32_t* len_count;    // [5] adjoint lists (see k_prepare)
  int32_t* len_list;     // [5][n_programs]
  int32_t short_words;
  // nonzero: also write the adjoint's per-word operands (aux) and its
  // program lists (an evaluation without gradients needs neither)
  int32_t adjoint;
  // programs k_prepare leaves to k_prepare_long (count zero at launch)
  int32_t* long_count;
  int32_t* long_list;  // [n_programs]
  // Disjoint ranges: every program is decoded in place of its tokens, so the
  // token ranges of different programs (and, for the adjoint, whose gradient
  // output has the constants' layout, the constant ranges) must not overlap.
  // layout[0], layout[1] (zero at launch): set by k_stage_and_check when the
  // token / constant ranges are not sorted and disjoint by program index;
  // then owner / cowner hold, per token / constant slot, the lowest index of
  // a program whose range covers it, and a program finding another index in
  // its range gets BEAGLE_PROG_BAD_LAYOUT.
  int32_t* layout;
  int32_t* owner;   // [n_tokens]
  int32_t* cowner;  // [n_consts] (adjoint only)
  // programs each wave of k_prepare_wave decodes (1..64)
  int32_t wave_programs;
};

struct StageArgs {
  const float* X;
  const float* y;
  int64_t M;
  int64_t Mp;
  int32_t D;
  float* Xt;  // [D x Mp]
  float* yp;  // [Mp]
};

// Partial sums per (chunk, program) of each fitness kind (the evaluator's
// epilogue: MSE 1, CORR 3, the paper's POINT score 1, its R4 score 7).
__host__ __device__ constexpr int kind_sums(int kind) {
  return kind == BEAGLE_FIT_MSE ? 1 : kind == BEAGLE_FIT_CORR ? 3 : kind == BEAGLE_FIT_POINT ? 1 : 7;
}
constexpr int MAX_SUMS = 8;

struct EvalArgs {
  const uint32_t* code;
  const float* cval;
  const int64_t* tok_offset;
  const ProgMeta* meta;
  const float* Xt;  // [D x Mp]
  const float* yp;  // [Mp]
  int64_t M;
  int64_t Mp;
  int32_t D;
  int32_t n_programs;
  int32_t n_chunks;
  int64_t chunk;          // cases per chunk, a multiple of CASES_PER_BLOCK_ITER
  double* part;           // [n_sums][n_chunks][n_programs]
  const double* stats;    // target statistics (correlation fitness)
  const int32_t* class_count;       // [N_CLASSES]
  const int32_t* class_list;        // [N_CLASSES][n_total] global program indices
  unsigned long long* work;         // [N_CLASSES] work-item counters, zero at launch
  int32_t n_total;                  // programs in the whole population
  int32_t prog_begin;               // first program of this launch (slice-local index 0)
  double smax = 0.0;                // the paper's scores: maximum score S
  // correlation and Eq. 2: when set, the resident-inputs kernels take each
  // class-0 and class-1 program's shift from their own first pass and store
  // it here (the same array as meta); the shift pass then covers class 2 only
  ProgMeta* meta_shift = nullptr;
};

struct FinalizeArgs {
  const ProgMeta* meta;
  const double* part;
  const double* stats;
  int64_t M;
  int32_t n_programs;
  int32_t n_chunks;
  int32_t kind;
  double* fitness;
  // correlation fitness only, or null: per program (alpha, beta, mu) of the
  // gradient seed dF/dyhat_i = alpha (w_i - mean w) + beta (yhat_i - mu)
  double* coef = nullptr;
  double smax = 0.0;  // the paper's scores: maximum score S
};

struct ValuesArgs {
  const uint32_t* code;
  const float* cval;
  const int64_t* tok_offset;
  ProgMeta* meta;
  const float* Xt;
  int64_t Mp;
  int64_t m;        // cases evaluated: [0, m)
  int32_t D;
  int32_t n_programs;
  float* out;       // [n_programs x m] or null (shift mode)
  int32_t shift_mode;
};

// One problem of a batched evaluation: an entry of the device problem table.
// Every pointer (the caller's arrays and this problem's share of the
// workspace) is resolved on the host before the table is uploaded.
struct BatchProblem {
  PrepareArgs prep;  // programs, decode targets, class lists, status output
  const float* X;    // [M x D] caller's cases
  const float* y;    // [M]
  float* Xt;         // [D x Mp]
  float* yp;         // [Mp]
  double* stats;     // [4] target statistics
  double* part;      // [n_sums][n_chunks][n_programs]
  double* fitness;   // [n_programs] caller's output
  int64_t M;
  int64_t Mp;
  int64_t chunk;
  int32_t n_chunks;
  int32_t kv;          // tile variant of class 0 for this problem
  int64_t prog_begin;  // first program of this problem in the batch-wide program index
  int64_t case_begin;  // first padded case of this problem in the batch-wide case index
};

// Work lists of a batched evaluation: class 0 wide tile, class 0 narrow
// tile, class 1, class 2; each split by the problems' variable count into
// N_DBUCKETS lists, launched separately so that each launch sizes its input
// tiles in LDS, and hence its occupancy, for its own largest D instead of the
// batch's.  The buckets (D <= 5, 6, 7..8, more) end where the workgroups
// per CU change: the 8-case tiles fit four workgroups up to D = 5 (their
// registers allow no more), three at 6, two at 7 and 8; the 4-case ones seven
// up to 5, six at 6, five at 7 and 8, four at 9.
constexpr int N_LISTS = 4;
constexpr int N_DBUCKETS = 4;
constexpr int N_BATCH_LISTS = N_LISTS * N_DBUCKETS;
static_assert(N_BATCH_LISTS <= 64, "one wave clears and offsets the work lists");
__host__ __device__ constexpr int d_bucket(int D) { return D <= 5 ? 0 : (D == 6 ? 1 : (D <= 8 ? 2 : 3)); }

struct BatchArgs {
  const BatchProblem* table;
  int32_t n_problems;
  int32_t kind;
  int64_t n_programs;          // over the whole table
  int64_t n_cases;             // padded cases over the whole table
  int64_t* item_off;           // [N_BATCH_LISTS][n_problems + 1] first work item of each problem per list
  unsigned long long* work;    // [N_BATCH_LISTS] work-item counters, zero at launch
};

// The problem holding batch-wide index x of a prefix field (prog_begin or
// case_begin): the last q with field(q) <= x.
template <class F>
__device__ __forceinline__ int batch_find(const BatchArgs& b, int64_t x, F field) {
  int lo = 0, hi = b.n_problems;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (field(b.table[mid]) <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

constexpr int EVAL_WAVES = 4;
constexpr int CASES_PER_WAVE_ITER = 64 * 8;                             // cases of one wave tile (K <= 8)
constexpr int CASES_PER_BLOCK_ITER = CASES_PER_WAVE_ITER * EVAL_WAVES;  // chunk granularity and case padding
// Cases per lane of the register-need classes (variant KV selects the
// narrower tile of class 0, used when the LDS input tile of the wide one
// would exceed WIDE_TILE_MAX_D variables).
constexpr int WIDE_TILE_MAX_D = 8;
// The resident-inputs evaluator (small case sets, register-need classes 0
// and 1): inputs of at most this many bytes per workgroup, populations of at
// least this many programs.
constexpr size_t RESIDENT_MAX_BYTES = 64 * 1024;
constexpr int32_t RESIDENT_MIN_PROGRAMS = 4096;
constexpr int RESIDENT_BATCH = 16;  // programs a wave claims per atomic (long lists)
__host__ __device__ constexpr int class_k(int c, int kv) { return c == 0 ? (kv == 0 ? 8 : 4) : (c == 1 ? 4 : 2); }

// decoding: programs of at most 64 tokens in k_prepare_wave (a wave per
// program) or k_prepare (a thread per program, narrow LDS scratch), the
// longer ones they list for k_prepare_long
// the disjoint-ranges check before decoding (see PrepareArgs::layout):
// neighbour comparison, then (only when that found unsorted or overlapping
// ranges) the owner arrays filled and marked
__global__ void k_layout_fill(PrepareArgs a);
__global__ void k_layout_mark(PrepareArgs a);
__global__ void k_layout_check_batch(BatchArgs b);
__global__ void k_layout_fill_batch(BatchArgs b);
__global__ void k_layout_mark_batch(BatchArgs b);
__global__ void k_prepare(PrepareArgs a);
// ADJ: also the adjoint's per-word operands and lists (PrepareArgs::adjoint)
template <bool ADJ>
__global__ void k_prepare_wave(PrepareArgs a);
__global__ void k_prepare_long(PrepareArgs a);
__global__ void k_stage_and_check(StageArgs sa, PrepareArgs pa, uint32_t stage_blocks);
__global__ void k_prepare_batch(BatchArgs b);
__global__ void k_stage_batch(BatchArgs b);
__global__ void k_target_stats_batch(BatchArgs b);
__global__ void k_values_batch(BatchArgs b);
__global__ void k_batch_items(BatchArgs b);
__global__ void k_finalize_batch(BatchArgs b);
__global__ void k_target_stats(const float* __restrict__ y, int64_t M, double* __restrict__ stats);
__global__ void k_finalize(FinalizeArgs a);
__global__ void k_values(ValuesArgs a);
// correlation shifts of the programs of register-need class 2 (a persistent
// grid walking its class list)
__global__ void k_values_deep(ValuesArgs a, const int32_t* class_count, const int32_t* class_list, int32_t stride);
// whether an evaluation of this shape takes the resident-inputs kernels for
// classes 0 and 1 (one chunk, enough programs, inputs within
// RESIDENT_MAX_BYTES)
bool resident_eligible(int64_t M, int32_t D, int32_t n_chunks, int32_t n_total);

// host launchers of the templated evaluation kernels (eval.hip)
// ev0/ev1 (may be null) are recorded on `s` right before and after the
// fast-path kernel.
// kv selects the tile variant of class 0 (forced to the narrow one above
// WIDE_TILE_MAX_D variables).
// counters_clear: a.work is known to be zero (else it is cleared first).
hipError_t launch_eval(int kind, int kv, const EvalArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                       bool counters_clear = false);
// The work-list kernels of a batched evaluation; max_d[v] is the largest D
// among the problems of list v (sizes the LDS tile), lists with
// has_items[v] == 0 are skipped.
hipError_t launch_eval_batch(int kind, const BatchArgs& b, const int* max_d, const int* has_items, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1);
// Runs the occupancy queries of those launches (before a stream capture).
void prime_eval_batch(int kind, const int* max_d, const int* has_items);

}  // namespace bgl
