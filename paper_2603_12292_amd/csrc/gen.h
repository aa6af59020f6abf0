// Argument blocks of the generation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgl {

constexpr int MAX_INIT_DEPTH = 11;  // 2^12 - 1 = 4095 tokens fit BEAGLE_MAX_LEN

// Microcosm selection: at most this many sampled individuals (one workgroup
// ranks them), individuals per block of the survivor compaction, and the
// counter fields of the sample's random stream.
constexpr int MICRO_MAX_SAMPLE = 1024;
constexpr int MICRO_BLOCK = 256;
constexpr uint32_t MICRO_INDEX = 0xFFFFFFFFu;
constexpr uint32_t MICRO_TAG = 0x40000000u;

struct GenStepArgs {
  const uint16_t* tokens;
  int64_t n_tokens;
  const int64_t* tok_offset;
  const int32_t* tok_len;
  const float* consts;
  int64_t n_consts;
  const int64_t* const_offset;
  const int32_t* const_count;
  const double* fitness;
  int32_t n;          // children
  int32_t n_parents;  // tournament range (equal to n for the classic step)
  // microcosm selection: parents A and B are drawn uniformly from
  // surv[0 .. *n_surv) (every parent when *n_surv == 0); NULL: tournaments
  const int32_t* surv;
  const int32_t* n_surv;
  int32_t D;
  int32_t tournament;
  float t_cross;  // operator thresholds on unit(u), binary32
  float t_mut;
  int32_t max_len;
  int32_t max_consts;
  float const_lo, const_hi;
  int32_t n_unary;  // 5: SIN..SQRT; 12: and SQUARE..TANH (the paper's set)
  uint64_t seed;
  uint32_t generation;
  uint32_t tag;
  uint16_t* child_tokens;
  int32_t* child_len;
  float* child_consts;
  int32_t* child_const_count;
  // the parents' layout when it is regular (slots[0] != 0: parent i's tokens
  // at slots[1] + i * slots[2], its constants at slots[3] + i * slots[4]), so
  // that a child need not read two header entries of a random parent; NULL:
  // always read them
  const int64_t* slots;
};

struct InitArgs {
  int32_t n, D;
  int32_t depth_min, depth_max;
  int32_t max_len, max_consts;
  float const_lo, const_hi;
  int32_t n_unary;
  uint64_t seed;
  uint32_t tag;
  uint16_t* tokens;
  int32_t* len;
  float* consts;
  int32_t* const_count;
};

struct MicroArgs {
  const double* fitness;
  int32_t n;       // parents
  int32_t sample;  // individuals drawn, 1 .. MICRO_MAX_SAMPLE
  int32_t k;       // position of the threshold in the sorted sample
  uint64_t seed;
  uint32_t generation;
  uint32_t tag;        // MICRO_TAG | problem
  int32_t n_blocks;    // ceil(n / MICRO_BLOCK)
  double* tau;         // [1] threshold
  int32_t* block_off;  // [n_blocks] survivor counts, then their exclusive prefix sums
  int32_t* n_surv;     // [1] survivors in total
  int32_t* surv;       // [n] survivor indices in index order
  // the parents' token and constant offsets, and [5] their layout test (see
  // GenStepArgs::slots): k_micro_threshold writes the layout of the first
  // two parents, k_micro_count clears slots[0] at any parent that breaks it
  const int64_t* tok_offset;
  const int64_t* const_offset;
  int64_t* slots;
};

__global__ void k_generation(GenStepArgs a);
__global__ void k_micro_threshold(MicroArgs a);
__global__ void k_micro_count(MicroArgs a);
__global__ void k_micro_scan(MicroArgs a);
__global__ void k_micro_scatter(MicroArgs a);
__global__ void k_init_population(InitArgs a);

}  // namespace bgl
