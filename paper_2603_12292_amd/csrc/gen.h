// Argument blocks of the generation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgl {

constexpr int MAX_INIT_DEPTH = 11;  // 2^12 - 1 = 4095 tokens fit BEAGLE_MAX_LEN

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
  int32_t n;  // parents = children
  int32_t D;
  int32_t tournament;
  float t_cross;  // operator thresholds on unit(u), binary32
  float t_mut;
  int32_t max_len;
  int32_t max_consts;
  float const_lo, const_hi;
  uint64_t seed;
  uint32_t generation;
  uint32_t tag;
  uint16_t* child_tokens;
  int32_t* child_len;
  float* child_consts;
  int32_t* child_const_count;
};

struct InitArgs {
  int32_t n, D;
  int32_t depth_min, depth_max;
  int32_t max_len, max_consts;
  float const_lo, const_hi;
  uint64_t seed;
  uint32_t tag;
  uint16_t* tokens;
  int32_t* len;
  float* consts;
  int32_t* const_count;
};

__global__ void k_generation(GenStepArgs a);
__global__ void k_init_population(InitArgs a);

}  // namespace bgl
