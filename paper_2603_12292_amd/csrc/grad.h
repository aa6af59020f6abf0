// Argument blocks and launchers of the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/beagle.h"
#include "beagle_device.h"

namespace bgl {

constexpr int GRAD_SHORT_WORDS = 64;   // tape in registers up to this many decoded words
constexpr int GRAD_LONG_WORDS = 256;   // tape in LDS up to this many (longer: TOO_LONG)
constexpr int GRAD_SMALL_WORDS = 48;   // small-stack adjoint (2 cases per lane) up to this many

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
  const int32_t* list_count;  // [4]: short tape, long tape, small stack <= 48 words, small stack <= 64
  const int32_t* list;        // [4][n_programs]
  unsigned long long* work;   // [4] work-item counters, zero at launch
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
  double* fitness;
  float* grad;
};

__global__ void k_grad_finalize(GradFinalizeArgs a);
size_t grad_lds_bytes(int D, bool long_tape);
hipError_t launch_grad(const GradArgs& a, hipStream_t s);

}  // namespace bgl
