// Host-side internals shared by the C ABI files: the context, error
// reporting, workspace management, argument checks and the tile-width tuner.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/beagle.h"
#include "kernels.h"

namespace bgl {
namespace host {

// Problem-shape bucket of the tile-width tuner: (kind, D, round(log2 M),
// round(log2 mean program length)).
using TuneKey = std::tuple<int, int, int, int>;

// A captured batched launch sequence and what it was captured for.
struct BatchGraph {
  std::string key;  // bytes of the problem table + kind + workspace address
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

}  // namespace host
}  // namespace bgl

struct beagle_ctx {
  int device = 0;
  size_t cap = 0;       // 0 = unlimited
  char* ws = nullptr;   // device workspace
  size_t ws_size = 0;
  bool timing = false;  // record events around the main evaluation kernel
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  int tuning = BEAGLE_TUNE_AUTO;
  int decoder = BEAGLE_DECODE_WAVE;  // decoder of programs of at most 64 tokens
  // side stream of the target statistics (beside the decoding), created on
  // first use, with its fork and join events
  hipStream_t side = nullptr;
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  std::map<bgl::host::TuneKey, int> tuned;  // bucket -> tile variant (0 wide, 1 narrow)
  std::string tune_file;                    // BEAGLE_AUTOTUNE_CACHE at creation ("" = none)
  // batched evaluation
  std::vector<bgl::host::BatchGraph> graphs;
  hipStream_t capture_stream = nullptr;  // graphs are captured here, launched on the caller's stream
  std::vector<bgl::BatchProblem> table;  // host copy of the last uploaded problem table
  hipEvent_t table_copied = nullptr;     // the last table upload has read `table`
  uint64_t use_clock = 0;
  int64_t graph_captures = 0, graph_replays = 0;
};

namespace bgl {
namespace host {

beagle_status fail(beagle_status s, const std::string& msg);
beagle_status hip_fail(hipError_t e, const char* where);
void clear_error();
const char* last_error();

// Makes ctx->device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Bump allocator over the context workspace (256-byte aligned pieces).
struct Carve {
  size_t used = 0;
  template <class T>
  size_t take(size_t count) {
    const size_t at = (used + 255) & ~size_t(255);
    used = at + count * sizeof(T);
    return at;
  }
};

// Grows the workspace to `bytes` (synchronises the device and drops the
// captured graphs when it moves).
beagle_status reserve(beagle_ctx* ctx, size_t bytes);
beagle_status check_programs(const beagle_programs* p);
beagle_status check_data(const beagle_dataset* d, int kind);
int64_t round_up(int64_t v, int64_t m);
// Case chunks of one call: at most max_chunk_cases cases each (rounded up to
// a multiple of unit, the cases one kernel iteration covers), more when the
// population alone gives too few work items.
void choose_chunks(int64_t M, int64_t N, int64_t* chunk, int32_t* n_chunks, int64_t max_chunk_cases, int64_t unit);
void zero_i32(int32_t* p, int64_t n, hipStream_t s);

// Tile variant of class 0 for a problem (0 wide, 1 narrow).  Under
// BEAGLE_TUNE_AUTO a bucket met for the first time is measured: `run(kv)`
// must enqueue one evaluation of the problem with that variant on `s`
// between the two events it is given.
using TuneRun = hipError_t (*)(void* user, int kv, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
beagle_status tile_variant(beagle_ctx* ctx, int kind, int D, int64_t M, double mean_len, hipStream_t s,
                           TuneRun run, void* user, int* kv);
// The variant without measuring: false when AUTO has not yet met the bucket.
bool known_tile_variant(const beagle_ctx* ctx, int kind, int D, int64_t M, double mean_len, int* kv);
void load_tune_file(beagle_ctx* ctx);
void release_graphs(beagle_ctx* ctx);

}  // namespace host
}  // namespace bgl
