// Tile-width tuner of the evaluator: picks, per problem-shape bucket, how
// many cases each lane carries for the common (stack <= 4) programs.  Both
// widths add the same cases in the same order, so the choice is a pure
// speed decision and never changes a result.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "host.h"

namespace bgl {
namespace host {

static TuneKey bucket(int kind, int D, int64_t M, double mean_len) {
  const int mlog = int(std::lround(std::log2(double(std::max<int64_t>(M, 1)))));
  const int llog = int(std::lround(std::log2(std::max(mean_len, 1.0))));
  return TuneKey(kind, D, mlog, llog);
}

void load_tune_file(beagle_ctx* ctx) {
  const char* path = std::getenv("BEAGLE_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  ctx->tune_file = path;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    int kind = 0, D = 0, ml = 0, ll = 0, kv = 0;
    if (is >> kind >> D >> ml >> ll >> kv && (kv == 0 || kv == 1)) ctx->tuned[TuneKey(kind, D, ml, ll)] = kv;
  }
}

static void save_tune_file(const beagle_ctx* ctx) {
  if (ctx->tune_file.empty()) return;
  const std::string tmp = ctx->tune_file + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return;
    f << "# kind D round(log2 M) round(log2 mean program length) variant (0: 8 cases per lane, 1: 4)\n";
    for (const auto& e : ctx->tuned)
      f << std::get<0>(e.first) << ' ' << std::get<1>(e.first) << ' ' << std::get<2>(e.first) << ' '
        << std::get<3>(e.first) << ' ' << e.second << '\n';
  }
  (void)std::rename(tmp.c_str(), ctx->tune_file.c_str());
}

bool known_tile_variant(const beagle_ctx* ctx, int kind, int D, int64_t M, double mean_len, int* kv) {
  if (D > WIDE_TILE_MAX_D || ctx->tuning == BEAGLE_TUNE_NARROW) {
    *kv = 1;
    return true;
  }
  if (ctx->tuning == BEAGLE_TUNE_WIDE) {
    *kv = 0;
    return true;
  }
  const auto it = ctx->tuned.find(bucket(kind, D, M, mean_len));
  if (it == ctx->tuned.end()) return false;
  *kv = it->second;
  return true;
}

beagle_status tile_variant(beagle_ctx* ctx, int kind, int D, int64_t M, double mean_len, hipStream_t s,
                           TuneRun run, void* user, int* kv) {
  if (known_tile_variant(ctx, kind, D, M, mean_len, kv)) return BEAGLE_OK;
  *kv = 0;
  // no measurement while the caller's stream is being captured into a graph
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return BEAGLE_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  // one warm-up per variant, then five alternating timed runs; the fastest
  // run of each decides (interference only ever slows a run down)
  constexpr int R = 5;
  float t[2][R] = {};
  for (int v = 0; v < 2 && e == hipSuccess; ++v) e = run(user, v, s, nullptr, nullptr);
  for (int r = 0; r < R && e == hipSuccess; ++r) {
    for (int v = 0; v < 2 && e == hipSuccess; ++v) {
      e = run(user, v, s, e0, e1);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t[v][r], e0, e1);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "tile-width measurement");
  for (auto& row : t) std::sort(row, row + R);
  *kv = t[1][0] < t[0][0] ? 1 : 0;
  ctx->tuned[bucket(kind, D, M, mean_len)] = *kv;
  save_tune_file(ctx);
  return BEAGLE_OK;
}

}  // namespace host
}  // namespace bgl
