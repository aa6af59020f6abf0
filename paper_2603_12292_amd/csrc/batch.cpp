// Ragged batching: many independent problems (each its own population,
// cases and variables) in one launch sequence, captured once as a HIP graph
// and replayed while the problem table is unchanged.
//
// The device problem table holds, per problem, the caller's pointers and
// that problem's share of the workspace.  Every kernel of the sequence
// covers the whole table: preparation and finalize run one thread per
// program of any problem, staging one thread per padded case, and the
// evaluation kernels pull (problem, chunk, program) items from work lists
// that span all problems.  Problems enter the table in decreasing order of
// estimated work (tokens x cases), so the small items of small problems
// fill the tail of each persistent launch.  Each problem keeps the case
// chunking, tile order and reduction order it has when evaluated alone, so
// its fitness values are bit-identical to beagle_eval's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/beagle.h"
#include "grad.h"
#include "host.h"
#include "kernels.h"

namespace bgl {
namespace host {

void release_graphs(beagle_ctx* ctx) {
  for (auto& g : ctx->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  ctx->graphs.clear();
}

}  // namespace host
}  // namespace bgl

namespace {

using namespace bgl::host;

constexpr size_t MAX_GRAPHS = 8;

struct Batch {
  bgl::BatchArgs args;
  int max_d[bgl::N_BATCH_LISTS];
  int has[bgl::N_BATCH_LISTS];
  int64_t n_programs = 0, n_cases = 0;
  int n = 0;
};

// Enqueues the whole batched evaluation on `s` (the capture stream).
hipError_t enqueue(const Batch& b, int32_t* counts, hipStream_t s) {
  zero_i32(counts, int64_t(64) * b.n, s);
  const uint32_t pgrid = uint32_t((b.n_programs + 255) / 256);
  hipLaunchKernelGGL(bgl::k_layout_check_batch, dim3(pgrid), dim3(256), 0, s, b.args);
  hipLaunchKernelGGL(bgl::k_layout_fill_batch, dim3(64, uint32_t(b.n)), dim3(256), 0, s, b.args);
  hipLaunchKernelGGL(bgl::k_layout_mark_batch, dim3(std::min<uint32_t>(pgrid, 1024)), dim3(256), 0, s, b.args);
  hipLaunchKernelGGL(bgl::k_prepare_batch, dim3(uint32_t((b.n_programs + 63) / 64)), dim3(64), 0, s, b.args);
  hipLaunchKernelGGL(bgl::k_stage_batch, dim3(uint32_t((b.n_cases + 255) / 256)), dim3(256), 0, s, b.args);
  if (b.args.kind == BEAGLE_FIT_CORR) {
    hipLaunchKernelGGL(bgl::k_target_stats_batch, dim3(uint32_t(b.n)), dim3(1024), 0, s, b.args);
    hipLaunchKernelGGL(bgl::k_values_batch, dim3(uint32_t(b.n_programs)), dim3(64), 0, s, b.args);
  }
  hipLaunchKernelGGL(bgl::k_batch_items, dim3(1), dim3(64), 0, s, b.args);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = bgl::launch_eval_batch(b.args.kind, b.args, b.max_d, b.has, s, nullptr, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bgl::k_finalize_batch, dim3(uint32_t((b.n_programs + 255) / 256)), dim3(256), 0, s, b.args);
  return hipGetLastError();
}

}  // namespace

extern "C" {

beagle_status beagle_eval_batched(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                                  int32_t n_problems, int kind, double* const* fitness, int8_t* const* status,
                                  beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  if (kind != BEAGLE_FIT_MSE && kind != BEAGLE_FIT_CORR) return fail(BEAGLE_E_INVALID_ARG, "unknown fitness kind");
  if (n_problems < 0 || n_problems > 65535) return fail(BEAGLE_E_INVALID_ARG, "n_problems must be in [0, 65535]");
  if (n_problems == 0) return BEAGLE_OK;
  if (!progs || !data || !fitness) return fail(BEAGLE_E_INVALID_ARG, "progs, data or fitness is NULL");
  std::vector<int> active;
  for (int q = 0; q < n_problems; ++q) {
    beagle_status st = check_programs(&progs[q]);
    if (st == BEAGLE_OK) st = check_data(&data[q], kind);
    if (st != BEAGLE_OK) return fail(st, "problem " + std::to_string(q) + ": " + last_error());
    if (progs[q].n_programs == 0) continue;
    if (!fitness[q]) return fail(BEAGLE_E_INVALID_ARG, "fitness[" + std::to_string(q) + "] is NULL");
    active.push_back(q);
  }
  if (active.empty()) return BEAGLE_OK;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n_sums = kind == BEAGLE_FIT_MSE ? 1 : 3;

  // tile widths: a bucket met for the first time is measured by evaluating
  // one of its problems alone (through beagle_eval, which tunes it)
  std::vector<int> kv(n_problems, 1);
  for (int q : active) {
    const double mean_len = double(progs[q].n_tokens) / progs[q].n_programs;
    if (!known_tile_variant(ctx, kind, data[q].D, data[q].M, mean_len, &kv[q])) {
      beagle_status st = beagle_eval(ctx, &progs[q], &data[q], kind, fitness[q], status ? status[q] : nullptr,
                                     stream);
      if (st != BEAGLE_OK) return st;
      if (!known_tile_variant(ctx, kind, data[q].D, data[q].M, mean_len, &kv[q])) kv[q] = 0;
    }
  }

  // table order: decreasing estimated work, ties by problem index
  std::stable_sort(active.begin(), active.end(), [&](int a, int b) {
    return double(progs[a].n_tokens) * double(data[a].M) > double(progs[b].n_tokens) * double(data[b].M);
  });
  const int n = int(active.size());

  // workspace layout
  Carve c;
  const size_t at_table = c.take<bgl::BatchProblem>(n);
  const size_t at_items = c.take<int64_t>(size_t(bgl::N_BATCH_LISTS) * (n + 1));
  const size_t at_work = c.take<unsigned long long>(bgl::N_BATCH_LISTS);
  const size_t at_counts = c.take<int32_t>(size_t(64) * n);
  struct Off {
    size_t code, aux, cval, s_stack, s_start, s_need, owner, meta, class_list, len_list, Xt, yp, stats, part;
    int64_t Mp, chunk;
    int32_t n_chunks;
  };
  std::vector<Off> off(n);
  for (int i = 0; i < n; ++i) {
    const beagle_programs& P = progs[active[i]];
    const beagle_dataset& d = data[active[i]];
    const int64_t nt = std::max<int64_t>(P.n_tokens, 1);
    const int64_t N = P.n_programs;
    Off& o = off[i];
    o.code = c.take<uint32_t>(nt);
    o.aux = c.take<uint32_t>(nt);
    o.cval = c.take<float>(nt);
    o.s_stack = c.take<int32_t>(nt);
    o.s_start = c.take<int32_t>(nt);
    o.s_need = c.take<int32_t>(nt);
    o.owner = c.take<int32_t>(nt);
    o.meta = c.take<bgl::ProgMeta>(N);
    o.class_list = c.take<int32_t>(size_t(bgl::N_CLASSES) * N);
    o.len_list = c.take<int32_t>(size_t(bgl::GRAD_LISTS) * N);
    o.Mp = round_up(d.M, bgl::CASES_PER_BLOCK_ITER);
    o.Xt = c.take<float>(size_t(d.D) * o.Mp);
    o.yp = c.take<float>(o.Mp);
    o.stats = c.take<double>(4);
    choose_chunks(d.M, N, &o.chunk, &o.n_chunks, 32768, bgl::CASES_PER_BLOCK_ITER);
    o.part = c.take<double>(size_t(n_sums) * o.n_chunks * N);
  }
  beagle_status st = reserve(ctx, c.used + 256);
  if (st != BEAGLE_OK) return st;
  char* ws = ctx->ws;

  // the previous upload must have read the host table before it is rewritten
  if (ctx->table_copied) {
    hipError_t e = hipEventSynchronize(ctx->table_copied);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  ctx->table.assign(n, bgl::BatchProblem{});
  Batch b;
  std::memset(&b.args, 0, sizeof(b.args));
  b.n = n;
  for (int v = 0; v < bgl::N_BATCH_LISTS; ++v) b.max_d[v] = b.has[v] = 0;
  int32_t* counts = reinterpret_cast<int32_t*>(ws + at_counts);
  for (int i = 0; i < n; ++i) {
    const int q = active[i];
    const beagle_programs& P = progs[q];
    const beagle_dataset& d = data[q];
    const Off& o = off[i];
    bgl::BatchProblem& t = ctx->table[i];
    std::memset(&t, 0, sizeof(t));
    bgl::PrepareArgs& pa = t.prep;
    pa.tokens = P.tokens;
    pa.n_tokens = P.n_tokens;
    pa.tok_offset = P.tok_offset;
    pa.tok_len = P.tok_len;
    pa.consts = P.consts;
    pa.n_consts = P.n_consts;
    pa.const_offset = P.const_offset;
    pa.const_count = P.const_count;
    pa.n_programs = P.n_programs;
    pa.D = d.D;
    pa.code = reinterpret_cast<uint32_t*>(ws + o.code);
    pa.aux = reinterpret_cast<uint32_t*>(ws + o.aux);
    pa.cval = reinterpret_cast<float*>(ws + o.cval);
    pa.max_words = bgl::MAX_LEN;
    pa.scr_stack = reinterpret_cast<int32_t*>(ws + o.s_stack);
    pa.scr_start = reinterpret_cast<int32_t*>(ws + o.s_start);
    pa.scr_need = reinterpret_cast<int32_t*>(ws + o.s_need);
    pa.meta = reinterpret_cast<bgl::ProgMeta*>(ws + o.meta);
    pa.status_out = status ? status[q] : nullptr;
    pa.class_count = counts + int64_t(64) * i;
    pa.class_list = reinterpret_cast<int32_t*>(ws + o.class_list);
    pa.len_count = counts + int64_t(64) * i + 8;
    pa.len_list = reinterpret_cast<int32_t*>(ws + o.len_list);
    pa.short_words = bgl::GRAD_SHORT_WORDS;
    pa.adjoint = 0;
    pa.long_count = nullptr;  // k_prepare_batch decodes every program itself
    pa.long_list = nullptr;
    pa.layout = counts + int64_t(64) * i + 32;
    pa.owner = reinterpret_cast<int32_t*>(ws + o.owner);
    pa.cowner = nullptr;
    pa.wave_programs = 64;
    t.X = d.X;
    t.y = d.y;
    t.Xt = reinterpret_cast<float*>(ws + o.Xt);
    t.yp = reinterpret_cast<float*>(ws + o.yp);
    t.stats = reinterpret_cast<double*>(ws + o.stats);
    t.part = reinterpret_cast<double*>(ws + o.part);
    t.fitness = fitness[q];
    t.M = d.M;
    t.Mp = o.Mp;
    t.chunk = o.chunk;
    t.n_chunks = o.n_chunks;
    t.kv = d.D <= bgl::WIDE_TILE_MAX_D ? kv[q] : 1;
    t.prog_begin = b.n_programs;
    t.case_begin = b.n_cases;
    b.n_programs += P.n_programs;
    b.n_cases += o.Mp;
    // the problem's lists: its class-0 tile variant and classes 1 and 2,
    // in the bucket of its variable count
    const int db = bgl::d_bucket(int(d.D));
    for (int v : {int(t.kv), 2, 3}) {
      const int vl = v * bgl::N_DBUCKETS + db;
      b.has[vl] = 1;
      b.max_d[vl] = std::max(b.max_d[vl], int(d.D));
    }
  }
  if (b.n_programs >= (int64_t(1) << 31)) return fail(BEAGLE_E_UNSUPPORTED, "more than 2^31 programs in a batch");
  bgl::BatchArgs& a = b.args;
  a.table = reinterpret_cast<const bgl::BatchProblem*>(ws + at_table);
  a.n_problems = n;
  a.kind = kind;
  a.n_programs = b.n_programs;
  a.n_cases = b.n_cases;
  a.item_off = reinterpret_cast<int64_t*>(ws + at_items);
  a.work = reinterpret_cast<unsigned long long*>(ws + at_work);

  // upload the table (outside the graph), then launch the graph for it
  const size_t table_bytes = sizeof(bgl::BatchProblem) * n;
  hipError_t e = hipMemcpyAsync(ws + at_table, ctx->table.data(), table_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "problem table upload");
  if (!ctx->table_copied && (e = hipEventCreateWithFlags(&ctx->table_copied, hipEventDisableTiming)) != hipSuccess)
    return hip_fail(e, "hipEventCreate");
  if ((e = hipEventRecord(ctx->table_copied, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");

  std::string key(reinterpret_cast<const char*>(ctx->table.data()), table_bytes);
  key.append(reinterpret_cast<const char*>(&a), sizeof(a));
  BatchGraph* gr = nullptr;
  for (auto& x : ctx->graphs)
    if (x.key == key) gr = &x;
  if (!gr) {
    if (!ctx->capture_stream &&
        (e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "hipStreamCreate");
    if (ctx->graphs.size() >= MAX_GRAPHS) {
      // evict the least recently used graph (none can be running: launches
      // of a graph exec are ordered on their streams, and an exec is only
      // destroyed after the device has drained)
      auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                  [](const BatchGraph& x, const BatchGraph& y) { return x.last_use < y.last_use; });
      if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      (void)hipGraphExecDestroy(lru->exec);
      (void)hipGraphDestroy(lru->graph);
      ctx->graphs.erase(lru);
    }
    BatchGraph ng;
    ng.key = key;
    bgl::prime_eval_batch(kind, b.max_d, b.has);
    e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = enqueue(b, counts, ctx->capture_stream);
    e = hipStreamEndCapture(ctx->capture_stream, &ng.graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (ng.graph) (void)hipGraphDestroy(ng.graph);
      return hip_fail(le != hipSuccess ? le : e, "batched launch capture");
    }
    e = hipGraphInstantiate(&ng.exec, ng.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(ng.graph);
      return hip_fail(e, "hipGraphInstantiate");
    }
    ctx->graphs.push_back(ng);
    gr = &ctx->graphs.back();
    ++ctx->graph_captures;
  }
  gr->last_use = ++ctx->use_clock;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (ctx->timing) {
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
      return fail(BEAGLE_E_HIP, "hipEventCreate");
    ctx->events.emplace_back(ev0, ev1);
    (void)hipEventRecord(ev0, s);
  }
  e = hipGraphLaunch(gr->exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  if (ev1) (void)hipEventRecord(ev1, s);
  ++ctx->graph_replays;
  clear_error();
  return BEAGLE_OK;
}

beagle_status beagle_ctx_graph_stats(beagle_ctx* ctx, int64_t* captures, int64_t* replays) {
  if (!ctx || !captures || !replays) return fail(BEAGLE_E_INVALID_ARG, "NULL argument");
  *captures = ctx->graph_captures;
  *replays = ctx->graph_replays;
  return BEAGLE_OK;
}

}  // extern "C"
