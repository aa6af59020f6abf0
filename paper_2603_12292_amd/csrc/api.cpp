// C ABI of the library: contexts, workspace, argument checks and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/beagle.h"
#include "beagle_device.h"
#include "gen.h"
#include "grad.h"
#include "host.h"
#include "kernels.h"

namespace bgl {
namespace host {

static thread_local std::string g_error;

beagle_status fail(beagle_status s, const std::string& msg) {
  g_error = msg;
  return s;
}

beagle_status hip_fail(hipError_t e, const char* where) {
  return fail(BEAGLE_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

void clear_error() { g_error.clear(); }

const char* last_error() { return g_error.c_str(); }

beagle_status reserve(beagle_ctx* ctx, size_t bytes) {
  if (ctx->cap && bytes > ctx->cap)
    return fail(BEAGLE_E_NOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the context cap of " +
                                    std::to_string(ctx->cap));
  if (bytes <= ctx->ws_size) return BEAGLE_OK;
  // the old workspace may still be in use by queued work on any stream
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  release_graphs(ctx);  // they point into the old workspace
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_size = 0;
  size_t want = std::max(bytes, size_t(1) << 20);
  if (!ctx->cap) want = std::max(want, bytes + bytes / 4);
  if (ctx->cap) want = std::min(want, ctx->cap);
  e = hipMalloc(reinterpret_cast<void**>(&ctx->ws), want);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    return fail(BEAGLE_E_NOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
  }
  ctx->ws_size = want;
  return BEAGLE_OK;
}

beagle_status check_programs(const beagle_programs* p) {
  if (!p) return fail(BEAGLE_E_INVALID_ARG, "programs is NULL");
  if (p->n_programs < 0) return fail(BEAGLE_E_INVALID_ARG, "n_programs < 0");
  if (p->n_tokens < 0 || p->n_consts < 0) return fail(BEAGLE_E_INVALID_ARG, "n_tokens or n_consts < 0");
  if (p->n_programs == 0) return BEAGLE_OK;
  if (!p->tok_offset || !p->tok_len || !p->const_offset || !p->const_count)
    return fail(BEAGLE_E_INVALID_ARG, "a program array pointer is NULL");
  if (p->n_tokens > 0 && !p->tokens) return fail(BEAGLE_E_INVALID_ARG, "tokens is NULL");
  if (p->n_consts > 0 && !p->consts) return fail(BEAGLE_E_INVALID_ARG, "consts is NULL");
  if (p->n_tokens >= (int64_t(1) << 31)) return fail(BEAGLE_E_UNSUPPORTED, "n_tokens >= 2^31");
  return BEAGLE_OK;
}

beagle_status check_data(const beagle_dataset* d, int kind) {
  if (!d) return fail(BEAGLE_E_INVALID_ARG, "data is NULL");
  if (d->D < 1 || d->D > BEAGLE_MAX_D) return fail(BEAGLE_E_UNSUPPORTED, "D must be in [1, 16]");
  if (d->M < 1) return fail(BEAGLE_E_INVALID_ARG, "M must be >= 1");
  if (kind == BEAGLE_FIT_CORR && d->M < 2) return fail(BEAGLE_E_INVALID_ARG, "correlation fitness needs M >= 2");
  if (d->M > (int64_t(1) << 40)) return fail(BEAGLE_E_UNSUPPORTED, "M too large");
  if (!d->X || !d->y) return fail(BEAGLE_E_INVALID_ARG, "X or y is NULL");
  return BEAGLE_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Case chunking of the evaluation grid: about 32K cases per chunk, more
// chunks when the population alone gives too few workgroups to fill the GPU.
void choose_chunks(int64_t M, int64_t N, int64_t* chunk, int32_t* n_chunks, int64_t max_chunk_cases, int64_t unit) {
  const int64_t max_chunks = std::max<int64_t>(1, (M + unit - 1) / unit);
  int64_t C = std::max<int64_t>(1, (M + max_chunk_cases - 1) / max_chunk_cases);
  const int64_t target_blocks = 4096;
  if (N * C < target_blocks) C = std::max<int64_t>(C, (target_blocks + N - 1) / std::max<int64_t>(N, 1));
  C = std::min(C, max_chunks);
  const int64_t ch = round_up((M + C - 1) / C, unit);
  *chunk = ch;
  *n_chunks = int32_t((M + ch - 1) / ch);
}

static __global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void zero_i32(int32_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, s, p, n);
}

}  // namespace host
}  // namespace bgl

namespace {

using namespace bgl::host;

// The pieces of workspace one evaluation uses.
struct EvalLayout {
  size_t code, aux, cval, s_stack, s_start, s_need, owner, cowner, meta, class_count, class_list, len_list, long_list,
      work, Xt, yp, stats, part, gpart, coef, total;
  int64_t Mp, chunk, gchunk;      // case chunks of the evaluation and of the adjoint
  int32_t n_chunks, gn_chunks, slice;
};

EvalLayout eval_layout(const beagle_programs* P, const beagle_dataset* d, int n_sums, int32_t slice,
                       bool with_grad = false) {
  EvalLayout L{};
  Carve c;
  const int64_t nt = std::max<int64_t>(P->n_tokens, 1);
  const int64_t N = std::max<int32_t>(P->n_programs, 1);
  L.code = c.take<uint32_t>(nt);
  L.aux = c.take<uint32_t>(nt);
  L.cval = c.take<float>(nt);
  L.s_stack = c.take<int32_t>(nt);
  L.s_start = c.take<int32_t>(nt);
  L.s_need = c.take<int32_t>(nt);
  L.owner = c.take<int32_t>(nt);
  L.cowner = with_grad ? c.take<int32_t>(std::max<int64_t>(P->n_consts, 1)) : 0;
  L.meta = c.take<bgl::ProgMeta>(N);
  L.class_count = c.take<int32_t>(64);  // [0..2] need classes, [8..9] length classes, [32..33] layout flags
  // right behind the counters (256 bytes): one clear covers both
  L.work = c.take<unsigned long long>(8);  // evaluation: one per class; adjoint: one per list
  L.class_list = c.take<int32_t>(size_t(bgl::N_CLASSES) * N);
  L.len_list = c.take<int32_t>(size_t(bgl::GRAD_LISTS) * N);
  L.long_list = c.take<int32_t>(size_t(N));
  L.Mp = round_up(d->M, bgl::CASES_PER_BLOCK_ITER);
  L.Xt = c.take<float>(size_t(d->D) * L.Mp);
  L.yp = c.take<float>(L.Mp);
  L.stats = c.take<double>(4);
  L.slice = slice;
  // the chunking depends on the whole population only, so that a sliced
  // evaluation sums every program's partials in the same order
  choose_chunks(d->M, N, &L.chunk, &L.n_chunks, 32768, bgl::CASES_PER_BLOCK_ITER);
  // the adjoint's kernels each walk one list of programs: shorter chunks
  // keep a short list from leaving most of the chip idle
  L.gchunk = 0;
  L.gn_chunks = 0;
  if (with_grad) choose_chunks(d->M, N, &L.gchunk, &L.gn_chunks, bgl::GRAD_CHUNK_CASES, bgl::GRAD_TILE_CASES);
  L.part = c.take<double>(std::max<size_t>(size_t(n_sums) * L.n_chunks * slice, size_t(L.gn_chunks) * N));
  L.gpart = with_grad ? c.take<double>(size_t(L.gn_chunks) * std::max<int64_t>(P->n_consts, 1)) : 0;
  L.coef = with_grad ? c.take<double>(size_t(3) * N) : 0;
  L.total = c.used + 256;
  return L;
}

// Validation + decoding of the programs and staging of the cases (shared by
// evaluation, prediction and the gradient).
beagle_status prepare(char* ws, const beagle_programs* P, const beagle_dataset* d, const EvalLayout& L,
                      int8_t* status, hipStream_t s, int decoder, int32_t max_words = bgl::MAX_LEN,
                      bool adjoint = false) {
  // the decoder's counters and flags, and the work counters of the first
  // interpreter launch
  zero_i32(reinterpret_cast<int32_t*>(ws + L.class_count), int64_t(L.work - L.class_count) / 4 + 16, s);
  bgl::PrepareArgs pa;
  pa.tokens = P->tokens;
  pa.n_tokens = P->n_tokens;
  pa.tok_offset = P->tok_offset;
  pa.tok_len = P->tok_len;
  pa.consts = P->consts;
  pa.n_consts = P->n_consts;
  pa.const_offset = P->const_offset;
  pa.const_count = P->const_count;
  pa.n_programs = P->n_programs;
  pa.D = d->D;
  pa.code = reinterpret_cast<uint32_t*>(ws + L.code);
  pa.aux = reinterpret_cast<uint32_t*>(ws + L.aux);
  pa.cval = reinterpret_cast<float*>(ws + L.cval);
  pa.max_words = max_words;
  pa.scr_stack = reinterpret_cast<int32_t*>(ws + L.s_stack);
  pa.scr_start = reinterpret_cast<int32_t*>(ws + L.s_start);
  pa.scr_need = reinterpret_cast<int32_t*>(ws + L.s_need);
  pa.meta = reinterpret_cast<bgl::ProgMeta*>(ws + L.meta);
  pa.status_out = status;
  pa.class_count = reinterpret_cast<int32_t*>(ws + L.class_count);
  pa.class_list = reinterpret_cast<int32_t*>(ws + L.class_list);
  pa.len_count = reinterpret_cast<int32_t*>(ws + L.class_count) + 8;
  pa.len_list = reinterpret_cast<int32_t*>(ws + L.len_list);
  pa.short_words = bgl::GRAD_SHORT_WORDS;
  pa.adjoint = adjoint ? 1 : 0;
  pa.long_count = reinterpret_cast<int32_t*>(ws + L.class_count) + 16;
  pa.long_list = reinterpret_cast<int32_t*>(ws + L.long_list);
  pa.layout = reinterpret_cast<int32_t*>(ws + L.class_count) + 32;
  pa.owner = reinterpret_cast<int32_t*>(ws + L.owner);
  pa.cowner = adjoint ? reinterpret_cast<int32_t*>(ws + L.cowner) : nullptr;
  pa.wave_programs = 64;
  bgl::StageArgs sa;
  sa.X = d->X;
  sa.y = d->y;
  sa.M = d->M;
  sa.Mp = L.Mp;
  sa.D = d->D;
  sa.Xt = reinterpret_cast<float*>(ws + L.Xt);
  sa.yp = reinterpret_cast<float*>(ws + L.yp);
  // staging of the cases beside the disjoint-ranges check (the fill and
  // mark passes return at once when the ranges are sorted and disjoint),
  // then programs of at most 64 tokens, then the ones longer than that
  const uint32_t pgrid = uint32_t((P->n_programs + 255) / 256);
  const uint32_t sgrid = uint32_t(std::min<int64_t>((L.Mp + 255) / 256, 1 << 16));
  hipLaunchKernelGGL(bgl::k_stage_and_check, dim3(sgrid + pgrid), dim3(256), 0, s, sa, pa, sgrid);
  hipLaunchKernelGGL(bgl::k_layout_fill, dim3(1024), dim3(256), 0, s, pa);
  hipLaunchKernelGGL(bgl::k_layout_mark, dim3(std::min<uint32_t>(pgrid, 1024)), dim3(256), 0, s, pa);
  if (decoder == BEAGLE_DECODE_THREAD)
    hipLaunchKernelGGL(bgl::k_prepare, dim3((P->n_programs + 63) / 64), dim3(64), 0, s, pa);
  else {
    // programs per wave: 32 for large populations (more, shorter waves end
    // more evenly; 64 left the last round's slowest waves alone on the chip:
    // 1-2 % longer at 2^20 programs, though short programs pack better),
    // fewer when that leaves under 4096 waves (16 per CU), so that small
    // populations still fill the chip
    const int64_t n = P->n_programs;
    pa.wave_programs = int32_t(std::max<int64_t>(1, std::min<int64_t>(32, n / 4096)));
    const int64_t waves = (n + pa.wave_programs - 1) / pa.wave_programs;
    hipLaunchKernelGGL(adjoint ? bgl::k_prepare_wave<true> : bgl::k_prepare_wave<false>,
                       dim3(uint32_t((waves + 3) / 4)), dim3(256), 0, s, pa);
  }
  hipLaunchKernelGGL(bgl::k_prepare_long, dim3(512), dim3(64), 0, s, pa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "prepare launch");
  return BEAGLE_OK;
}

// LDS of a values kernel: the case tile of D variables (256 floats each).
size_t values_lds(int32_t D) { return size_t(D < 1 ? 1 : D) * 256 * sizeof(float); }

beagle_status launch_values(char* ws, const beagle_programs* P, const beagle_dataset* d,
                            const EvalLayout& L, int64_t m, float* out, int shift_mode, hipStream_t s) {
  bgl::ValuesArgs va;
  va.code = reinterpret_cast<const uint32_t*>(ws + L.code);
  va.cval = reinterpret_cast<const float*>(ws + L.cval);
  va.tok_offset = P->tok_offset;
  va.meta = reinterpret_cast<bgl::ProgMeta*>(ws + L.meta);
  va.Xt = reinterpret_cast<const float*>(ws + L.Xt);
  va.Mp = L.Mp;
  va.m = m;
  va.D = d->D;
  va.n_programs = P->n_programs;
  va.out = out;
  va.shift_mode = shift_mode;
  const int64_t tiles = (m + 63) / 64;
  if (tiles > 65535) return fail(BEAGLE_E_UNSUPPORTED, "predict: M > 4194240");
  hipLaunchKernelGGL(bgl::k_values, dim3(P->n_programs, uint32_t(tiles)), dim3(64), values_lds(d->D), s, va);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "values launch");
  return BEAGLE_OK;
}

// The correlation shifts before an evaluation (correlation fitness and the
// Eq. 2 score).  When the shape takes the resident-inputs kernels, the
// shifts of classes 0 and 1 come from those kernels' first pass
// (*in_kernel = true) and only the class-2 programs run the shift pass here.
beagle_status launch_shifts(char* ws, const beagle_programs* P, const beagle_dataset* d, const EvalLayout& L,
                            hipStream_t s, bool* in_kernel) {
  *in_kernel = bgl::resident_eligible(d->M, d->D, L.n_chunks, P->n_programs);
  if (!*in_kernel) return launch_values(ws, P, d, L, 1, nullptr, 1, s);
  bgl::ValuesArgs va;
  va.code = reinterpret_cast<const uint32_t*>(ws + L.code);
  va.cval = reinterpret_cast<const float*>(ws + L.cval);
  va.tok_offset = P->tok_offset;
  va.meta = reinterpret_cast<bgl::ProgMeta*>(ws + L.meta);
  va.Xt = reinterpret_cast<const float*>(ws + L.Xt);
  va.Mp = L.Mp;
  va.m = 1;
  va.D = d->D;
  va.n_programs = P->n_programs;
  va.out = nullptr;
  va.shift_mode = 1;
  hipLaunchKernelGGL(bgl::k_values_deep, dim3(2048), dim3(64), values_lds(d->D), s, va,
                     reinterpret_cast<const int32_t*>(ws + L.class_count),
                     reinterpret_cast<const int32_t*>(ws + L.class_list), P->n_programs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "values launch");
  return BEAGLE_OK;
}

// Target statistics of data->y (correlation fitness, Eq. 2 score) into
// `stats`.  They read nothing else, so with a context they run on its side
// stream (default priority), forked from s here and beside the decoding and
// staging that follow on s; *join is then the event s waits for before the
// statistics are read.  Without a context they run on s (*join = null).
beagle_status launch_target_stats(beagle_ctx* ctx, const beagle_dataset* data, double* stats, hipStream_t s,
                                  hipEvent_t* join) {
  *join = nullptr;
  hipStream_t t = s;
  if (ctx) {
    if (!ctx->side) {
      hipStream_t ns = nullptr;
      hipEvent_t f = nullptr, j = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&ns, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
      if (e != hipSuccess) {
        if (ns) (void)hipStreamDestroy(ns);
        if (f) (void)hipEventDestroy(f);
        return hip_fail(e, "side stream");
      }
      ctx->side = ns;
      ctx->side_fork = f;
      ctx->side_join = j;
    }
    hipError_t e = hipEventRecord(ctx->side_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->side_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "side stream fork");
    t = ctx->side;
  }
  hipLaunchKernelGGL(bgl::k_target_stats, dim3(1), dim3(1024), 0, t, data->y, data->M, stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "target statistics launch");
  if (ctx) {
    if ((e = hipEventRecord(ctx->side_join, t)) != hipSuccess) return hip_fail(e, "side stream join");
    *join = ctx->side_join;
  }
  return BEAGLE_OK;
}

// s waits for the target statistics (when they ran on a side stream).
beagle_status join_target_stats(hipEvent_t join, hipStream_t s) {
  if (!join) return BEAGLE_OK;
  const hipError_t e = hipStreamWaitEvent(s, join, 0);
  return e == hipSuccess ? BEAGLE_OK : hip_fail(e, "side stream join");
}

// One evaluation slice for the tile-width tuner.
struct TuneSlice {
  int kind;
  bgl::EvalArgs ea;
};

hipError_t run_slice(void* user, int kv, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const TuneSlice* t = static_cast<const TuneSlice*>(user);
  return bgl::launch_eval(t->kind, kv, t->ea, s, ev0, ev1);
}

}  // namespace

extern "C" {

int beagle_abi_version(void) { return BEAGLE_ABI_VERSION; }

const char* beagle_last_error(void) { return bgl::host::last_error(); }

beagle_status beagle_ctx_create(beagle_ctx** out, int device, size_t max_workspace_bytes) {
  if (!out) return fail(BEAGLE_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(BEAGLE_E_INVALID_ARG, "no such device");
  beagle_ctx* c = new beagle_ctx;
  c->device = device;
  c->cap = max_workspace_bytes;
  load_tune_file(c);
  *out = c;
  clear_error();
  return BEAGLE_OK;
}

static void release_events(beagle_ctx* ctx) {
  for (auto& pr : ctx->events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  ctx->events.clear();
}

beagle_status beagle_ctx_enable_timing(beagle_ctx* ctx, int enable) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  release_events(ctx);
  ctx->timing = enable != 0;
  return BEAGLE_OK;
}

beagle_status beagle_ctx_kernel_time(beagle_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return fail(BEAGLE_E_INVALID_ARG, "NULL argument");
  DeviceGuard g(ctx->device);
  double total = 0.0;
  for (auto& pr : ctx->events) {
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    total += ms;
  }
  *total_ms = total;
  *launches = int64_t(ctx->events.size());
  return BEAGLE_OK;
}

void beagle_ctx_destroy(beagle_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    release_events(ctx);
    release_graphs(ctx);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
    if (ctx->side_join) (void)hipEventDestroy(ctx->side_join);
    if (ctx->table_copied) (void)hipEventDestroy(ctx->table_copied);
    if (ctx->ws) (void)hipFree(ctx->ws);
  }
  delete ctx;
}

beagle_status beagle_ctx_tile_width(beagle_ctx* ctx, int kind, int32_t D, int64_t M, int64_t n_tokens,
                                    int32_t n_programs, int32_t* cases_per_lane) {
  if (!ctx || !cases_per_lane) return fail(BEAGLE_E_INVALID_ARG, "NULL argument");
  if (kind != BEAGLE_FIT_MSE && kind != BEAGLE_FIT_CORR) return fail(BEAGLE_E_INVALID_ARG, "unknown fitness kind");
  if (D < 1 || D > BEAGLE_MAX_D || M < 1 || n_programs < 1 || n_tokens < 0)
    return fail(BEAGLE_E_INVALID_ARG, "bad problem shape");
  int kv = 0;
  *cases_per_lane =
      known_tile_variant(ctx, kind, D, M, double(n_tokens) / n_programs, &kv) ? bgl::class_k(0, kv) : 0;
  return BEAGLE_OK;
}

beagle_status beagle_ctx_set_decoder(beagle_ctx* ctx, int decoder) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  if (decoder != BEAGLE_DECODE_WAVE && decoder != BEAGLE_DECODE_THREAD)
    return fail(BEAGLE_E_INVALID_ARG, "unknown decoder");
  ctx->decoder = decoder;
  return BEAGLE_OK;
}

beagle_status beagle_ctx_set_tuning(beagle_ctx* ctx, int policy) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  if (policy != BEAGLE_TUNE_AUTO && policy != BEAGLE_TUNE_WIDE && policy != BEAGLE_TUNE_NARROW)
    return fail(BEAGLE_E_INVALID_ARG, "unknown tuning policy");
  ctx->tuning = policy;
  return BEAGLE_OK;
}

}  // extern "C"

namespace {

// Layout of a whole-population evaluation within `cap` bytes of workspace
// (0: unlimited): the largest program slice whose partials fit.
EvalLayout capped_layout(const beagle_programs* progs, const beagle_dataset* data, int kind, size_t cap,
                         int32_t* slice_out) {
  const int n_sums = bgl::kind_sums(kind);
  int32_t slice = progs->n_programs;
  EvalLayout L = eval_layout(progs, data, n_sums, slice);
  while (cap && L.total > cap && slice > 1) {
    slice = (slice + 1) / 2;
    L = eval_layout(progs, data, n_sums, slice);
  }
  *slice_out = slice;
  return L;
}

// The launches of one whole-population evaluation of any fitness kind
// (smax: the maximum score of the paper's scores) in workspace ws, laid out
// by L with `slice` programs per interpreter launch.  With a context, the
// tile width comes from its tuner and its timing events bracket each
// interpreter launch; without one, 4 cases per lane (the width changes no
// result bit) and nothing is created.
beagle_status evaluate_in(char* ws, const EvalLayout& L, int32_t slice, beagle_ctx* ctx,
                          const beagle_programs* progs, const beagle_dataset* data, int kind, double smax,
                          double* fitness, int8_t* status, hipStream_t s) {
  const bool with_stats = kind == BEAGLE_FIT_CORR || kind == BEAGLE_FIT_R4;
  hipEvent_t join = nullptr;
  beagle_status st = BEAGLE_OK;
  if (with_stats && (st = launch_target_stats(ctx, data, reinterpret_cast<double*>(ws + L.stats), s, &join)) !=
                        BEAGLE_OK)
    return st;
  st = prepare(ws, progs, data, L, status, s, ctx ? ctx->decoder : BEAGLE_DECODE_WAVE);
  if (st != BEAGLE_OK) return st;
  bool shift_in_kernel = false;
  if (with_stats) {
    // the shifts need only the decoded programs and the staged cases; the
    // interpreter launches that follow read the statistics
    st = launch_shifts(ws, progs, data, L, s, &shift_in_kernel);
    if (st != BEAGLE_OK) return st;
    if ((st = join_target_stats(join, s)) != BEAGLE_OK) return st;
  }
  auto slice_args = [&](int32_t p0, int32_t np) {
    bgl::EvalArgs ea;
    ea.code = reinterpret_cast<const uint32_t*>(ws + L.code);
    ea.cval = reinterpret_cast<const float*>(ws + L.cval);
    ea.tok_offset = progs->tok_offset + p0;
    ea.meta = reinterpret_cast<const bgl::ProgMeta*>(ws + L.meta) + p0;
    ea.Xt = reinterpret_cast<const float*>(ws + L.Xt);
    ea.yp = reinterpret_cast<const float*>(ws + L.yp);
    ea.M = data->M;
    ea.Mp = L.Mp;
    ea.D = data->D;
    ea.n_programs = np;
    ea.n_chunks = L.n_chunks;
    ea.chunk = L.chunk;
    ea.part = reinterpret_cast<double*>(ws + L.part);
    ea.stats = reinterpret_cast<const double*>(ws + L.stats);
    ea.class_count = reinterpret_cast<const int32_t*>(ws + L.class_count);
    ea.class_list = reinterpret_cast<const int32_t*>(ws + L.class_list);
    ea.work = reinterpret_cast<unsigned long long*>(ws + L.work);
    ea.n_total = progs->n_programs;
    ea.prog_begin = p0;
    ea.smax = smax;
    ea.meta_shift = shift_in_kernel ? reinterpret_cast<bgl::ProgMeta*>(ws + L.meta) + p0 : nullptr;
    return ea;
  };
  int kv = 1;
  // the work counters are clear for the first launch unless the tuner's
  // timed runs used them
  bool counters_clear = true;
  if (ctx) {
    counters_clear = known_tile_variant(ctx, kind, data->D, data->M,
                                        double(progs->n_tokens) / progs->n_programs, &kv);
    TuneSlice ts{kind, slice_args(0, std::min(slice, progs->n_programs))};
    st = tile_variant(ctx, kind, data->D, data->M, double(progs->n_tokens) / progs->n_programs, s, run_slice, &ts,
                      &kv);
    if (st != BEAGLE_OK) return st;
  }
  for (int32_t p0 = 0; p0 < progs->n_programs; p0 += slice) {
    const int32_t np = std::min(slice, progs->n_programs - p0);
    const bgl::EvalArgs ea = slice_args(p0, np);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx && ctx->timing) {
      if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
        return fail(BEAGLE_E_HIP, "hipEventCreate");
      ctx->events.emplace_back(ev0, ev1);
    }
    hipError_t e = bgl::launch_eval(kind, kv, ea, s, ev0, ev1, counters_clear && p0 == 0);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    bgl::FinalizeArgs fa;
    fa.meta = ea.meta;
    fa.part = ea.part;
    fa.stats = ea.stats;
    fa.M = data->M;
    fa.n_programs = np;
    fa.n_chunks = L.n_chunks;
    fa.kind = kind;
    fa.fitness = fitness + p0;
    fa.coef = nullptr;
    fa.smax = smax;
    hipLaunchKernelGGL(bgl::k_finalize, dim3((np + 255) / 256), dim3(256), 0, s, fa);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
  }
  return BEAGLE_OK;
}

// Whole-population evaluation in a context's workspace.
beagle_status evaluate(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data, int kind,
                       double smax, double* fitness, int8_t* status, beagle_stream stream) {
  beagle_status st = check_programs(progs);
  if (st != BEAGLE_OK) return st;
  st = check_data(data, kind);
  if (st != BEAGLE_OK) return st;
  if (progs->n_programs == 0) return BEAGLE_OK;
  if (!fitness) return fail(BEAGLE_E_INVALID_ARG, "fitness is NULL");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t slice = 0;
  const EvalLayout L = capped_layout(progs, data, kind, ctx->cap, &slice);
  st = reserve(ctx, L.total);
  if (st != BEAGLE_OK) return st;
  st = evaluate_in(ctx->ws, L, slice, ctx, progs, data, kind, smax, fitness, status, s);
  if (st != BEAGLE_OK) return st;
  clear_error();
  return BEAGLE_OK;
}

// Workspace of beagle_eval_static: one array per device, in the library's
// code object, never allocated or freed by a call.  In host code `scratch`
// names a host-side stand-in; its device address on each device comes from
// hipGetSymbolAddress with that device current (scratch_on).
static __device__ __align__(256) char scratch[BEAGLE_STATIC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char* g_scratch[MAX_DEVICES] = {};

beagle_status scratch_on(int dev, char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(BEAGLE_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch[dev];
  return BEAGLE_OK;
}

}  // namespace

extern "C" {

beagle_status beagle_eval_static(const beagle_programs* progs, const beagle_dataset* data, int kind, double* fitness,
                                 int8_t* status, beagle_stream stream) {
  if (kind != BEAGLE_FIT_MSE && kind != BEAGLE_FIT_CORR)
    return fail(BEAGLE_E_INVALID_ARG, "unknown fitness kind (MSE or CORR)");
  beagle_status st = check_programs(progs);
  if (st != BEAGLE_OK) return st;
  st = check_data(data, kind);
  if (st != BEAGLE_OK) return st;
  if (progs->n_programs == 0) return BEAGLE_OK;
  if (!fitness) return fail(BEAGLE_E_INVALID_ARG, "fitness is NULL");
  int32_t slice = 0;
  const EvalLayout L = capped_layout(progs, data, kind, BEAGLE_STATIC_SCRATCH_BYTES, &slice);
  if (L.total > BEAGLE_STATIC_SCRATCH_BYTES)
    return fail(BEAGLE_E_NOMEM, "beagle_eval_static: the evaluation needs " + std::to_string(L.total) +
                                    " bytes of scratch, the static array holds " +
                                    std::to_string(size_t(BEAGLE_STATIC_SCRATCH_BYTES)));
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  char* ws = nullptr;
  st = scratch_on(dev, &ws);
  if (st != BEAGLE_OK) return st;
  st = evaluate_in(ws, L, slice, nullptr, progs, data, kind, 0.0, fitness, status,
                   reinterpret_cast<hipStream_t>(stream));
  if (st != BEAGLE_OK) return st;
  clear_error();
  return BEAGLE_OK;
}

}  // extern "C"

extern "C" {

beagle_status beagle_eval(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data, int kind,
                          double* fitness, int8_t* status, beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  if (kind != BEAGLE_FIT_MSE && kind != BEAGLE_FIT_CORR)
    return fail(BEAGLE_E_INVALID_ARG, "unknown fitness kind (the paper's scores: beagle_eval_score)");
  return evaluate(ctx, progs, data, kind, 0.0, fitness, status, stream);
}

beagle_status beagle_eval_score(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data, int kind,
                                double max_score, double* score, int8_t* status, beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  if (kind != BEAGLE_FIT_POINT && kind != BEAGLE_FIT_R4)
    return fail(BEAGLE_E_INVALID_ARG, "beagle_eval_score takes BEAGLE_FIT_POINT or BEAGLE_FIT_R4");
  if (!(max_score > 0.0) || !std::isfinite(max_score))
    return fail(BEAGLE_E_INVALID_ARG, "max_score must be finite and > 0");
  return evaluate(ctx, progs, data, kind, max_score, score, status, stream);
}

beagle_status beagle_eval_workspace_size(const beagle_programs* progs, const beagle_dataset* data, int kind,
                                         size_t* bytes) {
  if (!bytes) return fail(BEAGLE_E_INVALID_ARG, "bytes is NULL");
  if (kind < BEAGLE_FIT_MSE || kind > BEAGLE_FIT_R4) return fail(BEAGLE_E_INVALID_ARG, "unknown fitness kind");
  beagle_status st = check_programs(progs);
  if (st != BEAGLE_OK) return st;
  st = check_data(data, kind);
  if (st != BEAGLE_OK) return st;
  *bytes = eval_layout(progs, data, bgl::kind_sums(kind), std::max(progs->n_programs, 1)).total;
  return BEAGLE_OK;
}

beagle_status beagle_predict(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                             float* yhat, int8_t* status, beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  beagle_status st = check_programs(progs);
  if (st != BEAGLE_OK) return st;
  st = check_data(data, BEAGLE_FIT_MSE);
  if (st != BEAGLE_OK) return st;
  if (progs->n_programs == 0) return BEAGLE_OK;
  if (!yhat) return fail(BEAGLE_E_INVALID_ARG, "yhat is NULL");
  if (int64_t(progs->n_programs) * data->M > (int64_t(1) << 31))
    return fail(BEAGLE_E_UNSUPPORTED, "predict: n_programs * M > 2^31");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  EvalLayout L = eval_layout(progs, data, 1, 1);
  st = reserve(ctx, L.total);
  if (st != BEAGLE_OK) return st;
  st = prepare(ctx->ws, progs, data, L, status, s, ctx->decoder);
  if (st != BEAGLE_OK) return st;
  st = launch_values(ctx->ws, progs, data, L, data->M, yhat, 0, s);
  if (st != BEAGLE_OK) return st;
  clear_error();
  return BEAGLE_OK;
}

static beagle_status check_gen_params(const beagle_gen_params* p, int32_t D) {
  if (!p) return fail(BEAGLE_E_INVALID_ARG, "params is NULL");
  if (D < 1 || D > BEAGLE_MAX_D) return fail(BEAGLE_E_UNSUPPORTED, "D must be in [1, 16]");
  if (p->tournament < 1 || p->tournament > 64) return fail(BEAGLE_E_INVALID_ARG, "tournament must be in [1, 64]");
  if (!(p->p_crossover >= 0.0f && p->p_mutation >= 0.0f && p->p_crossover + p->p_mutation <= 1.0f + 1e-6f))
    return fail(BEAGLE_E_INVALID_ARG, "operator probabilities must be >= 0 and sum to <= 1");
  if (p->max_len < 1 || p->max_len > BEAGLE_MAX_LEN) return fail(BEAGLE_E_UNSUPPORTED, "max_len must be in [1, 4096]");
  if (p->max_consts < 0 || p->max_consts > 255) return fail(BEAGLE_E_UNSUPPORTED, "max_consts must be in [0, 255]");
  if (!(p->const_lo <= p->const_hi)) return fail(BEAGLE_E_INVALID_ARG, "const_lo > const_hi");
  if (p->op_set != 0 && p->op_set != 1) return fail(BEAGLE_E_INVALID_ARG, "op_set must be 0 or 1");
  return BEAGLE_OK;
}

// unary operators of an operator set (see beagle_gen_params::op_set)
static int32_t n_unary_of(const beagle_gen_params* p) { return p->op_set == 1 ? 12 : 5; }

beagle_status beagle_init_population(beagle_ctx* ctx, const beagle_gen_params* params, int32_t n, int32_t D,
                                     uint64_t seed, uint32_t problem, uint16_t* tokens, int32_t* len,
                                     float* consts, int32_t* const_count, beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  beagle_status st = check_gen_params(params, D);
  if (st != BEAGLE_OK) return st;
  if (n < 0) return fail(BEAGLE_E_INVALID_ARG, "n < 0");
  if (params->init_depth_min < 0 || params->init_depth_max < params->init_depth_min ||
      params->init_depth_max > bgl::MAX_INIT_DEPTH)
    return fail(BEAGLE_E_INVALID_ARG, "init depths must satisfy 0 <= min <= max <= 11");
  if ((int64_t(1) << (params->init_depth_max + 1)) - 1 > params->max_len)
    return fail(BEAGLE_E_INVALID_ARG, "2^(init_depth_max+1) - 1 exceeds max_len");
  if (problem & 0x80000000u) return fail(BEAGLE_E_INVALID_ARG, "problem id must be < 2^31");
  if (n == 0) return BEAGLE_OK;
  if (!tokens || !len || !const_count || (params->max_consts > 0 && !consts))
    return fail(BEAGLE_E_INVALID_ARG, "an output pointer is NULL");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  bgl::InitArgs a;
  a.n = n;
  a.D = D;
  a.depth_min = params->init_depth_min;
  a.depth_max = params->init_depth_max;
  a.max_len = params->max_len;
  a.max_consts = params->max_consts;
  a.const_lo = params->const_lo;
  a.const_hi = params->const_hi;
  a.n_unary = n_unary_of(params);
  a.seed = seed;
  a.tag = 0x80000000u | problem;
  a.tokens = tokens;
  a.len = len;
  a.consts = consts;
  a.const_count = const_count;
  hipLaunchKernelGGL(bgl::k_init_population, dim3((n + 63) / 64), dim3(64), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "init launch");
  clear_error();
  return BEAGLE_OK;
}

beagle_status beagle_generation(beagle_ctx* ctx, const beagle_programs* parents, const double* fitness,
                                const beagle_gen_params* params, int32_t D, uint64_t seed, uint64_t generation,
                                uint32_t problem, uint16_t* child_tokens, int32_t* child_len,
                                float* child_consts, int32_t* child_const_count, beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  beagle_status st = check_programs(parents);
  if (st != BEAGLE_OK) return st;
  st = check_gen_params(params, D);
  if (st != BEAGLE_OK) return st;
  if (problem & 0x80000000u) return fail(BEAGLE_E_INVALID_ARG, "problem id must be < 2^31");
  const int32_t n = parents->n_programs;
  if (n == 0) return BEAGLE_OK;
  if (!fitness) return fail(BEAGLE_E_INVALID_ARG, "fitness is NULL");
  if (!child_tokens || !child_len || !child_const_count || (params->max_consts > 0 && !child_consts))
    return fail(BEAGLE_E_INVALID_ARG, "an output pointer is NULL");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  bgl::GenStepArgs a;
  a.tokens = parents->tokens;
  a.n_tokens = parents->n_tokens;
  a.tok_offset = parents->tok_offset;
  a.tok_len = parents->tok_len;
  a.consts = parents->consts;
  a.n_consts = parents->n_consts;
  a.const_offset = parents->const_offset;
  a.const_count = parents->const_count;
  a.fitness = fitness;
  a.n = n;
  a.n_parents = n;
  a.surv = nullptr;
  a.n_surv = nullptr;
  a.D = D;
  a.tournament = params->tournament;
  // operator thresholds in binary32: p_crossover and p_crossover + p_mutation
  const float pc = params->p_crossover;
  volatile float sum = pc + params->p_mutation;
  a.t_cross = pc;
  a.t_mut = sum;
  a.max_len = params->max_len;
  a.max_consts = params->max_consts;
  a.const_lo = params->const_lo;
  a.const_hi = params->const_hi;
  a.n_unary = n_unary_of(params);
  a.seed = seed;
  a.generation = uint32_t(generation);
  a.tag = problem;
  a.child_tokens = child_tokens;
  a.child_len = child_len;
  a.child_consts = child_consts;
  a.child_const_count = child_const_count;
  a.slots = nullptr;
  hipLaunchKernelGGL(bgl::k_generation, dim3((n + 63) / 64), dim3(64), 0, reinterpret_cast<hipStream_t>(stream),
                     a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "generation launch");
  clear_error();
  return BEAGLE_OK;
}

beagle_status beagle_generation_microcosm(beagle_ctx* ctx, const beagle_programs* parents, const double* fitness,
                                          const beagle_gen_params* params, int32_t D, int32_t sample, float keep,
                                          uint64_t seed, uint64_t generation, uint32_t problem, int32_t n_children,
                                          uint16_t* child_tokens, int32_t* child_len, float* child_consts,
                                          int32_t* child_const_count, double* threshold, int32_t* n_survivors,
                                          beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  beagle_status st = check_programs(parents);
  if (st != BEAGLE_OK) return st;
  st = check_gen_params(params, D);
  if (st != BEAGLE_OK) return st;
  if (problem & 0xC0000000u) return fail(BEAGLE_E_INVALID_ARG, "problem id must be < 2^30");
  if (sample < 1 || sample > bgl::MICRO_MAX_SAMPLE)
    return fail(BEAGLE_E_INVALID_ARG, "sample must be in 1.." + std::to_string(bgl::MICRO_MAX_SAMPLE));
  if (!(keep > 0.0f && keep <= 1.0f)) return fail(BEAGLE_E_INVALID_ARG, "keep must be in (0, 1]");
  if (n_children < 0) return fail(BEAGLE_E_INVALID_ARG, "n_children < 0");
  const int32_t n = parents->n_programs;
  if (n == 0 && n_children > 0) return fail(BEAGLE_E_INVALID_ARG, "children need at least one parent");
  if (n == 0) return BEAGLE_OK;
  if (!fitness) return fail(BEAGLE_E_INVALID_ARG, "fitness is NULL");
  if (n_children > 0 && (!child_tokens || !child_len || !child_const_count || (params->max_consts > 0 && !child_consts)))
    return fail(BEAGLE_E_INVALID_ARG, "an output pointer is NULL");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const int32_t n_blocks = int32_t((int64_t(n) + bgl::MICRO_BLOCK - 1) / bgl::MICRO_BLOCK);
  Carve cv;
  const size_t o_tau = cv.take<double>(1);
  const size_t o_ns = cv.take<int32_t>(1);
  const size_t o_off = cv.take<int32_t>(size_t(n_blocks));
  const size_t o_surv = cv.take<int32_t>(size_t(n));
  const size_t o_slots = cv.take<int64_t>(5);
  st = reserve(ctx, cv.used);
  if (st != BEAGLE_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bgl::MicroArgs m;
  m.fitness = fitness;
  m.n = n;
  m.sample = sample;
  // threshold position ceil(keep * sample) - 1 in the sorted sample (the
  // product in binary64, clamped to the sample)
  const double kq = std::ceil(double(keep) * double(sample)) - 1.0;
  m.k = int32_t(std::min(double(sample - 1), std::max(0.0, kq)));
  m.seed = seed;
  m.generation = uint32_t(generation);
  m.tag = bgl::MICRO_TAG | problem;
  m.n_blocks = n_blocks;
  m.tau = threshold ? threshold : reinterpret_cast<double*>(ctx->ws + o_tau);
  m.n_surv = n_survivors ? n_survivors : reinterpret_cast<int32_t*>(ctx->ws + o_ns);
  m.block_off = reinterpret_cast<int32_t*>(ctx->ws + o_off);
  m.surv = reinterpret_cast<int32_t*>(ctx->ws + o_surv);
  m.tok_offset = parents->tok_offset;
  m.const_offset = parents->const_offset;
  m.slots = reinterpret_cast<int64_t*>(ctx->ws + o_slots);
  hipLaunchKernelGGL(bgl::k_micro_threshold, dim3(1), dim3(bgl::MICRO_MAX_SAMPLE), 0, s, m);
  hipLaunchKernelGGL(bgl::k_micro_count, dim3(n_blocks), dim3(bgl::MICRO_BLOCK), 0, s, m);
  hipLaunchKernelGGL(bgl::k_micro_scan, dim3(1), dim3(1024), 0, s, m);
  hipLaunchKernelGGL(bgl::k_micro_scatter, dim3(n_blocks), dim3(bgl::MICRO_BLOCK), 0, s, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "microcosm selection launch");
  if (n_children > 0) {
    bgl::GenStepArgs a;
    a.tokens = parents->tokens;
    a.n_tokens = parents->n_tokens;
    a.tok_offset = parents->tok_offset;
    a.tok_len = parents->tok_len;
    a.consts = parents->consts;
    a.n_consts = parents->n_consts;
    a.const_offset = parents->const_offset;
    a.const_count = parents->const_count;
    a.fitness = fitness;
    a.n = n_children;
    a.n_parents = n;
    a.surv = m.surv;
    a.n_surv = m.n_surv;
    a.D = D;
    a.tournament = params->tournament;
    const float pc = params->p_crossover;
    volatile float sum = pc + params->p_mutation;
    a.t_cross = pc;
    a.t_mut = sum;
    a.max_len = params->max_len;
    a.max_consts = params->max_consts;
    a.const_lo = params->const_lo;
    a.const_hi = params->const_hi;
    a.n_unary = n_unary_of(params);
    a.seed = seed;
    a.generation = uint32_t(generation);
    a.tag = problem;
    a.child_tokens = child_tokens;
    a.child_len = child_len;
    a.child_consts = child_consts;
    a.child_const_count = child_const_count;
    a.slots = m.slots;
    hipLaunchKernelGGL(bgl::k_generation, dim3((n_children + 63) / 64), dim3(64), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "generation launch");
  }
  clear_error();
  return BEAGLE_OK;
}

}  // extern "C"

namespace {

// The correlation evaluation of the whole population (target statistics,
// shifts, interpreter, finalize) writing the fitness and the seed
// coefficients of the correlation adjoint.
// The target statistics were launched before the decoding; s waits for
// them through `join`.
beagle_status corr_pass(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                        const EvalLayout& L, double* fitness, hipEvent_t join, hipStream_t s) {
  char* ws = ctx->ws;
  bool shift_in_kernel = false;
  beagle_status st = launch_shifts(ws, progs, data, L, s, &shift_in_kernel);
  if (st != BEAGLE_OK) return st;
  if ((st = join_target_stats(join, s)) != BEAGLE_OK) return st;
  bgl::EvalArgs ea;
  ea.code = reinterpret_cast<const uint32_t*>(ws + L.code);
  ea.cval = reinterpret_cast<const float*>(ws + L.cval);
  ea.tok_offset = progs->tok_offset;
  ea.meta = reinterpret_cast<const bgl::ProgMeta*>(ws + L.meta);
  ea.Xt = reinterpret_cast<const float*>(ws + L.Xt);
  ea.yp = reinterpret_cast<const float*>(ws + L.yp);
  ea.M = data->M;
  ea.Mp = L.Mp;
  ea.D = data->D;
  ea.n_programs = progs->n_programs;
  ea.n_chunks = L.n_chunks;
  ea.chunk = L.chunk;
  ea.part = reinterpret_cast<double*>(ws + L.part);
  ea.stats = reinterpret_cast<const double*>(ws + L.stats);
  ea.class_count = reinterpret_cast<const int32_t*>(ws + L.class_count);
  ea.class_list = reinterpret_cast<const int32_t*>(ws + L.class_list);
  ea.work = reinterpret_cast<unsigned long long*>(ws + L.work);
  ea.n_total = progs->n_programs;
  ea.prog_begin = 0;
  ea.meta_shift = shift_in_kernel ? reinterpret_cast<bgl::ProgMeta*>(ws + L.meta) : nullptr;
  int kv = 0;
  TuneSlice ts{BEAGLE_FIT_CORR, ea};
  st = tile_variant(ctx, BEAGLE_FIT_CORR, data->D, data->M, double(progs->n_tokens) / progs->n_programs, s,
                    run_slice, &ts, &kv);
  if (st != BEAGLE_OK) return st;
  hipError_t e = bgl::launch_eval(BEAGLE_FIT_CORR, kv, ea, s, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(e, "eval launch");
  bgl::FinalizeArgs fa;
  fa.meta = ea.meta;
  fa.part = ea.part;
  fa.stats = ea.stats;
  fa.M = data->M;
  fa.n_programs = progs->n_programs;
  fa.n_chunks = L.n_chunks;
  fa.kind = BEAGLE_FIT_CORR;
  fa.fitness = fitness;
  fa.coef = reinterpret_cast<double*>(ws + L.coef);
  hipLaunchKernelGGL(bgl::k_finalize, dim3((progs->n_programs + 255) / 256), dim3(256), 0, s, fa);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "finalize launch");
  return BEAGLE_OK;
}

}  // namespace

extern "C" {

beagle_status beagle_eval_grad(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                               int kind, double* fitness, float* grad_consts, int8_t* status,
                               beagle_stream stream) {
  if (!ctx) return fail(BEAGLE_E_INVALID_ARG, "ctx is NULL");
  if (kind != BEAGLE_FIT_MSE && kind != BEAGLE_FIT_CORR) return fail(BEAGLE_E_INVALID_ARG, "unknown fitness kind");
  beagle_status st = check_programs(progs);
  if (st != BEAGLE_OK) return st;
  st = check_data(data, kind);
  if (st != BEAGLE_OK) return st;
  if (progs->n_programs == 0) return BEAGLE_OK;
  if (!fitness) return fail(BEAGLE_E_INVALID_ARG, "fitness is NULL");
  if (progs->n_consts > 0 && !grad_consts) return fail(BEAGLE_E_INVALID_ARG, "grad_consts is NULL");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool corr = kind == BEAGLE_FIT_CORR;
  EvalLayout L = eval_layout(progs, data, corr ? 3 : 1, progs->n_programs, true);
  st = reserve(ctx, L.total);
  if (st != BEAGLE_OK) return st;
  hipEvent_t join = nullptr;
  if (corr && (st = launch_target_stats(ctx, data, reinterpret_cast<double*>(ctx->ws + L.stats), s, &join)) !=
                  BEAGLE_OK)
    return st;
  st = prepare(ctx->ws, progs, data, L, status, s, ctx->decoder, bgl::GRAD_LONG_WORDS, true);
  if (st != BEAGLE_OK) return st;
  char* ws = ctx->ws;
  if (corr) {
    // first pass: the correlation fitness and every program's seed
    // coefficients, by the evaluator (its own chunking)
    st = corr_pass(ctx, progs, data, L, fitness, join, s);
    if (st != BEAGLE_OK) return st;
  }
  unsigned long long* work = reinterpret_cast<unsigned long long*>(ws + L.work);
  zero_i32(reinterpret_cast<int32_t*>(work), 2 * 8, s);
  bgl::GradArgs ga;
  ga.code = reinterpret_cast<const uint32_t*>(ws + L.code);
  ga.aux = reinterpret_cast<const uint32_t*>(ws + L.aux);
  ga.cval = reinterpret_cast<const float*>(ws + L.cval);
  ga.tok_offset = progs->tok_offset;
  ga.meta = reinterpret_cast<const bgl::ProgMeta*>(ws + L.meta);
  ga.const_offset = progs->const_offset;
  ga.const_count = progs->const_count;
  ga.Xt = reinterpret_cast<const float*>(ws + L.Xt);
  ga.yp = reinterpret_cast<const float*>(ws + L.yp);
  ga.M = data->M;
  ga.Mp = L.Mp;
  ga.D = data->D;
  ga.n_programs = progs->n_programs;
  ga.n_chunks = L.gn_chunks;
  ga.chunk = L.gchunk;
  ga.part = reinterpret_cast<double*>(ws + L.part);
  ga.gpart = reinterpret_cast<double*>(ws + L.gpart);
  ga.n_consts = progs->n_consts;
  ga.kind = kind;
  ga.coef = reinterpret_cast<const double*>(ws + L.coef);
  ga.stats = reinterpret_cast<const double*>(ws + L.stats);
  ga.list_count = reinterpret_cast<const int32_t*>(ws + L.class_count) + 8;
  ga.list = reinterpret_cast<const int32_t*>(ws + L.len_list);
  ga.work = work;
  hipError_t e = bgl::launch_grad(ga, s);
  if (e != hipSuccess) return hip_fail(e, "gradient launch");
  bgl::GradFinalizeArgs fa;
  fa.meta = ga.meta;
  fa.part = ga.part;
  fa.gpart = ga.gpart;
  fa.const_offset = progs->const_offset;
  fa.const_count = progs->const_count;
  fa.M = data->M;
  fa.n_consts = progs->n_consts;
  fa.n_programs = progs->n_programs;
  fa.n_chunks = L.gn_chunks;
  fa.kind = kind;
  fa.fitness = fitness;
  fa.grad = grad_consts;
  hipLaunchKernelGGL(bgl::k_grad_finalize, dim3(progs->n_programs), dim3(64), 0, s, fa);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gradient finalize launch");
  clear_error();
  return BEAGLE_OK;
}

}  // extern "C"
