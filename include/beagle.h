/*
 * beagle.h -- C ABI of the MI355X population evaluator for genetic
 * programming symbolic regression (arXiv 2603.12292, "GPU-Accelerated
 * Genetic Programming for Symbolic Regression with Beagle Framework").
 *
 * The paper's GPU side runs every genome of the population on a batch of
 * fitness cases and returns one aggregate fitness per individual (section
 * 2.1.2); genomes are reverse-Polish programs (section 2.1.4); the fitness is
 * point-to-point or correlation based (section 2.1.5, Eq. 1).  This library
 * is that evaluation step, plus a reverse-mode gradient with respect to the
 * programs' constants and a generation step (selection and variation) that
 * keeps the population on the device.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array pointers are DEVICE pointers owned by the caller; the library
 *    never frees them and keeps no reference after the call returns.
 *  - Calls are asynchronous: they check their scalar arguments on the host,
 *    enqueue kernels on `stream` (a hipStream_t; NULL = the null stream) and
 *    return.  Argument errors are reported synchronously by the return code
 *    and beagle_last_error(); per-program problems (malformed programs) are
 *    reported asynchronously in the optional `status` array.
 *  - A context owns its device workspace, grown on demand (hipMalloc; the
 *    growth synchronises the device) and released by beagle_ctx_destroy.
 *    One context must not be used by two host threads at once.
 *  - Nothing here takes the device's scalar data cache for writing, and no
 *    result depends on the order in which workgroups run: every reduction
 *    has a fixed order, so repeated calls give bit-identical outputs.
 *
 * Token format (section 2.1.4: the genome is a reverse-Polish program)
 * --------------------------------------------------------------------
 *  One uint16 per token: opcode | (arg << 8).
 *    0 ADD  1 SUB  2 MUL  3 DIV  4 SIN  5 COS  6 EXP  7 LOG  8 SQRT
 *    9 VAR   (arg = input variable k < D)
 *   10 CONST (arg = slot j < const_count of the program)
 *  A binary operator pops b (top) then a and pushes a op b.  The arg of an
 *  operator token is ignored.  Operator conventions (the paper keeps invalid
 *  values rather than protecting operators; these protected forms are the
 *  library's):
 *    DIV  b == 0 ? 1 : a / b         EXP  exp(clamp(x, -80, 80)), NaN -> NaN
 *    LOG  x == 0 ? 0 : log|x|        SQRT sqrt|x|        SIN, COS: IEEE
 *  Evaluation is in binary32 per fitness case.
 */
#ifndef BEAGLE_H
#define BEAGLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BEAGLE_ABI_VERSION 2

typedef struct beagle_ctx beagle_ctx;
typedef void* beagle_stream; /* hipStream_t */

/* Return codes of every entry point. */
typedef enum {
  BEAGLE_OK = 0,
  BEAGLE_E_INVALID_ARG = -1, /* a scalar argument or a NULL pointer is wrong      */
  BEAGLE_E_HIP = -2,         /* a HIP runtime call or kernel launch failed         */
  BEAGLE_E_NOMEM = -3,       /* workspace allocation failed or exceeds the cap     */
  BEAGLE_E_UNSUPPORTED = -4  /* a size beyond the limits below                     */
} beagle_status;

/* Fitness kinds (section 2.1.5).  MSE = (1/M) sum (yhat - y)^2.  CORR =
 * 1 - r^2 with r Pearson's correlation (Eq. 1), its sums accumulated in
 * binary64 and clamped to [0, 1].  Classification: MSE follows IEEE
 * arithmetic of its case terms yhat - y: NaN if any is NaN (a NaN output or
 * target, or an infinite output meeting the same infinite target), else
 * +Inf if any is infinite; CORR is NaN if any yhat or y is not finite, 1 if
 * every yhat is equal, NaN if every y is equal.
 * POINT and R4 are the paper's own scores (higher is better; see
 * beagle_eval_score): POINT the sum over cases of Eq. 3, R4 Eq. 2. */
typedef enum {
  BEAGLE_FIT_MSE = 0,
  BEAGLE_FIT_CORR = 1,
  BEAGLE_FIT_POINT = 2,
  BEAGLE_FIT_R4 = 3
} beagle_fitness_kind;

/* Per-program status codes written to the optional status[] outputs.  A
 * program with a non-zero status gets fitness NaN.  Tokens are checked in
 * order; the first faulty token decides, checking opcode range, variable
 * index, constant slot, then stack underflow. */
enum {
  BEAGLE_PROG_OK = 0,
  BEAGLE_PROG_EMPTY = 1,           /* tok_len == 0                              */
  BEAGLE_PROG_BAD_OPCODE = 2,      /* opcode > 10                               */
  BEAGLE_PROG_UNDERFLOW = 3,       /* an operator finds too few operands        */
  BEAGLE_PROG_BAD_FINAL_DEPTH = 4, /* the program leaves != 1 value             */
  BEAGLE_PROG_BAD_VAR = 5,         /* VAR arg >= D                              */
  BEAGLE_PROG_BAD_CONST = 6,       /* CONST arg >= const_count                  */
  BEAGLE_PROG_TOO_LONG = 7,        /* tok_len > BEAGLE_MAX_LEN                  */
  BEAGLE_PROG_BAD_LAYOUT = 8       /* offsets/lengths outside the given arrays,
                                      or a range overlapping another program's */
};

#define BEAGLE_MAX_LEN 4096 /* tokens per program                               */
#define BEAGLE_MAX_D 16     /* input variables                                   */

/* A population in packed layout.  Program p is
 *   tokens[tok_offset[p] .. tok_offset[p] + tok_len[p])
 * and its constant table is
 *   consts[const_offset[p] .. const_offset[p] + const_count[p]).
 * n_tokens and n_consts are the lengths of tokens[] and consts[]; ranges
 * outside them give BEAGLE_PROG_BAD_LAYOUT.  Each program is decoded into
 * workspace at its own token offset, so the token ranges of different
 * programs must not overlap (for beagle_eval_grad, whose gradient has the
 * constants' layout, neither may the constant ranges): a program whose
 * range overlaps a lower-indexed program's gets BEAGLE_PROG_BAD_LAYOUT and
 * NaN, the others are unaffected.  Ranges may come in any order. */
typedef struct {
  const uint16_t* tokens;
  int64_t n_tokens;
  const int64_t* tok_offset; /* [n_programs] */
  const int32_t* tok_len;    /* [n_programs] */
  const float* consts;
  int64_t n_consts;
  const int64_t* const_offset; /* [n_programs] */
  const int32_t* const_count;  /* [n_programs] */
  int32_t n_programs;
} beagle_programs;

/* Fitness cases: X[M x D] row-major (case-major) binary32, y[M] binary32. */
typedef struct {
  const float* X;
  const float* y;
  int64_t M;
  int32_t D;
} beagle_dataset;

int beagle_abi_version(void);

/* Message describing the last failure on the calling host thread; "" if
 * none, and after a call that launched its work successfully. */
const char* beagle_last_error(void);

/* Create a context on HIP device `device`.  max_workspace_bytes caps the
 * workspace (0 = no cap); an evaluation that would need more is split into
 * several passes over slices of the population, with identical results. */
beagle_status beagle_ctx_create(beagle_ctx** out, int device, size_t max_workspace_bytes);
void beagle_ctx_destroy(beagle_ctx* ctx);

/* Kernel timing (instrumentation).  While enabled, every beagle_eval call
 * records a pair of HIP events on its stream around its main evaluation
 * kernel (the fast-path interpreter launch), and every beagle_eval_batched
 * call around its whole graph launch.  beagle_ctx_kernel_time waits
 * for the recorded events and returns the summed elapsed time and the
 * number of launches since timing was last enabled.  Enabling resets. */
beagle_status beagle_ctx_enable_timing(beagle_ctx* ctx, int enable);
beagle_status beagle_ctx_kernel_time(beagle_ctx* ctx, double* total_ms, int64_t* launches);

/* Whole-population evaluation (section 2.1.2: every program runs on every
 * fitness case and one aggregate fitness per program comes back).
 *   fitness  double[n_programs] out, device
 *   status   int8[n_programs] out, device, may be NULL
 * Needs M >= 1 (M >= 2 for CORR), 1 <= D <= BEAGLE_MAX_D. */
beagle_status beagle_eval(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                          int kind, double* fitness, int8_t* status, beagle_stream stream);

/* The paper's scores (section 2.1.5), which pair invalid values (NaN, +Inf,
 * -Inf) of the output and of the target instead of discarding them; higher
 * is better.  S = max_score (finite, > 0).
 *   BEAGLE_FIT_POINT  sum over cases of Eq. 3: both valid: S if both are 0,
 *                     else round(S min/max - [yhat y < 0] S/11) with
 *                     min/max of |yhat|, |y| in binary64, S/11 real-valued
 *                     and round() half to even; both invalid: S; one
 *                     invalid: -S
 *   BEAGLE_FIT_R4     Eq. 2: S r^4 (M - c1 - c2) - S (c1 - c2), c1 the cases
 *                     with exactly one invalid value, c2 those with two, r
 *                     Pearson's r (Eq. 1) over the cases where both are
 *                     valid (0 with fewer than two such cases or zero
 *                     variance), its sums in binary64
 *   score   double[n_programs] out, device (NaN for an invalid program)
 *   status  int8[n_programs] out, device, may be NULL
 * y may hold invalid values.  Needs M >= 1, 1 <= D <= BEAGLE_MAX_D. */
beagle_status beagle_eval_score(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                                int kind, double max_score, double* score, int8_t* status, beagle_stream stream);

/* Workspace bytes beagle_eval (beagle_eval_score for its kinds) needs for
 * this population and dataset in one pass (before any capping); only the
 * sizes in `progs` and `data` are read. */
beagle_status beagle_eval_workspace_size(const beagle_programs* progs, const beagle_dataset* data, int kind,
                                         size_t* bytes);

/* beagle_eval without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results (bit for bit) as
 * beagle_eval, on the calling thread's current device, with every piece of
 * workspace taken from one static device array of
 * BEAGLE_STATIC_SCRATCH_BYTES per device, part of the library's code object
 * (each device the library runs on holds it until the process ends).  The
 * call allocates and frees nothing, creates no events and does not tune:
 * 4 cases per lane (beagle_eval's tile width changes no result bit).  The
 * caller owns progs, data, fitness and status as for beagle_eval.
 *   kind    BEAGLE_FIT_MSE or BEAGLE_FIT_CORR
 * A population whose workspace exceeds the array is evaluated in program
 * slices (as under a context's workspace cap, identical results); when even
 * one program's share does not fit, BEAGLE_E_NOMEM and nothing is launched.
 * Every call on a device shares that device's array and leaves its
 * contents behind: calls that overlap in time on one device (two streams,
 * two threads) race and give undefined results; calls on one stream are
 * ordered and safe. */
#define BEAGLE_STATIC_SCRATCH_BYTES (32u << 20)
beagle_status beagle_eval_static(const beagle_programs* progs, const beagle_dataset* data, int kind,
                                 double* fitness, int8_t* status, beagle_stream stream);

/* Per-case outputs yhat[p * M + i] (binary32) of every program -- the
 * model outputs each fitness of section 2.1.5 compares with the targets,
 * from the same interpreter code: a debugging and testing aid for small
 * populations (n_programs * M <= 2^31).  Invalid programs give NaN rows. */
beagle_status beagle_predict(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                             float* yhat, int8_t* status, beagle_stream stream);

/* Fitness and its gradient with respect to every program's constants (not
 * in the paper: reverse-mode differentiation over the postfix tape so a
 * program's ephemeral constants can be tuned by gradient steps).
 *   kind         BEAGLE_FIT_MSE, or BEAGLE_FIT_CORR: the gradient of
 *                1 - r^2 (r of Eq. 1), unclamped where the fitness is
 *                clamped to [0, 1], zero for a constant output (fitness 1),
 *                NaN for a NaN fitness; the fitness is the one beagle_eval
 *                gives (same kernels)
 *   fitness      double[n_programs] out, device
 *   grad_consts  float[n_consts] out, device, same layout as consts; slots
 *                outside every program's range are left untouched
 *   status       int8[n_programs] out, device, may be NULL
 * Derivatives are taken as 0 where a protected branch replaces the
 * operator by a constant (DIV by 0, EXP outside [-80, 80], LOG of 0, SQRT of
 * 0).  Programs of more than 256 decoded words get status TOO_LONG. */
beagle_status beagle_eval_grad(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                               int kind, double* fitness, float* grad_consts, int8_t* status,
                               beagle_stream stream);

/* Decoders of the programs of at most 64 tokens (beagle_ctx_set_decoder). */
typedef enum { BEAGLE_DECODE_WAVE = 0, BEAGLE_DECODE_THREAD = 1 } beagle_decoder;

/* Which kernel validates and decodes (section 2.1.4's reverse-Polish
 * genomes into the interpreter's words) the programs of at most 64 tokens
 * in every later call of this context: BEAGLE_DECODE_WAVE (the default),
 * one wave per program with a token per lane, or BEAGLE_DECODE_THREAD, one
 * thread per program.  Both give the same statuses and bit-identical
 * results; the choice exists for testing and comparison.  Longer programs
 * always take the thread decoder.  Unknown decoder: BEAGLE_E_INVALID_ARG. */
beagle_status beagle_ctx_set_decoder(beagle_ctx* ctx, int decoder);

/* Tile-width policies of the evaluator (beagle_ctx_set_tuning). */
typedef enum { BEAGLE_TUNE_AUTO = 0, BEAGLE_TUNE_WIDE = 1, BEAGLE_TUNE_NARROW = 2 } beagle_tuning;

/* How many fitness cases each lane carries through the interpreter for the
 * common programs (stack of at most 4 values): 8 (BEAGLE_TUNE_WIDE, used
 * only where D <= 8) or 4 (BEAGLE_TUNE_NARROW).  BEAGLE_TUNE_AUTO, the
 * default, times both the first time an evaluation meets a problem-shape
 * bucket (fitness kind, D, log2 M, log2 of the mean program length) -- that
 * call synchronises the device -- and keeps the faster in the context.  When
 * the environment variable BEAGLE_AUTOTUNE_CACHE names a file, buckets are
 * read from it when a context is created and every new measurement is
 * written back to it.  The choice changes no result bit: with either width a
 * lane adds the same cases in the same order.  Unknown policy:
 * BEAGLE_E_INVALID_ARG. */
beagle_status beagle_ctx_set_tuning(beagle_ctx* ctx, int policy);

/* The tile width beagle_eval uses for a problem shape under the current
 * policy (instrumentation): *cases_per_lane = 8 or 4, or 0 when
 * BEAGLE_TUNE_AUTO has not measured the bucket yet.  Only sizes are read. */
beagle_status beagle_ctx_tile_width(beagle_ctx* ctx, int kind, int32_t D, int64_t M, int64_t n_tokens,
                                    int32_t n_programs, int32_t* cases_per_lane);

/* Ragged batching: n_problems independent populations, each on its own
 * dataset (its own M and D), evaluated by one launch sequence whose work
 * lists span every problem (the paper batches the population onto the GPU,
 * section 2.1.2, and runs many benchmark problems, section 2.4).
 *   progs, data  HOST arrays of n_problems descriptors (device pointers inside)
 *   fitness      HOST array of n_problems device pointers,
 *                double[progs[q].n_programs] out
 *   status       HOST array of n_problems device pointers (int8[n_programs]
 *                out), or NULL; entries may be NULL
 * The context captures the launch sequence in a HIP graph the first time it
 * meets a problem table (every pointer and size above, the tile widths and
 * the workspace) and replays that graph while the table is unchanged; the
 * table itself is copied to the device before every launch.  Results are
 * bit-identical to beagle_eval on each problem alone, except on problems
 * that beagle_eval gives to its resident-inputs kernel (at least 4096
 * programs on a case set whose inputs fit 64 KB in one chunk): there the
 * partial sums are added in another order (same accuracy).  Problems with no
 * programs are skipped.  The workspace must hold every problem at once
 * (BEAGLE_E_NOMEM beyond the context cap: no slicing here).  Correlation
 * fitness needs M >= 2 in every problem.  n_problems <= 65535. */
beagle_status beagle_eval_batched(beagle_ctx* ctx, const beagle_programs* progs, const beagle_dataset* data,
                                  int32_t n_problems, int kind, double* const* fitness, int8_t* const* status,
                                  beagle_stream stream);

/* Graph cache counters of beagle_eval_batched (instrumentation): graphs
 * captured and graph launches since the context was created. */
beagle_status beagle_ctx_graph_stats(beagle_ctx* ctx, int64_t* captures, int64_t* replays);

/* Parameters of initialisation and of one generation step. */
typedef struct {
  int32_t tournament;     /* entrants per tournament, >= 1                       */
  float p_crossover;      /* probability of subtree crossover                    */
  float p_mutation;       /* probability of point mutation; rest = copy          */
  int32_t max_len;        /* token capacity of a child slot, <= BEAGLE_MAX_LEN    */
  int32_t max_consts;     /* constant capacity of a child slot, <= 255           */
  float const_lo;         /* new constants ~ U(const_lo, const_hi)               */
  float const_hi;
  int32_t init_depth_min; /* ramped half-and-half depths, 2^(max+1)-1 <= max_len */
  int32_t init_depth_max;
  int32_t op_set;         /* operators drawn by initialisation and mutation:
                             0 = + - * / sin cos exp log sqrt;
                             1 = those and the rest of the paper's table
                             (parameter table, section 2.1.7): x^2, 1/x, tan,
                             asin, acos, atan, tanh.  Function draws are
                             uniform over the set in the order + - * /, then
                             the unary operators in opcode order            */
} beagle_gen_params;

/* The initial population of the evolutionary loop (sections 1 and 2.1.2:
 * initialise, then evaluate, select and vary each generation), by ramped
 * half-and-half (the paper does not name its initialisation):
 * n programs over D variables
 * into fixed-capacity slots: tokens[c * max_len ...] (zero padded),
 * len[c], consts[c * max_consts ...] (zero padded), const_count[c].
 * Random draws come from Philox4x32-10 keyed by `seed` (see
 * beagle_generation for the counter layout; initialisation uses generation
 * field 0 and tag 0x80000000 | problem). */
beagle_status beagle_init_population(beagle_ctx* ctx, const beagle_gen_params* params, int32_t n, int32_t D,
                                     uint64_t seed, uint32_t problem, uint16_t* tokens, int32_t* len,
                                     float* consts, int32_t* const_count, beagle_stream stream);

/* One generation of the loop of sections 1 and 2.1.2 (select, then vary
 * the genomes; mutation as the random correction of section 2.1.4,
 * crossover beside it): for every child slot c in [0, n_programs), size-t
 * tournament selection on `fitness` (lower is better, NaN worst, ties to
 * the lower index), then subtree crossover, point mutation or a copy, into
 * fixed-capacity child slots laid out as for beagle_init_population.
 * Child c draws from Philox4x32-10 with key = seed (low word first) and
 * counter (c, generation, block, problem); draw j is word j % 4 of block
 * j / 4, in this layout: 0 operator choice, 1..t tournament A, t+1..2t
 * tournament B, 2t+1 and 2t+2 crossover points in A and B, 2t+3 mutation
 * position, 2t+4 mutation symbol, 2t+5 mutation constant.  Children are
 * bit-exact functions of (parents, fitness, params, D, seed, generation,
 * problem).  Parents must be valid programs (use the status output of an
 * evaluation); the child arrays must not overlap the parents. */
beagle_status beagle_generation(beagle_ctx* ctx, const beagle_programs* parents, const double* fitness,
                                const beagle_gen_params* params, int32_t D, uint64_t seed, uint64_t generation,
                                uint32_t problem, uint16_t* child_tokens, int32_t* child_len,
                                float* child_consts, int32_t* child_const_count, beagle_stream stream);

/* One generation under microcosm selection (the paper's Monte-Carlo
 * population control, section 2.1.6): a random sample of `sample`
 * individuals, sorted by fitness, stands in for the ranking of the whole
 * population; its entry at position ceil(keep * sample) - 1 (keep in
 * (0, 1], the product in binary64) is the threshold tau, and one pass over
 * the population keeps every individual whose fitness is not NaN and
 * <= tau (every non-NaN one when tau is NaN; every individual when none
 * survives).  Then n_children child slots (any count, so that the
 * population can follow a size schedule) are filled as in
 * beagle_generation, except that parents A and B are survivors drawn
 * uniformly: survivor[below(draw 1, S)] and survivor[below(draw t+1, S)],
 * S the survivor count, survivors in index order.  With p_crossover = 0
 * and p_mutation = 1 every child is a point mutant of a survivor.
 *   sample      1 .. 1024 individuals, drawn with replacement: draw j of the
 *               Philox4x32-10 stream with key = seed and counter
 *               (0xFFFFFFFF, generation, j / 4, 0x40000000 | problem),
 *               word j % 4, picks individual below(u, n_programs)
 *   order       lower fitness first, NaN last, ties by draw position
 *   problem     < 2^30
 *   threshold   DEVICE double[1] out (tau), or NULL
 *   n_survivors DEVICE int32[1] out (survivors; 0 means none survived and
 *               every parent was eligible), or NULL
 * Children are bit-exact functions of (parents, fitness, params, D, sample,
 * keep, seed, generation, problem).  The survivor list lives in the context
 * workspace (4 bytes per parent): calls on one context must be ordered, as
 * for the evaluations.  n_children may be 0 (selection only). */
beagle_status beagle_generation_microcosm(beagle_ctx* ctx, const beagle_programs* parents, const double* fitness,
                                          const beagle_gen_params* params, int32_t D, int32_t sample, float keep,
                                          uint64_t seed, uint64_t generation, uint32_t problem, int32_t n_children,
                                          uint16_t* child_tokens, int32_t* child_len, float* child_consts,
                                          int32_t* child_const_count, double* threshold, int32_t* n_survivors,
                                          beagle_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BEAGLE_H */
