/*
 * pcfgsmc -- SMC over PPL control-flow graphs on AMD Instinct MI355X (gfx950).
 *
 * C interface of libpcfgsmc.so. It follows the statement of the problem in
 * Lunden et al., "Compiling Universal Probabilistic Programming Languages with
 * Efficient Parallel Sequential Monte Carlo Inference" (ESOP 2022):
 *
 *   smc_model_register  <->  a PCFG (B, S, sim, b0, b_stop, L)          Sec. 3.1
 *   smc_init            <->  Algorithm 1, step 1 (initialisation)      Sec. 3.2
 *   smc_step            <->  Algorithm 1, step 2 (propagation)         Sec. 3.2
 *   smc_resample        <->  Algorithm 1, step 3 (resampling), with the
 *                            systematic scheme and the normalising-constant
 *                            estimate of the RootPPL engine              Sec. 3.3
 *   smc_done            <->  the engine's termination check            Sec. 3.3
 *   smc_log_z           <->  the normalising-constant estimate          Sec. 3.3
 *   SMC_MODEL_PROGRAM   <->  a PCFG compiled from a program (Algorithm 2,
 *                            explicit call-stack frames)                 Sec. 4
 *
 * Conventions
 *  - Every handle is opaque. Every function returns an smc_status; no C++
 *    exception crosses this interface. On an error, smc_last_error() returns a
 *    thread-local message describing the most recent failure on that thread.
 *  - Pointers marked "host" are ordinary CPU memory owned by the caller and
 *    only read (or written, for outputs) during the call. Device memory is
 *    allocated by the library through the context's allocator and released by
 *    the matching destroy call.
 *  - Work is enqueued on the context's HIP stream and runs asynchronously.
 *    smc_done, smc_log_z, smc_read, smc_run_stats, smc_batch_poll,
 *    smc_resample_weights, smc_snapshot, smc_restore, smc_set_bucketing, the
 *    self-tests and the destroy calls synchronise with that stream.
 *    smc_program_check needs no device at all.
 *  - Runs are deterministic: the same model, particle count and seed give the
 *    same ancestors, block indices and states, alone or inside a batch.
 *
 * Random numbers. Word k drawn by particle n in round r is word (k mod 4) of
 * Philox4x32-10 (Salmon et al., SC'11) with counter {k/4, n, r, 0} and key
 * {seed & 0xffffffff, seed >> 32}; the resampling offset of round r is word 0
 * of counter {0, 0, r, 1}. A uniform from word w is (2w + 1) 2^-33.
 *
 * Resampling. With M = max lw, w_n = exp(lw_n - M) is rounded to the grid
 * 2^-G, G = min(32, 53 - ceil(log2 N)), so the FP64 prefix sums are exact; with
 * Q_n the inclusive sums and U the round's offset word, output j takes the
 * ancestor a_j = min{ i : N Q_i 2^32 > (j 2^32 + U) Q_{N-1} }. log Z gains
 * (M + log sum_n exp(lw_n - M)) - log N per round, and once more, without
 * resampling, when every particle has stopped.
 */
#ifndef PCFGSMC_H
#define PCFGSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smc_status;
enum {
    SMC_OK = 0,
    SMC_FINISHED = 1,        /* informational: every particle reached b_stop */
    SMC_ERR_INVALID = -1,    /* bad argument; nothing was allocated or enqueued */
    SMC_ERR_OOM = -2,        /* the allocator returned NULL */
    SMC_ERR_DEVICE = -3,     /* a HIP call failed; see smc_last_error() */
    SMC_ERR_STATE = -4,      /* call out of order (e.g. two smc_step without smc_resample) */
    SMC_ERR_NAN = -5,        /* a log-weight was NaN or +inf (a model bug) */
    SMC_DEGENERATE = -6      /* every log-weight was -inf; log Z = -inf and the run stops */
};

typedef struct smc_ctx smc_ctx;
typedef struct smc_model smc_model;
typedef struct smc_run smc_run;
typedef struct smc_batch smc_batch;

/* Device-memory allocator. alloc(ctx, bytes) returns device memory or NULL;
 * free(ctx, p) releases it. Both are called on the host thread that makes the
 * library call. Passing NULL for the allocator selects hipMalloc / hipFree. */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes);
    void (*free)(void* ctx, void* p);
    void* ctx;
} smc_allocator;

/* Built-in block tables. */
enum {
    SMC_MODEL_GEOMETRIC = 0, /* Sec. 2, Fig. 2: weighted geometric program */
    SMC_MODEL_LGSSM = 1,     /* eq. (2), Fig. 4: linear-Gaussian state-space model */
    SMC_MODEL_CRBD = 2,      /* Appendix B listing: constant-rate birth-death */
    SMC_MODEL_CLADS = 3,     /* birth-death with cladogenetic rate shifts */
    SMC_MODEL_SEIR = 4,      /* Appendix listing: vector-borne disease (SEIR) */
    SMC_MODEL_CRBD_DS = 5,   /* CRBD with static delayed sampling (Sec. 5.3) */
    SMC_MODEL_PROGRAM = 6    /* compiled program: bytecode blocks over a per-particle stack (Sec. 4) */
};

/* Compiled programs (SMC_MODEL_PROGRAM). Sec. 4 compiles CorePPL programs to
 * PCFGs whose blocks share a program state holding an explicit call stack
 * (Sec. 4.1); the host tool paper_2112_00364_amd/ppl.py produces such PCFGs
 * (Algorithm 2 for the block split) as bytecode for the library's
 * interpreter. Per particle the state is the block index, a stack pointer sp
 * and a stack of stack_words 8-byte words (FP64; block indices and relative
 * addresses are stored as exact integers); resampling copies only the live
 * part [0, sp) of the ancestor's stack (Sec. 3.3).
 *
 * Instructions are 64-bit words: op | x << 8 | y << 16 | z << 24 | imm << 32
 * (imm: 32 bits, signed where it is a number). r[0..15] are FP64 registers
 * that live for one block execution; fp is the frame base of the running
 * block. Block b is code[block_start[b] .. block_start[b + 1]).
 *   1 FRAME F        fp = sp - F (first instruction of every block; F = the
 *                    frame size of the block's function, 0 for a block that
 *                    belongs to none)
 *   2 CONST x, k     r[x] = consts[k]            3 IMM x, v   r[x] = v
 *   4 MOV x, y       r[x] = r[y]
 *   5 LDF x, o       r[x] = stack[fp + o]        6 STF x, o   stack[fp + o] = r[x]   (o < F)
 *   7..10 ADD SUB MUL DIV x, y, z                r[x] = r[y] op r[z]
 *   11..14 LT LE EQ NE x, y, z                   r[x] = 1 if r[y] op r[z] else 0
 *   15..20 NEG NOT LOG EXP SQRT FLOOR x, y       r[x] = f(r[y]) (NOT: 1 iff r[y] == 0)
 *   21 DATA x, y, a  r[x] = element r[y] of data array a
 *   22 LEN x, a      r[x] = length of data array a
 *   23 SAMPLE x, y, z, d    r[x] ~ distribution d with arguments r[y], r[z]
 *   24 OBSERVE x, y, z, d   log-weight += log density of r[x] under d(r[y], r[z])
 *   25 WEIGHT x      log-weight += r[x]
 *   26 JZ x, t       if r[x] == 0 continue at code[t]   27 JMP t   continue at code[t]
 *                    (t must lie after the jump, inside the same block)
 *   28 CALLFRAME F   open a callee frame of F words at sp (F <= stack_words - sp)
 *   29 STN x, o      stack[sp + o] = r[x]        (o < the open callee frame's F)
 *   30 ADDR x, o     r[x] = fp + o (a relative address)
 *   31 PUSH F        sp += F (closes the open callee frame; same F)
 *   32 STRET x       stack[stack[fp + 1]] = r[x] (the return-value location)
 *   33 GOTO b        next block b, same round     34 CKPT b   next block b after the checkpoint
 *   35 JRET F        next block stack[fp] (a block or 255 = b_stop), sp -= F
 *   36 FAULT         the particle's weight becomes -inf and it stops
 * Every block's last instruction is GOTO, CKPT, JRET or FAULT. Distributions
 * d: 0 uniform(a, b), 1 normal(mean, sd), 2 exponential(rate), 3 gamma(shape
 * >= 1, scale), 4 beta(a >= 1, b >= 1), 5 bernoulli(p), 6 poisson(mean),
 * 7 binomial(n, p); OBSERVE takes 0, 1, 2, 5, 6, 7. Draws use the samplers of
 * the built-in models (word order included).
 * Run-time faults make the particle's weight -inf and stop it: stack
 * overflow, a frame larger than sp, a data index that is not an integer in
 * range, an invalid sampler argument (gamma or beta shape below 1, Poisson
 * mean above 10^4, binomial n not a count in [0, 2^31) or p outside [0, 1]),
 * a return-value location or return block that is out of range, and more
 * than 65536 block executions by one particle in one round.
 * The block index is a byte: at most 254 blocks (255 is b_stop). */
typedef struct {
    uint32_t n_blocks;           /* block 0 is b0, executed first by every particle */
    const uint32_t* block_start; /* [n_blocks + 1], increasing, last = n_code */
    const uint64_t* code;        /* [n_code] */
    uint32_t n_code;             /* at most 2^20 */
    const double* consts;        /* [n_consts] */
    uint32_t n_consts;
    const double* data;          /* every data array, concatenated */
    uint32_t n_data;
    const uint32_t* array_start; /* [n_arrays + 1], increasing from 0 to n_data */
    uint32_t n_arrays;
    uint32_t stack_words;        /* stack capacity per particle, 1 .. 4096 words */
} smc_program_desc;

/* Validates a program description (the same checks smc_model_register makes
 * for SMC_MODEL_PROGRAM; no device needed): SMC_OK, or SMC_ERR_INVALID with
 * smc_last_error naming the first problem (block and instruction). */
smc_status smc_program_check(const smc_program_desc* program);

/* Model description (all pointers are host memory, deep-copied to the device
 * by smc_model_register; the caller keeps ownership).
 *
 * precision: 32 or 64, the storage precision of real-valued particle state.
 *   Block arithmetic is FP64; log-weights and resampling are always FP64.
 * params, by kind (positions are part of the interface):
 *   GEOMETRIC  {p_heads, weight factor}; checkpoint = 1 resamples after every
 *              heads, 0 gives one importance-sampling pass.
 *   LGSSM      {a, b, q_sd, r_sd, m0, s0_sd}: x0 ~ N(m0, s0),
 *              x_t = a x_{t-1} + b + N(0, q), y_t ~ N(x_t, r); y has T entries.
 *   CRBD       {rho, lambda scale, mu scale, fixed lambda (>0 fixes it),
 *              fixed mu (>=0 fixes it), max hidden events, max depth}.
 *   CLADS      {rho, lambda0 scale, eps lo, eps hi, alpha lo, alpha hi,
 *              sigma scale, max events, max depth, fixed lambda0 (>0),
 *              fixed eps (>=0), fixed alpha (>0), fixed sigma (>=0)}.
 *   CRBD_DS    as CRBD (fixed-rate entries unused; the prior scales must be
 *              positive): lambda and mu are not sampled but marginalised by
 *              Gamma conjugacy, each particle carrying their posterior shape
 *              and scale (fields a_lambda, th_lambda, a_mu, th_mu, then the
 *              node). Hidden speciation counts come from the Negative Binomial
 *              predictive and hidden lifetimes from the Lomax predictive;
 *              branch survival weighs -a_mu log(1 + th_mu t) and an observed
 *              speciation log(a_lambda th_lambda), each followed by the
 *              conjugate update.
 *   SEIR       {humans n in [1, 10^7], fixed hLambda, hDelta, hGamma, mLambda,
 *              mDelta, rho (each in [0, 1]; < 0 draws it from the listing's
 *              Beta prior), fixed initial hE, hI, hR, mS (integers; < 0 draws
 *              them)}; y has T daily counts of reported new cases (-1 =
 *              missing). The init block conditions on y_0 and each later
 *              round simulates one day t and conditions on y_t. Fields: six
 *              rates (storage precision), then int32 hS, hE, hI, hR, mS, mE,
 *              mI, mR, z (new infectious humans since the last observation)
 *              and the day.
 * Hidden-event budgets must lie in [0, 10^6] and recursion depths in [1, 32].
 * ess_threshold: 0 resamples every round (Algorithm 1). A value tau in (0, 1]
 *   turns on resampling triggered by the effective sample size (listed among
 *   RootPPL's features in Sec. 3.3): after each propagation the ESS is taken on
 *   the quantised weights q of the resampling step, ESS = (sum q)^2 / sum q^2,
 *   and the round resamples iff ESS < t N / 2^16 with t = rint(tau 2^16)
 *   (decided exactly in integers). A round that does not resample keeps the
 *   log-weights (the next propagation adds to them), takes the identity as
 *   ancestors and leaves log Z unchanged; the next resampling, or the end of
 *   the run, folds the carried weights into log Z. Values outside [0, 1] are
 *   rejected.
 * Trees (CRBD, CLADS): n_nodes = 2 tips - 1 nodes in preorder, root 0, left
 * subtree first; parent[root] = -1, left/right = -1 at tips; age = time before
 * the present (tips 0). */
typedef struct {
    int32_t kind;
    int32_t precision;
    int32_t checkpoint;
    int32_t n_nodes;
    const int32_t* parent;
    const int32_t* left;
    const int32_t* right;
    const double* age;
    int32_t T;
    const double* y;
    double params[16];
    double ess_threshold;
    const smc_program_desc* program; /* SMC_MODEL_PROGRAM only (precision must be 64) */
} smc_model_desc;

/* Context: one device, one stream. stream is a hipStream_t (NULL = the null
 * stream); allocator may be NULL. */
smc_status smc_ctx_create(int32_t device, void* stream, const smc_allocator* allocator, smc_ctx** out);
smc_status smc_ctx_destroy(smc_ctx* ctx); /* NULL-safe; the caller destroys runs, batches and models first */

/* Register a PCFG (Sec. 3.1): validates the description and uploads constant
 * data (tree arrays, observations). */
smc_status smc_model_register(smc_ctx* ctx, const smc_model_desc* desc, smc_model** out);
smc_status smc_model_destroy(smc_model* model); /* NULL-safe */

/* Algorithm 1 step 1: N particles at block b0 with zero state and zero
 * log-weight. N must be in [1, 2^24]. */
smc_status smc_init(smc_model* model, uint64_t n_particles, uint64_t seed, smc_run** out);

/* Algorithm 1 step 2: every particle not at b_stop runs blocks until a
 * checkpoint or b_stop (one kernel launch). Must alternate with smc_resample. */
smc_status smc_step(smc_run* run);

/* Algorithm 1 step 3: log Z update, systematic ancestors, and the gather of
 * (state, block) by ancestor (performed on read by the next smc_step). When
 * every particle is at b_stop, only the log Z update runs and the run
 * finishes. With an ESS threshold, a round whose ESS is high enough skips the
 * resampling and the log Z update and carries the weights (see
 * smc_model_desc). */
smc_status smc_resample(smc_run* run);

/* Termination check (synchronises): *done = 1 when the run finished,
 * degenerated or failed; returns that status. */
smc_status smc_done(smc_run* run, int32_t* done);

/* Normalising-constant estimate so far (synchronises). */
smc_status smc_log_z(smc_run* run, double* out);

/* Step and resample until the run ends. For models whose particles advance in
 * lockstep (LGSSM, CRBD, CLADS) all rounds are enqueued before one termination
 * check; once a run has been reset (smc_reset), its rounds are captured into
 * one HIP graph and every later run of it replays that graph. Other models
 * check termination every 16 rounds. Returns SMC_FINISHED or the failure
 * status. */
smc_status smc_run_to_end(smc_run* run);

/* Checkpoint and resume. smc_snapshot copies a run's complete state between
 * calls (control block with round, log Z and status, both particle buffers,
 * log-weights, ancestors, auxiliary stacks, and where the run stands in
 * Algorithm 1's step/resample alternation) to a caller-owned host buffer: with
 * host_dst NULL it only stores the size needed in *bytes. smc_restore loads
 * such a snapshot into a run of the same model kind, precision and particle
 * count (a fresh smc_init, or the same run later), after which the run
 * continues exactly as the snapshotted one would have. Both synchronise;
 * a snapshot of another shape is rejected with SMC_ERR_INVALID. */
smc_status smc_snapshot(smc_run* run, void* host_dst, size_t* bytes);
smc_status smc_restore(smc_run* run, const void* host_src, size_t bytes);

/* Lanes per work-group of a single run's propagation: 128 or 256 (the
 * default depends on the model kind; batches keep it). The results do not
 * depend on it. Synchronises; a captured graph of the run is dropped. */
smc_status smc_set_workgroup(smc_run* run, int32_t lanes);

/* Block bucketing. Particles may sit at different blocks of the PCFG at the
 * same time (Sec. 3.2), and lanes of one wavefront running different blocks
 * take turns. enable = 1: before every smc_step the
 * run's particle slots are sorted, stably, by the block each will resume at
 * (b_stop last), and lane i of the propagation takes the i-th slot of that
 * order, so the lanes of a wavefront mostly run the same block. Slots keep
 * their random streams: results are bit-identical either way. Costs three
 * small launches per round and N + 256 (N / 1024 + 1) 32-bit words of device
 * memory (allocated on first use); pays off when particles resume at
 * different blocks (compiled programs). Single runs only (not batches).
 * Synchronises; a captured graph of the run is dropped and captured again. */
smc_status smc_set_bucketing(smc_run* run, int32_t enable);

/* Algorithm 1 step 1 again on the run's existing buffers, with a new seed:
 * no allocation; the next smc_run_to_end replays (capturing it the first time)
 * a graph of all rounds. */
smc_status smc_reset(smc_run* run, uint64_t seed);

/* Copy per-particle data to a caller-owned host buffer (synchronises).
 * what: SMC_READ_BLK (uint8 per particle; 255 = b_stop), SMC_READ_LW (double),
 * SMC_READ_ANC (uint32: ancestors of the last smc_resample; the identity when
 * the ESS rule kept the weights), or
 * SMC_READ_FIELD0 + k for state field k in the model's field order (real fields
 * in the storage precision, then int32 fields, then the ClaDS rate stack as
 * [particle][level] with smc_run_stats().stack_depth levels; for a compiled
 * program: int32 stack pointer, then the stack as [particle][word] of
 * stack_words FP64 words, of which the first sp are live). State is returned
 * as Algorithm 1 holds it: after smc_resample, already gathered by ancestor.
 * bytes must be at least the size of the array. */
enum { SMC_READ_BLK = 0, SMC_READ_LW = 1, SMC_READ_ANC = 2, SMC_READ_FIELD0 = 16 };
smc_status smc_read(smc_run* run, int32_t what, void* host_dst, size_t bytes);

typedef struct {
    uint32_t round;          /* rounds propagated so far */
    int32_t status;          /* SMC_OK while running */
    uint64_t block_steps;    /* executions of the model's blocks (b_stop excluded) */
    double log_z;
    int32_t stack_depth;     /* ClaDS: pending-rate stack levels per particle */
    uint32_t resamples;      /* rounds that resampled (every round but the last without an ESS threshold) */
} smc_stats;
smc_status smc_run_stats(smc_run* run, smc_stats* out);

smc_status smc_run_destroy(smc_run* run); /* NULL-safe */

/* Per-kernel timing with HIP events recorded on the context stream around
 * every launch a run makes while profiling is on (smc_step, smc_resample,
 * smc_run_to_end). Index 0 = propagation (with the deep-stack recomputation),
 * 1 = block bucketing (smc_set_bucketing), 2 = reduction (+ the fold of the tile sums for runs above 2^20
 * particles), 3 = scan and ancestors (log Z, next round); ms = summed
 * durations, launches = count. smc_profile(run, 1) clears previous records;
 * both calls synchronise. */
typedef struct {
    double ms[4];
    uint64_t launches[4];
} smc_kernel_times;
smc_status smc_profile(smc_run* run, int32_t enable);
smc_status smc_profile_read(smc_run* run, smc_kernel_times* out);

/* Resampling alone (Algorithm 1 step 3) on a device array of n log-weights:
 * writes the log Z increment (device double) and the n ancestors (device
 * uint32) for round `round` under `seed`. lw, anc and logz_inc are device
 * pointers owned by the caller. Returns SMC_DEGENERATE / SMC_ERR_NAN as a run
 * would (synchronises to report them). */
smc_status smc_resample_weights(smc_ctx* ctx, const double* lw, uint64_t n, uint64_t seed,
                                uint32_t round, uint32_t* anc, double* logz_inc);

/* smc_resample_weights for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same results and status codes, the same
 * kernels, but no hipMalloc, hipFree or allocator call. Its control block,
 * group slots and per-tile partials live in a static device array of about
 * 390 KB that each GPU holds from smc_ctx_create (which looks up its address)
 * until the process ends; n is limited to 2^24 (SMC_ERR_INVALID beyond). Every
 * call on one GPU shares that array and re-initialises it on the device, so
 * calls on one GPU must not overlap (two streams or threads at once race).
 * Synchronises with the context stream. */
smc_status smc_resample_weights_noalloc(smc_ctx* ctx, const double* lw, uint64_t n, uint64_t seed,
                                        uint32_t round, uint32_t* anc, double* logz_inc);

/* Batches: many independent runs advanced together (the batching of many SMC
 * runs on one GPU; the paper's engine runs one). Segmented runs: every round
 * of a tick is one propagation launch per (model kind, precision, work-group
 * size) group over a (run, tile) table of all live runs, then one reduction
 * and one scan launch over a table of every run's reduction tiles; each run's
 * tiles read that run's own control block, so runs of different sizes, trees
 * and round counts share the launches and finished runs drop out at once.
 * Owned runs (smc_batch_set_owned): one work-group advances the run through
 * all the rounds of a tick by itself, one launch per (kind, precision) for
 * all such runs, so each moves at its own pace. Results are identical to the
 * same runs executed alone either way. */
smc_status smc_batch_create(smc_ctx* ctx, smc_batch** out);
/* Add a run (Algorithm 1 step 1 for it); *slot receives its index. The model
 * may be registered on another context of the same device (registration
 * synchronises its own stream, so a server can register on an idle context
 * while the batch's stream is busy). */
smc_status smc_batch_add(smc_batch* b, smc_model* model, uint64_t n_particles, uint64_t seed, int32_t* slot);
/* Advance every live run by up to `rounds` rounds (step + resample each).
 * From the second tick with the same runs and round count on, the tick's
 * launch sequence is captured once into a HIP graph and replayed; adding or
 * retiring a run drops the graph. Results are the same either way. */
/* Lanes per propagation work-group of the run in `slot` (128 or 256, as
 * smc_set_workgroup for a single run; a launch option chosen by the
 * autotuner, results unchanged). The run's tiles move to the launch group of
 * that size at the next tick. */
smc_status smc_batch_set_workgroup(smc_batch* b, int32_t slot, int32_t lanes);
/* owned != 0: from the next tick one work-group of 256 lanes owns the run in
 * `slot` through every round of each tick (its propagation, reduction and
 * scan tiles in turn); owned == 0: back to the segmented launches. Only
 * built-in models (not SMC_MODEL_PROGRAM) of at most 4096 particles can be
 * owned (SMC_ERR_INVALID otherwise). A launch option, results unchanged. */
smc_status smc_batch_set_owned(smc_batch* b, int32_t slot, int32_t owned);
smc_status smc_batch_tick(smc_batch* b, int32_t rounds);
/* Synchronises. done[i] = 1 for finished (or failed) slots; log_z[i] their
 * estimates; status[i] their status. Arrays are host, length = slots. */
smc_status smc_batch_poll(smc_batch* b, int32_t slots, int32_t* done, double* log_z, int32_t* status,
                          uint64_t* block_steps);
/* Free a finished slot's device memory; the slot may be reused by smc_batch_add. */
smc_status smc_batch_retire(smc_batch* b, int32_t slot);
smc_status smc_batch_destroy(smc_batch* b); /* NULL-safe */

/* Self-test entry points: evaluate the device's pinned primitives on n inputs.
 * in and out are device arrays of doubles.
 * op 0 exp(x), 1 log(x), 2 cos(2 pi u), 3 sqrt(x), 4 uniform from word w
 * (input = w as a double), 5 Box-Muller normal from the word pair
 * (in[2i], in[2i+1]) -> out[i], 6 Poisson(in[2i]) drawn from the stream of
 * seed in[2i+1] (an integer below 2^53), particle i, round 0, tag 0, from word
 * 0 -> out[i] (-1 when the mean exceeds the event cap); 7 Binomial(in[3i],
 * in[3i+1]) and 8 Gamma(in[3i]) (in[3i+1] < 0) or Beta(in[3i], in[3i+1]), each
 * the first draw of the stream of seed in[3i+2], particle 0, round 0, tag 0;
 * 9 log k! of k = in[i]; 10 log of the Binomial(in[3i+1], in[3i+2])
 * probability of in[3i]; 11 the Negative Binomial predictive of a
 * Poisson(rate) count and 12 the Lomax predictive of an Exponential(rate)
 * lifetime, rate ~ Gamma(shape in[3i], scale in[3i+1]), first draw of the
 * stream of seed in[3i+2]; 13 exp, 14 log and 15 cos(2 pi u) in the form with
 * compiler-placed polynomial coefficients (the ClaDS propagation's), which
 * must give the same bits as ops 0-2. */
smc_status smc_selftest_math(smc_ctx* ctx, int32_t op, const double* in, double* out, uint64_t n);
/* Philox4x32-10 on n counters: ctr (device, 4 x uint32 each), key (2 x uint32
 * each), out (device, 4 x uint32 each). */
smc_status smc_selftest_philox(smc_ctx* ctx, const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n);

const char* smc_last_error(void);
const char* smc_version(void);

#ifdef __cplusplus
}
#endif
#endif
