/*
 * CPU oracle for SMC over PPL control-flow graphs (PCFGs).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, single-threaded,
 * obviously-correct reference that the GPU path is checked against. Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it. It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (Lunden et al., "Compiling Universal Probabilistic
 * Programming Languages with Efficient Parallel Sequential Monte Carlo
 * Inference", ESOP 2022):
 *   - a PCFG (B, S, sim, b0, b_stop, L) as a block table over per-particle
 *     state (Sec. 3.1);
 *   - Algorithm 1 (Sec. 3.2): initialisation, propagation until every particle
 *     reaches a checkpoint, resampling; finished particles keep taking part in
 *     resampling (the b_stop fixpoint, Sec. 3.2);
 *   - systematic resampling (Sec. 3.3) and the normalising-constant estimate
 *     log Z (Sec. 3.3).
 * Every choice the paper leaves open (RNG, elementary functions, samplers,
 * weight quantisation before the cumulative sum, caps on the recursion of the
 * birth-death simulation) is pinned in the comments of smc_oracle.c.
 */
#ifndef SMC_ORACLE_H
#define SMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_GEOMETRIC = 0, OR_LGSSM = 1, OR_CRBD = 2, OR_CLADS = 3, OR_SEIR = 4, OR_CRBD_DS = 5 };
enum { OR_OK = 0, OR_FINISHED = 1, OR_ERR_INVALID = -1, OR_ERR_NAN = -5, OR_DEGENERATE = -6 };
enum { OR_TAG_PROPAGATE = 0, OR_TAG_RESAMPLE = 1 };
#define OR_STOP 255u

/* Model description. Parameters are read per model kind (see smc_oracle.c). */
typedef struct {
    int32_t kind;       /* OR_GEOMETRIC .. OR_CRBD_DS */
    int32_t precision;  /* 32 or 64: storage precision of real-valued particle state */
    int32_t checkpoint; /* geometric only: 1 = checkpoint after each heads, 0 = none */
    int32_t n_nodes;    /* trees: 2*tips-1 nodes in preorder, root = 0 */
    const int32_t* parent;   /* [n_nodes], -1 for the root */
    const int32_t* left;     /* [n_nodes], -1 for tips */
    const int32_t* right;    /* [n_nodes], -1 for tips */
    const double* age;       /* [n_nodes], tips 0, root largest */
    int32_t T;               /* state-space models: number of observations */
    const double* y;         /* [T] */
    double p[16];            /* model parameters, meaning per kind */
    double ess_threshold;    /* 0: resample every round; (0, 1]: ESS-triggered (see or_ess_resamples) */
} or_model;

typedef struct or_run or_run;

/* Primitives, exported for pin tests. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_exp(double x);
double or_log(double x);
double or_cos2pi(double u);
uint32_t or_word(uint64_t seed, uint32_t k, uint32_t particle, uint32_t round, uint32_t tag);
double or_uniform_from_word(uint32_t w);
int64_t or_poisson_words(double m, const uint32_t* words, int32_t n_words, int32_t* used);
double or_log_factorial(int64_t k);
double or_log_binomial_pmf(int64_t y, int64_t z, double p);
void or_sample(int32_t kind, double a, double b, uint64_t seed, int64_t count, double* out);
/* One draw of a compiled program's sampler from a particle's stream at word *k. */
double or_draw(int32_t dist, double a, double b, uint64_t seed, uint32_t particle, uint32_t round,
               uint32_t* k, int32_t* fault);

/* Resampling alone (Alg. 1 step 3) on a given log-weight vector. */
void or_ancestors(const uint64_t* Q, uint64_t n, uint32_t U, uint32_t* anc);
int32_t or_systematic(const double* lw, uint64_t n, uint64_t seed, uint32_t round,
                      uint32_t* anc, double* logz_increment, uint64_t* qtot_units);
/* The ESS rule on a log-weight vector: 1 = resample, 0 = carry the weights.
 * -1 when the threshold is outside [0, 1]. */
int32_t or_ess_resamples(const double* lw, uint64_t n, double threshold);

/* A run: Alg. 1 driven one step at a time. */
or_run* or_create(const or_model* m, uint64_t n, uint64_t seed);
void or_destroy(or_run* r);
int32_t or_step(or_run* r);      /* Alg. 1 step 2 */
int32_t or_resample(or_run* r);  /* Alg. 1 step 3 (+ log Z); finishes the run when all stopped */
int32_t or_run_to_end(or_run* r);
double or_log_z(const or_run* r);
int32_t or_status(const or_run* r);
uint32_t or_round(const or_run* r);
uint64_t or_block_steps(const or_run* r);
uint32_t or_resamples(const or_run* r);  /* rounds that resampled */
int32_t or_read(const or_run* r, int32_t what, void* dst);
int32_t or_max_stack(const or_run* r);
int32_t or_propagate_particle(const or_model* m, uint64_t seed, uint32_t slot, uint32_t round,
                              uint8_t* blk, double* lw, double* reals, int32_t* ints, double* stack);

/* or_read selectors */
enum { OR_READ_BLK = 0, OR_READ_LW = 1, OR_READ_ANC = 2, OR_READ_FIELD0 = 16 };

#ifdef __cplusplus
}
#endif
#endif
