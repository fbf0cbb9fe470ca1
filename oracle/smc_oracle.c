/*
 * CPU oracle for SMC over PPL control-flow graphs -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded C. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the GPU library never does, and
 * the two share no code. Build: gcc -O2 -ffp-contract=off -fPIC -shared
 * (no -ffast-math: every floating-point operation below is meant to round
 * exactly once, in the order written).
 *
 * Paper: Lunden et al., "Compiling Universal Probabilistic Programming
 * Languages with Efficient Parallel Sequential Monte Carlo Inference".
 *   Sec. 3.1  PCFG (B, S, sim, b0, b_stop, L)
 *   Sec. 3.2  Algorithm 1 (SMC over a PCFG) and the b_stop fixpoint
 *   Sec. 3.3  RootPPL engine: per-particle random streams, systematic
 *             resampling, normalising-constant estimate
 *   Sec. 3.3, Fig. 4 / eq. (2)  the state-space model
 *   Sec. 2, Fig. 2  the weighted geometric program
 *   Appendix B, CRBD listing  the constant-rate birth-death model
 *
 * Pinned readings of what the paper leaves open (each side of the parity
 * check implements these independently):
 *   RNG      Philox4x32-10 (Salmon et al., SC'11). Word k of particle n in
 *            round r under tag g is word (k mod 4) of
 *            Philox(counter = {k/4, n, r, g}, key = {seed lo32, seed hi32}).
 *            Tag 0 = propagation, tag 1 = resampling.
 *   uniform  u = (2w + 1) * 2^-33 from one 32-bit word w: open (0,1), exact.
 *   exp/log  the algorithms in or_exp / or_log below (Cody-Waite reduction,
 *            Taylor / atanh series, Horner with fused multiply-add).
 *   cos2pi   exact quadrant reduction + Taylor series (or_cos2pi).
 *   samplers Exponential(rate) = -log(u)/rate; Gamma(1, scale) = -scale*log(u);
 *            Uniform(a,b) = a + (b-a)u; Bernoulli(p) = [u < p];
 *            Normal = Box-Muller cosine branch; Poisson = chunked inversion.
 *   weights  resampling quantises w_n = exp(lw_n - max lw) onto the grid 2^-G,
 *            G = min(32, 53 - ceil(log2 N)); every partial sum is then exact.
 *   caps     birth-death hidden-event simulation: at most 10^4 events per
 *            block and recursion depth 32; exceeding either gives weight -inf.
 */
#include "smc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the       */
/* Philox S-box on a 128-bit counter under a 64-bit key bumped each round.   */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u; /* golden-ratio Weyl increment */
            k1 += 0xBB67AE85u; /* sqrt(3)-1 Weyl increment */
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t or_word(uint64_t seed, uint32_t k, uint32_t particle, uint32_t round, uint32_t tag)
{
    uint32_t ctr[4] = {k / 4u, particle, round, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return out[k % 4u];
}

double or_uniform_from_word(uint32_t w)
{
    return (2.0 * (double)w + 1.0) * 0x1p-33;
}

/* A particle's random stream for one round: words are drawn in program order. */
typedef struct {
    uint64_t seed;
    uint32_t particle, round, tag, k;
} stream;

static uint32_t next_word(stream* s)
{
    uint32_t w = or_word(s->seed, s->k, s->particle, s->round, s->tag);
    s->k += 1;
    return w;
}

static double next_uniform(stream* s) { return or_uniform_from_word(next_word(s)); }

/* ------------------------------------------------------------------------- */
/* Elementary functions, pinned algorithms (FP64, one rounding per op).      */
/* ------------------------------------------------------------------------- */
static const double OR_LN2_HI = 0.693147182464599609375;            /* ln 2 rounded to 24 bits */
static const double OR_LN2_LO = -1.904654299957767878541823431924e-9; /* ln 2 - OR_LN2_HI */
static const double OR_INV_LN2 = 1.442695040888963407359924681001892137427;
static const double OR_SQRT2 = 1.41421356237309504880168872420969807857;
static const double OR_TWO_PI = 6.283185307179586476925286766559005768394;

static double pow2i(int n) /* 2^n for -1022 <= n <= 1023 */
{
    uint64_t bits = (uint64_t)(n + 1023) << 52;
    double r;
    memcpy(&r, &bits, sizeof r);
    return r;
}

/* exp(x): n = rint(x/ln2), r = (x - n*ln2_hi) - n*ln2_lo, exp(r) by its Taylor
 * polynomial of degree 13 in Horner form with fma, then times 2^n.
 * Results that would be subnormal are flushed: x < -708 gives +0, and
 * x > 709 gives +inf. */
double or_exp(double x)
{
    if (x != x) return x;
    if (x > 709.0) return INFINITY;
    if (x < -708.0) return 0.0;
    double n = nearbyint(x * OR_INV_LN2);
    double r = (x - n * OR_LN2_HI) - n * OR_LN2_LO;
    double p = 1.0 / 6227020800.0;      /* 1/13! */
    p = fma(p, r, 1.0 / 479001600.0);   /* 1/12! */
    p = fma(p, r, 1.0 / 39916800.0);    /* 1/11! */
    p = fma(p, r, 1.0 / 3628800.0);     /* 1/10! */
    p = fma(p, r, 1.0 / 362880.0);      /* 1/9! */
    p = fma(p, r, 1.0 / 40320.0);       /* 1/8! */
    p = fma(p, r, 1.0 / 5040.0);        /* 1/7! */
    p = fma(p, r, 1.0 / 720.0);         /* 1/6! */
    p = fma(p, r, 1.0 / 120.0);         /* 1/5! */
    p = fma(p, r, 1.0 / 24.0);          /* 1/4! */
    p = fma(p, r, 1.0 / 6.0);           /* 1/3! */
    p = fma(p, r, 0.5);                 /* 1/2! */
    p = fma(p, r, 1.0);                 /* 1/1! */
    p = fma(p, r, 1.0);                 /* 1/0! */
    return p * pow2i((int)n);
}

/* log(x): x = 2^k m with m in [sqrt(2)/2, sqrt(2)); f = m - 1; s = f/(2+f);
 * log m = 2 atanh(s) = 2s + 2s z R(z), z = s^2, R(z) = sum_{j=0..9} z^j/(2j+3);
 * log x = k ln2_hi + (k ln2_lo + log m). */
double or_log(double x)
{
    if (x != x) return x;
    if (x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (x == INFINITY) return x;
    int k = 0;
    if (x < 0x1p-1022) { x = x * 0x1p54; k = -54; }
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    k += (int)((bits >> 52) & 0x7ff) - 1023;
    uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mbits, sizeof m);
    if (m > OR_SQRT2) { m = m * 0.5; k += 1; }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    double R = 1.0 / 21.0;
    R = fma(R, z, 1.0 / 19.0);
    R = fma(R, z, 1.0 / 17.0);
    R = fma(R, z, 1.0 / 15.0);
    R = fma(R, z, 1.0 / 13.0);
    R = fma(R, z, 1.0 / 11.0);
    R = fma(R, z, 1.0 / 9.0);
    R = fma(R, z, 1.0 / 7.0);
    R = fma(R, z, 1.0 / 5.0);
    R = fma(R, z, 1.0 / 3.0);
    double two_s = 2.0 * s;
    double log_m = fma(two_s, z * R, two_s);
    double kd = (double)k;
    return kd * OR_LN2_HI + (kd * OR_LN2_LO + log_m);
}

/* cos(2 pi u): q = rint(4u), t = u - q/4 in [-1/8, 1/8] (exact), theta = 2 pi t,
 * then cos(theta + q pi/2) from the Taylor series of sin / cos in theta^2. */
double or_cos2pi(double u)
{
    double q = nearbyint(4.0 * u);
    double t = u - q * 0.25;
    double th = t * OR_TWO_PI;
    double z = th * th;
    double S = 1.0 / 355687428096000.0;    /* 1/17! */
    S = fma(S, z, -1.0 / 1307674368000.0); /* -1/15! */
    S = fma(S, z, 1.0 / 6227020800.0);     /* 1/13! */
    S = fma(S, z, -1.0 / 39916800.0);      /* -1/11! */
    S = fma(S, z, 1.0 / 362880.0);         /* 1/9! */
    S = fma(S, z, -1.0 / 5040.0);          /* -1/7! */
    S = fma(S, z, 1.0 / 120.0);            /* 1/5! */
    S = fma(S, z, -1.0 / 6.0);             /* -1/3! */
    S = fma(S, z, 1.0);
    double sin_th = th * S;
    double C = -1.0 / 6402373705728000.0;  /* -1/18! */
    C = fma(C, z, 1.0 / 20922789888000.0); /* 1/16! */
    C = fma(C, z, -1.0 / 87178291200.0);   /* -1/14! */
    C = fma(C, z, 1.0 / 479001600.0);      /* 1/12! */
    C = fma(C, z, -1.0 / 3628800.0);       /* -1/10! */
    C = fma(C, z, 1.0 / 40320.0);          /* 1/8! */
    C = fma(C, z, -1.0 / 720.0);           /* -1/6! */
    C = fma(C, z, 1.0 / 24.0);             /* 1/4! */
    C = fma(C, z, -0.5);                   /* -1/2! */
    C = fma(C, z, 1.0);
    double cos_th = C;
    int quadrant = ((int)q) & 3;
    if (quadrant == 0) return cos_th;
    if (quadrant == 1) return -sin_th;
    if (quadrant == 2) return -cos_th;
    return sin_th;
}

/* ------------------------------------------------------------------------- */
/* Samplers (pinned).                                                        */
/* ------------------------------------------------------------------------- */
#define OR_POISSON_CAP 10000.0
#define OR_POISSON_MAX_K 10000

/* Poisson(m) by inversion, with m split into ceil(m/32) equal chunks (a sum of
 * independent Poissons is Poisson). One uniform per chunk. Returns -1 when
 * m > 10^4 (the event cap is certainly exceeded) or m is not a number. */
static int64_t poisson_from(double m, uint32_t (*word)(void*), void* ctx)
{
    if (!(m >= 0.0)) return -1;
    if (m > OR_POISSON_CAP) return -1;
    if (m == 0.0) return 0;
    int chunks = (int)ceil(m / 32.0);
    double mc = m / (double)chunks;
    int64_t total = 0;
    for (int c = 0; c < chunks; ++c) {
        double u = or_uniform_from_word(word(ctx));
        double p = or_exp(-mc);
        double F = p;
        int k = 0;
        while (u > F && k < OR_POISSON_MAX_K) {
            k += 1;
            p = p * mc / (double)k;
            F = F + p;
        }
        total += k;
    }
    return total;
}

static uint32_t stream_word_cb(void* ctx) { return next_word((stream*)ctx); }

static int64_t poisson(stream* s, double m) { return poisson_from(m, stream_word_cb, s); }

typedef struct { const uint32_t* w; int32_t n, i; } word_list;
static uint32_t list_word_cb(void* ctx)
{
    word_list* l = (word_list*)ctx;
    uint32_t w = l->i < l->n ? l->w[l->i] : 0u;
    l->i += 1;
    return w;
}

int64_t or_poisson_words(double m, const uint32_t* words, int32_t n_words, int32_t* used)
{
    word_list l = {words, n_words, 0};
    int64_t k = poisson_from(m, list_word_cb, &l);
    if (used) *used = l.i;
    return k;
}

static double exponential(stream* s, double rate) { return -or_log(next_uniform(s)) / rate; }

static double gamma1(stream* s, double scale) { return -scale * or_log(next_uniform(s)); }

static double uniform_ab(stream* s, double a, double b) { return a + (b - a) * next_uniform(s); }

static int bernoulli(stream* s, double p) { return next_uniform(s) < p; }

static double normal01(stream* s)
{
    double u1 = next_uniform(s);
    double u2 = next_uniform(s);
    double radius = sqrt(-2.0 * or_log(u1));
    return radius * or_cos2pi(u2);
}

static double lognormal(stream* s, double mu_ln, double sigma)
{
    double z = normal01(s);
    return or_exp(mu_ln + sigma * z);
}

/* ------------------------------------------------------------------------- */
/* Samplers for the vector-borne disease model (Appendix listing). The paper  */
/* names the distributions (Beta, Binomial, Poisson, Uniform) but not the     */
/* algorithms; the readings:                                                  */
/*  - log k! (or_log_factorial): the sum of log i for k < 16, else the        */
/*    Stirling series in x = k + 1 up to the x^-7 term;                       */
/*  - Gamma(a, 1), a >= 1: Marsaglia and Tsang (2000) without the squeeze:    */
/*    d = a - 1/3, c = 1/sqrt(9d); draw z ~ N(0,1) (Box-Muller as above),     */
/*    v = (1 + c z)^3, rejected if 1 + c z <= 0, else u ~ U(0,1) and accept   */
/*    d v iff log u < z^2/2 + d - d v + d log v;                              */
/*  - Beta(a, b) = X / (X + Y), X ~ Gamma(a), Y ~ Gamma(b);                   */
/*  - Binomial(n, p): 0 when n = 0 or p = 0 (no draw), n when p = 1; for      */
/*    p > 1/2 it is n - Binomial(n, 1 - p); with m = n p < 10, inversion by   */
/*    sequential search from k = 0 (one uniform); otherwise Hoermann's (1993) */
/*    transformed rejection with squeeze, BTRS (two uniforms per try).        */
/* Rejection loops stop after OR_MAX_TRIES tries (probability below 1e-100)  */
/* and then return the last candidate's fallback stated at each sampler.     */
/* ------------------------------------------------------------------------- */
#define OR_MAX_TRIES 256

double or_log_factorial(int64_t k)
{
    if (k < 2) return 0.0;
    if (k < 16) {
        double s = 0.0;
        for (int64_t i = 2; i <= k; ++i) s = s + or_log((double)i);
        return s;
    }
    double x = (double)(k + 1);
    double x2 = x * x;
    double series = (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0 - 1.0 / (1680.0 * x2)) / x2) / x2) / x;
    return ((x - 0.5) * or_log(x) - x) + (0.5 * or_log(OR_TWO_PI) + series);
}

/* log k! - [(k + 1/2) log(k + 1) - (k + 1) + log(2 pi) / 2]: the tail of
 * Stirling's formula used by BTRS. */
static double stirling_tail(int64_t k)
{
    double x = (double)(k + 1);
    return or_log_factorial(k) - (((double)k + 0.5) * or_log(x) - x + 0.5 * or_log(OR_TWO_PI));
}

static double gamma_mt(stream* s, double a)
{
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (int it = 0; it < OR_MAX_TRIES; ++it) {
        double z = normal01(s);
        double w = 1.0 + c * z;
        if (w <= 0.0) continue;
        double v = w * w * w;
        double u = next_uniform(s);
        if (or_log(u) < 0.5 * z * z + d - d * v + d * or_log(v)) return d * v;
    }
    return d; /* fallback: the mode (never reached in practice) */
}

static double beta_draw(stream* s, double a, double b)
{
    double x = gamma_mt(s, a);
    double y = gamma_mt(s, b);
    return x / (x + y);
}

static int64_t binomial_small(stream* s, int64_t n, double p)
{
    double q = 1.0 - p;
    double pk = or_exp((double)n * or_log(q));
    double ratio = p / q;
    double u = next_uniform(s);
    int64_t k = 0;
    while (u > pk && k < n) {
        u = u - pk;
        k += 1;
        pk = pk * ((double)(n - k + 1) / (double)k * ratio);
    }
    return k;
}

static int64_t binomial_btrs(stream* s, int64_t n, double p)
{
    double q = 1.0 - p;
    double spq = sqrt((double)n * p * q);
    double b = 1.15 + 2.53 * spq;
    double a = -0.0873 + 0.0248 * b + 0.01 * p;
    double c = (double)n * p + 0.5;
    double v_r = 0.92 - 4.2 / b;
    double r = p / q;
    double alpha = (2.83 + 5.1 / b) * spq;
    int64_t m = (int64_t)floor((double)(n + 1) * p);
    double h = ((double)m + 0.5) * or_log(((double)m + 1.0) / (r * (double)(n - m + 1))) +
               (stirling_tail(m) + stirling_tail(n - m));
    int64_t k = (int64_t)floor(c);
    for (int it = 0; it < OR_MAX_TRIES; ++it) {
        double u = next_uniform(s) - 0.5;
        double v = next_uniform(s);
        double us = 0.5 - fabs(u);
        double kf = floor((2.0 * a / us + b) * u + c);
        if (us >= 0.07 && v <= v_r) return (int64_t)kf;
        if (kf < 0.0 || kf > (double)n) continue;
        k = (int64_t)kf;
        double lv = or_log(v * alpha / (a / (us * us) + b));
        double bound = h + ((double)(n + 1) * or_log((double)(n - m + 1) / (double)(n - k + 1)) +
                            ((double)k + 0.5) * or_log(r * (double)(n - k + 1) / ((double)k + 1.0))) -
                       (stirling_tail(k) + stirling_tail(n - k));
        if (lv <= bound) return k;
    }
    return (int64_t)floor(c); /* fallback: the mean, rounded (never reached in practice) */
}

static int64_t binomial_draw(stream* s, int64_t n, double p)
{
    if (n <= 0 || !(p > 0.0)) return 0;
    if (p >= 1.0) return n;
    if (p > 0.5) return n - binomial_draw(s, n, 1.0 - p);
    if ((double)n * p < 10.0) return binomial_small(s, n, p);
    return binomial_btrs(s, n, p);
}

/* log of the Binomial(z, p) probability of y, with 0 log 0 = 0. */
double or_log_binomial_pmf(int64_t y, int64_t z, double p)
{
    if (y < 0 || y > z) return -INFINITY;
    double lw = or_log_factorial(z) - (or_log_factorial(y) + or_log_factorial(z - y));
    if (y > 0) lw = lw + (double)y * or_log(p);
    if (z - y > 0) lw = lw + (double)(z - y) * or_log(1.0 - p);
    return lw;
}

/* Negative Binomial predictive of a Poisson(lambda t) count, lambda ~
 * Gamma(a, th): inversion by sequential search; -1 beyond the event cap. */
static int64_t neg_binomial_draw(stream* s, double a, double th, double t)
{
    double lq = or_log(1.0 + th * t);
    double pk = or_exp(-a * lq);
    double q = th * t / (1.0 + th * t);
    double u = next_uniform(s);
    int64_t k = 0;
    while (u > pk) {
        if (k >= OR_POISSON_MAX_K) return -1;
        u = u - pk;
        k += 1;
        pk = pk * (((double)(k - 1) + a) / (double)k * q);
    }
    return k;
}

static double lomax_draw(stream* s, double a, double th)
{
    double u = next_uniform(s);
    return (or_exp(-or_log(u) / a) - 1.0) / th;
}

/* Sampler checks: `count` draws in sequence from the stream of (seed,
 * particle 0, round 0, tag 0). kind 0: Binomial(n = a, p = b); 1: Gamma(a);
 * 2: Beta(a, b); 3: the Negative Binomial predictive of a Poisson(lambda) count
 * with lambda ~ Gamma(a, b); 4: the Lomax predictive of an Exponential(mu)
 * lifetime with mu ~ Gamma(a, b). Results as doubles. */
void or_sample(int32_t kind, double a, double b, uint64_t seed, int64_t count, double* out)
{
    stream s = {seed, 0, 0, OR_TAG_PROPAGATE, 0};
    for (int64_t i = 0; i < count; ++i) {
        if (kind == 0) out[i] = (double)binomial_draw(&s, (int64_t)a, b);
        else if (kind == 1) out[i] = gamma_mt(&s, a);
        else if (kind == 2) out[i] = beta_draw(&s, a, b);
        else if (kind == 3) out[i] = (double)neg_binomial_draw(&s, a, b, 1.0);
        else out[i] = lomax_draw(&s, a, b);
    }
}

/* One draw of a compiled program (Sec. 4) from the stream of particle slot
 * `particle` in round `round`, starting at word *k (advanced past the words
 * used). Distributions: 0 uniform(a, b) = a + (b - a) u; 1 normal(mean a,
 * sd b) = a + b z; 2 exponential(rate a) = -log u / a; 3 gamma(shape a, scale
 * b) = b g, shape >= 1; 4 beta(a, b), both >= 1; 5 bernoulli(a): 1 if u < a;
 * 6 poisson(a); 7 binomial(n = a, p = b) with n a count below 2^31 and p in
 * [0, 1]. *fault = 1 (and 0 returned) when an argument is outside these
 * ranges or the Poisson mean exceeds the event cap; such a particle takes
 * weight -inf and stops. */
double or_draw(int32_t dist, double a, double b, uint64_t seed, uint32_t particle, uint32_t round,
               uint32_t* k, int32_t* fault)
{
    stream s = {seed, particle, round, OR_TAG_PROPAGATE, *k};
    double v = 0.0;
    *fault = 0;
    switch (dist) {
    case 0: v = uniform_ab(&s, a, b); break;
    case 1: v = a + b * normal01(&s); break;
    case 2: v = exponential(&s, a); break;
    case 3:
        if (!(a >= 1.0)) { *fault = 1; break; }
        v = b * gamma_mt(&s, a);
        break;
    case 4:
        if (!(a >= 1.0 && b >= 1.0)) { *fault = 1; break; }
        v = beta_draw(&s, a, b);
        break;
    case 5: v = bernoulli(&s, a) ? 1.0 : 0.0; break;
    case 6: {
        int64_t c = poisson(&s, a);
        if (c < 0) *fault = 1;
        else v = (double)c;
        break;
    }
    case 7:
        if (!(a >= 0.0 && a < 2147483648.0 && a == floor(a) && b >= 0.0 && b <= 1.0)) { *fault = 1; break; }
        v = (double)binomial_draw(&s, (int64_t)a, b);
        break;
    default: *fault = 1;
    }
    *k = s.k;
    return *fault ? 0.0 : v;
}

/* ------------------------------------------------------------------------- */
/* Particle storage (one array per field, as the paper lays particles out).  */
/* ------------------------------------------------------------------------- */
#define OR_MAX_FIELDS 12

struct or_run {
    or_model m;
    uint64_t n, seed;
    uint32_t round;
    int32_t status;
    double log_z;
    uint64_t block_steps;
    int n_real, n_int;         /* real fields (stored as double, rounded to P) and int fields */
    int stack_depth;           /* ClaDS pending-rate stack capacity */
    uint8_t* blk;
    double* lw;
    uint32_t* anc;
    double* real[OR_MAX_FIELDS];
    int32_t* ints[OR_MAX_FIELDS];
    double* stack;             /* [n * stack_depth] */
    uint32_t ess_t;            /* ESS threshold numerator over 2^16 (0: always resample) */
    uint32_t resamples;        /* rounds that resampled */
    /* derived constants, computed once from the model parameters */
    double ln2, log_rho, corr, log_w, obs_c, obs_var, ln10;
    int tips;
};

static double store_p(const or_run* r, double v)
{
    return r->m.precision == 32 ? (double)(float)v : v;
}

/* ------------------------------------------------------------------------- */
/* Geometric (Sec. 2, Fig. 2): flip a coin with P(heads) = p[0]; heads weights */
/* by p[1] and flips again; tails stops. Field int0 = number of flips.       */
/* The checkpointed variant resamples after every heads.                     */
/* ------------------------------------------------------------------------- */
static int geometric_block(or_run* r, uint64_t i, stream* s, int* ckpt)
{
    int heads = bernoulli(s, r->m.p[0]);
    r->ints[0][i] += 1;
    if (heads) {
        r->lw[i] = r->lw[i] + r->log_w;
        *ckpt = r->m.checkpoint != 0;
        return 0;
    }
    *ckpt = 1;
    return (int)OR_STOP;
}

/* ------------------------------------------------------------------------- */
/* Linear-Gaussian state-space model (eq. (2), Fig. 4):                       */
/*   x_0 ~ N(m0, s0), x_t = a x_{t-1} + b + N(0, q), y_t ~ N(x_t, r)  (sd's). */
/* Blocks: 0 init (non-checkpoint jump to iter), 1 iter (checkpoint).        */
/* p = {a, b, q, r, m0, s0}. Fields: real0 = x, int0 = t.                     */
/* ------------------------------------------------------------------------- */
static int lgssm_block(or_run* r, uint64_t i, int b, stream* s, int* ckpt)
{
    const double* p = r->m.p;
    if (b == 0) {
        double z = normal01(s);
        r->real[0][i] = store_p(r, p[4] + p[5] * z);
        r->ints[0][i] = 0;
        *ckpt = 0;
        return 1;
    }
    double z = normal01(s);
    double x = r->real[0][i];
    r->real[0][i] = store_p(r, (p[0] * x + p[1]) + p[2] * z);
    double d = r->m.y[r->ints[0][i]] - r->real[0][i];
    r->lw[i] = r->lw[i] + (r->obs_c - (d * d) / (2.0 * r->obs_var));
    r->ints[0][i] += 1;
    *ckpt = 1;
    return r->ints[0][i] == r->m.T ? (int)OR_STOP : 1;
}

/* ------------------------------------------------------------------------- */
/* CRBD (Appendix B listing): lambda ~ Gamma(1, p[1]), mu ~ Gamma(1, p[2]),   */
/* correction (n-1) log 2 - log n!, then one observed branch per checkpoint  */
/* in preorder (left subtree first). p = {rho, scale_lambda, scale_mu,       */
/* fixed lambda (>0 to fix), fixed mu (>=0 to fix), max events, max depth}.  */
/* Fields: real0 = lambda, real1 = mu, int0 = node cursor.                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    stream* s;
    double lambda, mu, rho;
    int events, max_events, max_depth;
} crbd_ctx;

/* crbdGoesUndetected: a hidden lineage born at time (age) t_start. */
static int crbd_undetected(crbd_ctx* c, double t_start, int depth)
{
    if (depth > c->max_depth) return 0;
    double duration = exponential(c->s, c->mu);
    if (duration > t_start) {
        if (bernoulli(c->s, c->rho)) return 0; /* survives and is sampled: detected */
    }
    double branch_len = duration < t_start ? duration : t_start;
    int64_t n = poisson(c->s, c->lambda * branch_len);
    if (n < 0) return 0;
    for (int64_t e = 0; e < n; ++e) { /* iter */
        if (c->events >= c->max_events) return 0;
        c->events += 1;
        double t = uniform_ab(c->s, t_start - branch_len, t_start);
        if (!crbd_undetected(c, t, depth + 1)) return 0;
    }
    return 1;
}

static int crbd_block(or_run* r, uint64_t i, int b, stream* s, int* ckpt)
{
    const double* p = r->m.p;
    *ckpt = 1;
    if (b == 0) {
        double lambda = p[3] > 0.0 ? p[3] : gamma1(s, p[1]);
        double mu = p[4] >= 0.0 ? p[4] : gamma1(s, p[2]);
        r->real[0][i] = store_p(r, lambda);
        r->real[1][i] = store_p(r, mu);
        r->lw[i] = r->lw[i] + r->corr;
        r->ints[0][i] = 1;
        return r->m.n_nodes > 1 ? 1 : (int)OR_STOP;
    }
    int node = r->ints[0][i];
    int par = r->m.parent[node];
    double lambda = r->real[0][i], mu = r->real[1][i];
    double t_p = r->m.age[par], t_c = r->m.age[node];
    double ln_p1 = -mu * (t_p - t_c);
    double ln_p2 = r->m.left[node] >= 0 ? or_log(lambda) : r->log_rho;
    crbd_ctx c = {s, lambda, mu, p[0], 0, (int)p[5], (int)p[6]};
    int64_t n = poisson(s, lambda * (t_p - t_c));
    double ln_p3 = 0.0;
    if (n < 0) {
        ln_p3 = -INFINITY;
    } else {
        for (int64_t e = 0; e < n; ++e) { /* simBranch */
            if (c.events >= c.max_events) { ln_p3 = -INFINITY; break; }
            c.events += 1;
            double t = uniform_ab(s, t_c, t_p);
            if (crbd_undetected(&c, t, 1)) {
                ln_p3 = ln_p3 + r->ln2;
            } else {
                ln_p3 = -INFINITY;
                break;
            }
        }
    }
    r->lw[i] = r->lw[i] + (ln_p1 + (ln_p2 + ln_p3));
    r->ints[0][i] = node + 1;
    return node + 1 < r->m.n_nodes ? 1 : (int)OR_STOP;
}

/* ------------------------------------------------------------------------- */
/* CRBD with static delayed sampling (Sec. 5.3 runs CRBD "with delayed        */
/* sampling"; the paper gives no derivation, this is the library's reading):  */
/* lambda ~ Gamma(k, theta) and mu ~ Gamma(k, theta) are never sampled; each  */
/* particle carries their posterior shapes and scales and every quantity that */
/* depends on a rate is drawn from, or weighted by, its predictive under the  */
/* current posterior, which is then updated by conjugacy:                     */
/*  - survival of an observed branch of length t, factor exp(-mu t):          */
/*      lw += -a_mu log(1 + th_mu t);  th_mu <- th_mu / (1 + th_mu t);         */
/*  - the speciation factor lambda at an internal node:                       */
/*      lw += log(a_l th_l);  a_l <- a_l + 1;                                  */
/*  - a count K ~ Poisson(lambda t): K from the Negative Binomial predictive  */
/*      P(K = k) = C(k + a - 1, k) p^a (1 - p)^k, p = 1 / (1 + th t),         */
/*      by inversion with one uniform (more than the event cap: -1);          */
/*      a_l <- a_l + K;  th_l <- th_l / (1 + th_l t);                          */
/*  - a lifetime d ~ Exponential(mu): the Lomax predictive by inversion,      */
/*      d = (exp(-log(u) / a_mu) - 1) / th_mu;                                 */
/*      a_mu <- a_mu + 1;  th_mu <- th_mu / (1 + th_mu d).                     */
/* Everything else (program order, caps, the detection of hidden lineages,    */
/* lw += l1 + (l2 + l3)) is as in crbd_block. The priors: p[1], p[2] are the  */
/* scales of the shape-1 Gamma priors of lambda and mu.                       */
/* Fields: real0..3 = a_l, th_l, a_mu, th_mu; int0 = node cursor.             */
/* ------------------------------------------------------------------------- */
typedef struct {
    stream* s;
    double a_l, th_l, a_mu, th_mu, rho;
    int events, max_events, max_depth;
} crbd_ds_ctx;

static int crbd_ds_undetected(crbd_ds_ctx* c, double t_start, int depth)
{
    if (depth > c->max_depth) return 0;
    double duration = lomax_draw(c->s, c->a_mu, c->th_mu);
    c->a_mu = c->a_mu + 1.0;
    c->th_mu = c->th_mu / (1.0 + c->th_mu * duration);
    if (duration > t_start) {
        if (bernoulli(c->s, c->rho)) return 0;
    }
    double branch_len = duration < t_start ? duration : t_start;
    int64_t n = neg_binomial_draw(c->s, c->a_l, c->th_l, branch_len);
    if (n < 0) return 0;
    c->a_l = c->a_l + (double)n;
    c->th_l = c->th_l / (1.0 + c->th_l * branch_len);
    for (int64_t e = 0; e < n; ++e) {
        if (c->events >= c->max_events) return 0;
        c->events += 1;
        double t = uniform_ab(c->s, t_start - branch_len, t_start);
        if (!crbd_ds_undetected(c, t, depth + 1)) return 0;
    }
    return 1;
}

static int crbd_ds_block(or_run* r, uint64_t i, int b, stream* s, int* ckpt)
{
    const double* p = r->m.p;
    *ckpt = 1;
    if (b == 0) {
        r->real[0][i] = store_p(r, 1.0);
        r->real[1][i] = store_p(r, p[1]);
        r->real[2][i] = store_p(r, 1.0);
        r->real[3][i] = store_p(r, p[2]);
        r->lw[i] = r->lw[i] + r->corr;
        r->ints[0][i] = 1;
        return r->m.n_nodes > 1 ? 1 : (int)OR_STOP;
    }
    int node = r->ints[0][i];
    int par = r->m.parent[node];
    crbd_ds_ctx c = {s, r->real[0][i], r->real[1][i], r->real[2][i], r->real[3][i], p[0], 0, (int)p[5], (int)p[6]};
    double t_p = r->m.age[par], t_c = r->m.age[node];
    double len = t_p - t_c;
    double ln_p1 = -c.a_mu * or_log(1.0 + c.th_mu * len);
    c.th_mu = c.th_mu / (1.0 + c.th_mu * len);
    double ln_p2 = r->log_rho;
    if (r->m.left[node] >= 0) {
        ln_p2 = or_log(c.a_l * c.th_l);
        c.a_l = c.a_l + 1.0;
    }
    int64_t n = neg_binomial_draw(s, c.a_l, c.th_l, len);
    double ln_p3 = 0.0;
    if (n < 0) {
        ln_p3 = -INFINITY;
    } else {
        c.a_l = c.a_l + (double)n;
        c.th_l = c.th_l / (1.0 + c.th_l * len);
        for (int64_t e = 0; e < n; ++e) {
            if (c.events >= c.max_events) { ln_p3 = -INFINITY; break; }
            c.events += 1;
            double t = uniform_ab(s, t_c, t_p);
            if (crbd_ds_undetected(&c, t, 1)) {
                ln_p3 = ln_p3 + r->ln2;
            } else {
                ln_p3 = -INFINITY;
                break;
            }
        }
    }
    r->real[0][i] = store_p(r, c.a_l);
    r->real[1][i] = store_p(r, c.th_l);
    r->real[2][i] = store_p(r, c.a_mu);
    r->real[3][i] = store_p(r, c.th_mu);
    r->lw[i] = r->lw[i] + (ln_p1 + (ln_p2 + ln_p3));
    r->ints[0][i] = node + 1;
    return node + 1 < r->m.n_nodes ? 1 : (int)OR_STOP;
}

/* ------------------------------------------------------------------------- */
/* ClaDS-style model (cladogenetic rate shifts on a CRBD skeleton):          */
/*   lambda0 ~ Gamma(1, p[1]), eps ~ U(p[2], p[3]), alpha ~ U(p[4], p[5]),    */
/*   sigma ~ Gamma(1, p[6]); mu = eps * lambda on every lineage; at every     */
/*   speciation both daughters get rate lambda * LogNormal(log alpha, sigma). */
/* Observed branches are simulated with sequential waiting times; each       */
/* hidden speciation spawns a side lineage that must die out unobserved     */
/* (weight log 2 when it does, -inf otherwise).                              */
/* p = {rho, scale_l0, eps_lo, eps_hi, alpha_lo, alpha_hi, scale_sigma,      */
/*      max events, max depth, fixed l0 (>0), fixed eps (>=0),              */
/*      fixed alpha (>0), fixed sigma (>=0)}.                                */
/* Fields: real0 = current lineage rate, real1 = eps, real2 = alpha,        */
/* real3 = sigma, int0 = node cursor, int1 = stack size; stack = pending     */
/* right-daughter rates.                                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    stream* s;
    double eps, log_alpha, sigma, rho;
    int events, max_events, max_depth;
} clads_ctx;

static int clads_side_undetected(clads_ctx* c, double t_start, double rate, int depth)
{
    if (depth > c->max_depth) return 0;
    if (c->events >= c->max_events) return 0;
    c->events += 1;
    double w = exponential(c->s, rate * (1.0 + c->eps));
    if (t_start - w <= 0.0) {
        return !bernoulli(c->s, c->rho); /* reaches the present: detected w.p. rho */
    }
    double t = t_start - w;
    if (next_uniform(c->s) < 1.0 / (1.0 + c->eps)) { /* speciation */
        double d1 = rate * lognormal(c->s, c->log_alpha, c->sigma);
        double d2 = rate * lognormal(c->s, c->log_alpha, c->sigma);
        if (!clads_side_undetected(c, t, d1, depth + 1)) return 0;
        return clads_side_undetected(c, t, d2, depth + 1);
    }
    return 1; /* extinction */
}

static int clads_block(or_run* r, uint64_t i, int b, stream* s, int* ckpt)
{
    const double* p = r->m.p;
    double* st = r->stack + i * (uint64_t)r->stack_depth;
    *ckpt = 1;
    if (b == 0) {
        double l0 = p[9] > 0.0 ? p[9] : gamma1(s, p[1]);
        double eps = p[10] >= 0.0 ? p[10] : uniform_ab(s, p[2], p[3]);
        double alpha = p[11] > 0.0 ? p[11] : uniform_ab(s, p[4], p[5]);
        double sigma = p[12] >= 0.0 ? p[12] : gamma1(s, p[6]);
        r->real[1][i] = store_p(r, eps);
        r->real[2][i] = store_p(r, alpha);
        r->real[3][i] = store_p(r, sigma);
        r->lw[i] = r->lw[i] + r->corr;
        double log_alpha = or_log(r->real[2][i]);
        double left = l0 * lognormal(s, log_alpha, r->real[3][i]);
        double right = l0 * lognormal(s, log_alpha, r->real[3][i]);
        st[0] = store_p(r, right);
        r->ints[1][i] = 1;
        r->real[0][i] = store_p(r, left);
        r->ints[0][i] = 1;
        return r->m.n_nodes > 1 ? 1 : (int)OR_STOP;
    }
    int node = r->ints[0][i];
    int par = r->m.parent[node];
    double eps = r->real[1][i];
    double log_alpha = or_log(r->real[2][i]);
    double sigma = r->real[3][i];
    clads_ctx c = {s, eps, log_alpha, sigma, p[0], 0, (int)p[7], (int)p[8]};
    double lambda = r->real[0][i];
    double t = r->m.age[par], t_c = r->m.age[node];
    double lw = r->lw[i];
    int dead = 0;
    for (;;) {
        if (c.events >= c.max_events) { dead = 1; break; }
        c.events += 1;
        double w = exponential(s, lambda);
        if (t - w <= t_c) {
            lw = lw + (-(eps * lambda) * (t - t_c));
            break;
        }
        lw = lw + (-(eps * lambda) * w);
        t = t - w;
        double cont = lambda * lognormal(s, log_alpha, sigma);
        double side = lambda * lognormal(s, log_alpha, sigma);
        if (!clads_side_undetected(&c, t, side, 1)) { dead = 1; break; }
        lw = lw + r->ln2;
        lambda = cont;
    }
    int sp = r->ints[1][i];
    if (dead) {
        lw = -INFINITY;
        /* the rest of the block still runs without random draws so the stack
         * bookkeeping stays identical across particles */
        if (r->m.left[node] >= 0) {
            st[sp] = store_p(r, lambda);
            r->ints[1][i] = sp + 1;
            r->real[0][i] = store_p(r, lambda);
        } else if (sp > 0) {
            r->real[0][i] = st[sp - 1];
            r->ints[1][i] = sp - 1;
        }
    } else if (r->m.left[node] >= 0) {
        lw = lw + or_log(lambda);
        double left = lambda * lognormal(s, log_alpha, sigma);
        double right = lambda * lognormal(s, log_alpha, sigma);
        st[sp] = store_p(r, right);
        r->ints[1][i] = sp + 1;
        r->real[0][i] = store_p(r, left);
    } else {
        lw = lw + r->log_rho;
        if (sp > 0) {
            r->real[0][i] = st[sp - 1];
            r->ints[1][i] = sp - 1;
        }
    }
    r->lw[i] = lw;
    r->ints[0][i] = node + 1;
    return node + 1 < r->m.n_nodes ? 1 : (int)OR_STOP;
}

/* ------------------------------------------------------------------------- */
/* sim: one block execution (Sec. 3.1). Returns the successor block.         */
/* ------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------- */
/* Vector-borne disease (SEIR) model of the Appendix listing: humans and     */
/* mosquitoes, susceptible / exposed / infectious / recovered counts per     */
/* day, new human cases observed as Binomial(z, rho) where z counts the      */
/* new infectious humans since the last observation. Parameters:             */
/* p = {n humans, fixed hLambda, hDelta, hGamma, mLambda, mDelta, rho (each  */
/* >= 0 fixes it, < 0 draws it from its Beta prior), fixed initial hE (>= 0),*/
/* hI (>= 0), hR (>= 0), mS (>= 0)}. Observations y[T] (-1 = missing); the   */
/* init block conditions on y_0 and day t = 1 .. T-1 on y_t (the listing's   */
/* recursion bound would read one observation past the end; this is the     */
/* reading). Fields: real0..5 = hLambda, hDelta, hGamma, mLambda, mDelta,    */
/* rho; int0..9 = hS, hE, hI, hR, mS, mE, mI, mR, z, t.                      */
/* ------------------------------------------------------------------------- */
static double seir_param(stream* s, double fixed, double a, double b)
{
    return fixed >= 0.0 ? fixed : beta_draw(s, a, b);
}

/* condition t: z accumulates new infectious humans; an observed day adds the
 * Binomial(z, rho) log-probability of y_t and restarts z. */
static void seir_condition(or_run* r, uint64_t i, int t, int64_t new_infectious)
{
    int64_t z = (int64_t)r->ints[8][i] + new_infectious;
    int64_t y = (int64_t)r->m.y[t];
    if (y != -1) {
        r->lw[i] = r->lw[i] + or_log_binomial_pmf(y, z, r->real[5][i]);
        z = 0;
    }
    r->ints[8][i] = (int32_t)z;
}

static int seir_block(or_run* r, uint64_t i, int b, stream* s, int* ckpt)
{
    const double* p = r->m.p;
    const int64_t n = (int64_t)p[0];
    *ckpt = 1;
    if (b == 0) {
        r->real[0][i] = store_p(r, seir_param(s, p[1], 1.0, 1.0));
        r->real[1][i] = store_p(r, seir_param(s, p[2], 1.0 + 2.0 / 4.4, 3.0 - 2.0 / 4.4));
        r->real[2][i] = store_p(r, seir_param(s, p[3], 1.0 + 2.0 / 4.5, 3.0 - 2.0 / 4.5));
        r->real[3][i] = store_p(r, seir_param(s, p[4], 1.0, 1.0));
        r->real[4][i] = store_p(r, seir_param(s, p[5], 1.0 + 2.0 / 6.5, 3.0 - 2.0 / 6.5));
        r->real[5][i] = store_p(r, seir_param(s, p[6], 1.0, 1.0));
        int64_t hI = p[8] >= 0.0 ? (int64_t)p[8] : 1 + poisson(s, 5.0);
        int64_t hE = p[7] >= 0.0 ? (int64_t)p[7] : poisson(s, 5.0);
        int64_t hR = p[9] >= 0.0 ? (int64_t)p[9]
                                 : (int64_t)floor(uniform_ab(s, 0.0, (double)(n - hI - hE + 1)));
        int64_t mS = p[10] >= 0.0 ? (int64_t)p[10]
                                  : (int64_t)floor((double)n * or_exp(uniform_ab(s, -1.0, 2.0) * r->ln10));
        r->ints[0][i] = (int32_t)(n - hE - hI - hR);
        r->ints[1][i] = (int32_t)hE;
        r->ints[2][i] = (int32_t)hI;
        r->ints[3][i] = (int32_t)hR;
        r->ints[4][i] = (int32_t)mS;
        r->ints[5][i] = r->ints[6][i] = r->ints[7][i] = 0;
        r->ints[8][i] = 0;
        r->ints[9][i] = 0;
        seir_condition(r, i, 0, hI); /* the initial deltas: hDeltaI = hI */
        r->ints[9][i] = 1;
        return r->m.T > 1 ? 1 : (int)OR_STOP;
    }
    const int t = r->ints[9][i];
    const double hLambda = r->real[0][i], hDelta = r->real[1][i], hGamma = r->real[2][i];
    const double mLambda = r->real[3][i], mDelta = r->real[4][i];
    const double mNu = 1.0 / 7.0, mMu = 6.0 / 7.0, mGamma = 0.0;
    int64_t hSP = r->ints[0][i], hEP = r->ints[1][i], hIP = r->ints[2][i], hRP = r->ints[3][i];
    int64_t mSP = r->ints[4][i], mEP = r->ints[5][i], mIP = r->ints[6][i], mRP = r->ints[7][i];
    /* humans */
    int64_t hN = hSP + hEP + hIP + hRP;
    int64_t hTau = binomial_draw(s, hSP, 1.0 - or_exp(-((double)mIP / (double)hN)));
    int64_t hDeltaE = binomial_draw(s, hTau, hLambda);
    int64_t hDeltaI = binomial_draw(s, hEP, hDelta);
    int64_t hDeltaR = binomial_draw(s, hIP, hGamma);
    int64_t hS = hSP - hDeltaE;
    int64_t hE = hEP + hDeltaE - hDeltaI;
    int64_t hI = hIP + hDeltaI - hDeltaR;
    int64_t hR = hRP + hDeltaR;
    /* mosquitoes */
    int64_t mTau = binomial_draw(s, mSP, 1.0 - or_exp(-((double)hIP / (double)hN)));
    int64_t mN = mSP + mEP + mIP + mRP;
    int64_t mDeltaE = binomial_draw(s, mTau, mLambda);
    int64_t mDeltaI = binomial_draw(s, mEP, mDelta);
    int64_t mDeltaR = binomial_draw(s, mIP, mGamma);
    int64_t mS = mSP - mDeltaE;
    int64_t mE = mEP + mDeltaE - mDeltaI;
    int64_t mI = mIP + mDeltaI - mDeltaR;
    int64_t mR = mRP + mDeltaR;
    mS = binomial_draw(s, mS, mMu);
    mE = binomial_draw(s, mE, mMu);
    mI = binomial_draw(s, mI, mMu);
    mR = binomial_draw(s, mR, mMu);
    int64_t mDeltaS = binomial_draw(s, mN, mNu);
    mS = mS + mDeltaS;
    r->ints[0][i] = (int32_t)hS;
    r->ints[1][i] = (int32_t)hE;
    r->ints[2][i] = (int32_t)hI;
    r->ints[3][i] = (int32_t)hR;
    r->ints[4][i] = (int32_t)mS;
    r->ints[5][i] = (int32_t)mE;
    r->ints[6][i] = (int32_t)mI;
    r->ints[7][i] = (int32_t)mR;
    seir_condition(r, i, t, hDeltaI);
    r->ints[9][i] = t + 1;
    return t + 1 < r->m.T ? 1 : (int)OR_STOP;
}

static int sim(or_run* r, uint64_t i, int b, stream* s, int* ckpt)
{
    switch (r->m.kind) {
    case OR_GEOMETRIC: return geometric_block(r, i, s, ckpt);
    case OR_LGSSM: return lgssm_block(r, i, b, s, ckpt);
    case OR_CRBD: return crbd_block(r, i, b, s, ckpt);
    case OR_SEIR: return seir_block(r, i, b, s, ckpt);
    case OR_CRBD_DS: return crbd_ds_block(r, i, b, s, ckpt);
    default: return clads_block(r, i, b, s, ckpt);
    }
}

/* ------------------------------------------------------------------------- */
/* Run setup (Alg. 1 step 1).                                                */
/* ------------------------------------------------------------------------- */
static int tree_stack_depth(const or_model* m)
{
    /* pending right daughters along the preorder walk, plus one */
    int depth = 1, cur = 1;
    for (int node = 1; node < m->n_nodes; ++node) {
        if (m->left[node] >= 0) cur += 1; else cur -= 1;
        if (cur > depth) depth = cur;
    }
    return depth + 1;
}

or_run* or_create(const or_model* m, uint64_t n, uint64_t seed)
{
    if (n == 0 || n > (1ull << 24)) return NULL;
    if (m->kind < OR_GEOMETRIC || m->kind > OR_CRBD_DS) return NULL;
    if (m->kind == OR_SEIR && (m->T < 1 || !m->y || !(m->p[0] >= 1.0 && m->p[0] <= 1e8))) return NULL;
    if (m->precision != 32 && m->precision != 64) return NULL;
    if ((m->kind == OR_CRBD || m->kind == OR_CLADS || m->kind == OR_CRBD_DS) &&
        (m->n_nodes < 1 || !m->parent || !m->age || !m->left))
        return NULL;
    if (m->kind == OR_LGSSM && (m->T < 1 || !m->y)) return NULL;
    if (!(m->ess_threshold >= 0.0 && m->ess_threshold <= 1.0)) return NULL;
    or_run* r = (or_run*)calloc(1, sizeof *r);
    r->ess_t = (uint32_t)nearbyint(m->ess_threshold * 65536.0);
    r->m = *m;
    r->n = n;
    r->seed = seed;
    r->ln2 = or_log(2.0);
    switch (m->kind) {
    case OR_GEOMETRIC: r->n_int = 1; break;
    case OR_LGSSM: r->n_real = 1; r->n_int = 1; break;
    case OR_CRBD: r->n_real = 2; r->n_int = 1; break;
    case OR_SEIR: r->n_real = 6; r->n_int = 10; break;
    case OR_CRBD_DS: r->n_real = 4; r->n_int = 1; break;
    default: r->n_real = 4; r->n_int = 2; break;
    }
    r->ln10 = or_log(10.0);
    r->blk = (uint8_t*)calloc(n, 1);             /* a_n = b0 */
    r->lw = (double*)calloc(n, sizeof(double));  /* log weights 0 */
    r->anc = (uint32_t*)calloc(n, sizeof(uint32_t));
    for (int f = 0; f < r->n_real; ++f) r->real[f] = (double*)calloc(n, sizeof(double));
    for (int f = 0; f < r->n_int; ++f) r->ints[f] = (int32_t*)calloc(n, sizeof(int32_t));
    for (uint64_t i = 0; i < n; ++i) r->anc[i] = (uint32_t)i;
    if (m->kind == OR_GEOMETRIC) r->log_w = or_log(m->p[1]);
    if (m->kind == OR_LGSSM) {
        r->obs_var = m->p[3] * m->p[3];
        r->obs_c = -0.5 * or_log(OR_TWO_PI * r->obs_var);
    }
    if (m->kind == OR_CRBD || m->kind == OR_CLADS || m->kind == OR_CRBD_DS) {
        r->tips = (m->n_nodes + 1) / 2;
        r->log_rho = or_log(m->p[0]);
        double log_fact = 0.0;
        for (int k = 2; k <= r->tips; ++k) log_fact = log_fact + or_log((double)k);
        r->corr = (double)(r->tips - 1) * r->ln2 - log_fact;
    }
    if (m->kind == OR_CLADS) {
        r->stack_depth = tree_stack_depth(m);
        r->stack = (double*)calloc(n * (uint64_t)r->stack_depth, sizeof(double));
    }
    return r;
}

void or_destroy(or_run* r)
{
    if (!r) return;
    free(r->blk); free(r->lw); free(r->anc); free(r->stack);
    for (int f = 0; f < OR_MAX_FIELDS; ++f) { free(r->real[f]); free(r->ints[f]); }
    free(r);
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 step 2: every particle not at b_stop runs blocks until a           */
/* checkpoint or b_stop. A particle at b_stop does nothing (the fixpoint).   */
/* ------------------------------------------------------------------------- */
/* Particle i's blocks for this round, drawing from the stream of slot `slot`. */
static void propagate_one(or_run* r, uint64_t i, uint32_t slot)
{
    if (r->blk[i] == OR_STOP) return;
    stream s = {r->seed, slot, r->round, OR_TAG_PROPAGATE, 0};
    int b = r->blk[i];
    for (;;) {
        int ckpt = 0;
        b = sim(r, i, b, &s, &ckpt);
        r->block_steps += 1;
        if (ckpt || b == (int)OR_STOP) break;
    }
    r->blk[i] = (uint8_t)b;
}

int32_t or_step(or_run* r)
{
    if (r->status != OR_OK) return r->status;
    for (uint64_t i = 0; i < r->n; ++i) propagate_one(r, i, (uint32_t)i);
    return OR_OK;
}

/* One particle's propagation in isolation (for checking sampled particles of a
 * large run): the particle sits in slot `slot` of round `round` with the given
 * block, state and zero log-weight. Real fields are read and written in FP64
 * (already rounded to the storage precision); ints and the ClaDS stack follow
 * the field order of or_read. */
int32_t or_propagate_particle(const or_model* m, uint64_t seed, uint32_t slot, uint32_t round,
                              uint8_t* blk, double* lw, double* reals, int32_t* ints, double* stack)
{
    or_run* r = or_create(m, 1, seed);
    if (!r) return OR_ERR_INVALID;
    r->round = round;
    r->blk[0] = *blk;
    for (int f = 0; f < r->n_real; ++f) r->real[f][0] = reals[f];
    for (int f = 0; f < r->n_int; ++f) r->ints[f][0] = ints[f];
    if (r->stack && stack) memcpy(r->stack, stack, (size_t)r->stack_depth * sizeof(double));
    propagate_one(r, 0, slot);
    *blk = r->blk[0];
    *lw = r->lw[0];
    for (int f = 0; f < r->n_real; ++f) reals[f] = r->real[f][0];
    for (int f = 0; f < r->n_int; ++f) ints[f] = r->ints[f][0];
    if (r->stack && stack) memcpy(stack, r->stack, (size_t)r->stack_depth * sizeof(double));
    or_destroy(r);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Systematic resampling on quantised weights.                               */
/* ------------------------------------------------------------------------- */
static int grid_bits(uint64_t n)
{
    int ceil_log2 = 0;
    while ((1ull << ceil_log2) < n) ceil_log2 += 1;
    int g = 53 - ceil_log2;
    return g < 32 ? g : 32;
}

/* Systematic ancestors from the inclusive cumulative grid weights Q (Q[n-1] > 0)
 * and the round's uniform word U: output j sits at (j + U/2^32)/N of the total
 * mass and takes the first particle whose cumulative mass lies beyond it,
 *   a_j = min{ i : N Q_i 2^32 > (j 2^32 + U) Q_{N-1} }   (exact 128-bit). */
void or_ancestors(const uint64_t* Q, uint64_t n, uint32_t U, uint32_t* anc)
{
    unsigned __int128 total = (unsigned __int128)Q[n - 1];
    uint64_t i = 0;
    for (uint64_t j = 0; j < n; ++j) {
        unsigned __int128 rhs = (((unsigned __int128)j << 32) + U) * total;
        while (i < n && !((unsigned __int128)n * Q[i] * ((unsigned __int128)1 << 32) > rhs)) i += 1;
        anc[j] = (uint32_t)i;
    }
}

/* Log Z increment and ancestors for one resampling step.
 *  M = max lw, S = sum exp(lw - M), increment = (M + log S) - log N.
 *  q_n = rint(exp(lw_n - M) 2^G) grid units, Q_n = q_0 + ... + q_n (exact).
 *  One uniform word U per round (tag 1). Offspring positions (j + U/2^32)/N of
 *  the total mass: a_j = min{ i : N Q_i 2^32 > (j 2^32 + U) Q_{N-1} }. */
static int32_t systematic_core(const double* lw, uint64_t n, uint64_t seed, uint32_t round,
                               int do_ancestors, uint32_t* anc, double* inc, uint64_t* qtot_out)
{
    double M = -INFINITY;
    for (uint64_t i = 0; i < n; ++i) {
        if (lw[i] != lw[i]) return OR_ERR_NAN;
        if (lw[i] > M) M = lw[i];
    }
    if (M == -INFINITY) { *inc = -INFINITY; return OR_DEGENERATE; }
    if (M == INFINITY) return OR_ERR_NAN;
    double* e = (double*)malloc(n * sizeof(double));
    double S = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        e[i] = or_exp(lw[i] - M);
        S = S + e[i];
    }
    *inc = (M + or_log(S)) - or_log((double)n);
    if (!do_ancestors) { free(e); return OR_OK; }
    int G = grid_bits(n);
    uint64_t* Q = (uint64_t*)malloc(n * sizeof(uint64_t));
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t q = (uint64_t)nearbyint(ldexp(e[i], G));
        acc += q;
        Q[i] = acc;
    }
    *qtot_out = acc;
    uint32_t U = or_word(seed, 0, 0, round, OR_TAG_RESAMPLE);
    or_ancestors(Q, n, U, anc);
    free(Q);
    free(e);
    return OR_OK;
}

int32_t or_systematic(const double* lw, uint64_t n, uint64_t seed, uint32_t round,
                      uint32_t* anc, double* logz_increment, uint64_t* qtot_units)
{
    uint64_t qtot = 0;
    int32_t st = systematic_core(lw, n, seed, round, 1, anc, logz_increment, &qtot);
    if (qtot_units) *qtot_units = qtot;
    return st;
}

/* ------------------------------------------------------------------------- */
/* ESS-triggered resampling. Sec. 3.3 lists adaptive resampling on the        */
/* effective sample size among RootPPL's features without fixing the rule;   */
/* the reading here: the ESS is taken on the quantised weights of the        */
/* resampling step, q_n = rint(exp(lw_n - M) 2^G),                            */
/*   ESS = (sum q)^2 / sum q^2,                                               */
/* and a round resamples iff ESS < t N / 2^16, t = rint(threshold 2^16),      */
/* decided exactly in integers: 2^16 (sum q)^2 < t N sum q^2 (both sides are  */
/* below 2^126 because N 2^G <= 2^53). t = 0 resamples every round.           */
/* ------------------------------------------------------------------------- */
static int ess_rule(const double* lw, uint64_t n, uint32_t t)
{
    if (t == 0) return 1;
    double M = -INFINITY;
    for (uint64_t i = 0; i < n; ++i) {
        if (lw[i] != lw[i] || lw[i] == INFINITY) return 1; /* the resampling step reports it */
        if (lw[i] > M) M = lw[i];
    }
    if (M == -INFINITY) return 1;
    int G = grid_bits(n);
    uint64_t s1 = 0;
    unsigned __int128 s2 = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t q = (uint64_t)nearbyint(ldexp(or_exp(lw[i] - M), G));
        s1 += q;
        s2 += (unsigned __int128)q * q;
    }
    unsigned __int128 lhs = (unsigned __int128)s1 * s1 * 65536u;
    unsigned __int128 rhs = (unsigned __int128)t * n * s2;
    return lhs < rhs;
}

int32_t or_ess_resamples(const double* lw, uint64_t n, double threshold)
{
    if (!(threshold >= 0.0 && threshold <= 1.0) || n == 0) return -1;
    return ess_rule(lw, n, (uint32_t)nearbyint(threshold * 65536.0));
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 step 3 plus the log Z update (Sec. 3.3). When every particle is at */
/* b_stop the run ends: the last weights still enter log Z, no resampling.   */
/* ------------------------------------------------------------------------- */
int32_t or_resample(or_run* r)
{
    if (r->status != OR_OK) return r->status;
    int any_active = 0;
    for (uint64_t i = 0; i < r->n; ++i) any_active |= (r->blk[i] != OR_STOP);
    /* While particles are still active, the ESS rule may keep the weights:
     * no resampling, identity ancestors, log Z unchanged, weights carried. */
    int resample = any_active && ess_rule(r->lw, r->n, r->ess_t);
    double inc = 0.0;
    uint64_t qtot = 0;
    int32_t st = systematic_core(r->lw, r->n, r->seed, r->round, resample, r->anc, &inc, &qtot);
    if (st == OR_DEGENERATE) { r->log_z = -INFINITY; r->status = st; return st; }
    if (st != OR_OK) { r->status = st; return st; }
    if (!any_active) { r->log_z = r->log_z + inc; r->status = OR_FINISHED; return OR_FINISHED; }
    if (!resample) {
        for (uint64_t j = 0; j < r->n; ++j) r->anc[j] = (uint32_t)j;
        r->round += 1;
        return OR_OK;
    }
    r->log_z = r->log_z + inc;
    r->resamples += 1;
    /* (s'_n, b'_n) = (s_{a_n}, b_{a_n}); weights reset. */
    uint64_t n = r->n;
    uint8_t* nb = (uint8_t*)malloc(n);
    for (uint64_t j = 0; j < n; ++j) nb[j] = r->blk[r->anc[j]];
    memcpy(r->blk, nb, n);
    free(nb);
    double* tmp = (double*)malloc(n * sizeof(double));
    for (int f = 0; f < r->n_real; ++f) {
        for (uint64_t j = 0; j < n; ++j) tmp[j] = r->real[f][r->anc[j]];
        memcpy(r->real[f], tmp, n * sizeof(double));
    }
    free(tmp);
    int32_t* itmp = (int32_t*)malloc(n * sizeof(int32_t));
    for (int f = 0; f < r->n_int; ++f) {
        for (uint64_t j = 0; j < n; ++j) itmp[j] = r->ints[f][r->anc[j]];
        memcpy(r->ints[f], itmp, n * sizeof(int32_t));
    }
    free(itmp);
    if (r->stack) {
        uint64_t d = (uint64_t)r->stack_depth;
        double* st2 = (double*)malloc(n * d * sizeof(double));
        for (uint64_t j = 0; j < n; ++j) memcpy(st2 + j * d, r->stack + (uint64_t)r->anc[j] * d, d * sizeof(double));
        memcpy(r->stack, st2, n * d * sizeof(double));
        free(st2);
    }
    for (uint64_t j = 0; j < n; ++j) r->lw[j] = 0.0;
    r->round += 1;
    return OR_OK;
}

int32_t or_run_to_end(or_run* r)
{
    while (r->status == OR_OK) {
        or_step(r);
        or_resample(r);
    }
    return r->status;
}

double or_log_z(const or_run* r) { return r->log_z; }
int32_t or_status(const or_run* r) { return r->status; }
uint32_t or_round(const or_run* r) { return r->round; }
uint64_t or_block_steps(const or_run* r) { return r->block_steps; }
uint32_t or_resamples(const or_run* r) { return r->resamples; }
int32_t or_max_stack(const or_run* r) { return r->stack_depth; }

/* Copy out per-particle arrays; real fields come out in the storage precision. */
int32_t or_read(const or_run* r, int32_t what, void* dst)
{
    uint64_t n = r->n;
    if (what == OR_READ_BLK) { memcpy(dst, r->blk, n); return OR_OK; }
    if (what == OR_READ_LW) { memcpy(dst, r->lw, n * sizeof(double)); return OR_OK; }
    if (what == OR_READ_ANC) { memcpy(dst, r->anc, n * sizeof(uint32_t)); return OR_OK; }
    int f = what - OR_READ_FIELD0;
    if (f >= 0 && f < r->n_real) {
        if (r->m.precision == 32) {
            float* o = (float*)dst;
            for (uint64_t i = 0; i < n; ++i) o[i] = (float)r->real[f][i];
        } else {
            memcpy(dst, r->real[f], n * sizeof(double));
        }
        return OR_OK;
    }
    f -= r->n_real;
    if (f >= 0 && f < r->n_int) { memcpy(dst, r->ints[f], n * sizeof(int32_t)); return OR_OK; }
    f -= r->n_int;
    if (f == 0 && r->stack) {
        uint64_t cnt = n * (uint64_t)r->stack_depth;
        if (r->m.precision == 32) {
            float* o = (float*)dst;
            for (uint64_t i = 0; i < cnt; ++i) o[i] = (float)r->stack[i];
        } else {
            memcpy(dst, r->stack, cnt * sizeof(double));
        }
        return OR_OK;
    }
    return OR_ERR_INVALID;
}
