// Device primitives for the particle blocks: counter-based random words,
// uniforms, the pinned FP64 elementary functions and the samplers.
//
// Every function here rounds exactly once per written operation (the library
// is compiled with -ffp-contract=off; fused multiply-adds are explicit), so a
// block computes the same bits wherever it runs. The pinned algorithms are the
// library's reading of what the paper leaves open: the paper's engine draws
// per-thread random numbers (Sec. 3.3) and its listings use exp, log,
// Exponential, Poisson, Uniform, Bernoulli and Gamma draws (Appendix B).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcfg {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c; on the device one three-input bit operation (truth table 0x96)
// in place of two xors.
__host__ __device__ inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

__host__ __device__ inline Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Words4{c0, c1, c2, c3};
}

enum : uint32_t { kTagPropagate = 0, kTagResample = 1 };

// One particle's words for one round, drawn in program order. Word k is lane
// k%4 of the Philox block with counter {k/4, particle, round, tag}. The block
// is consumed as a shift register (always lane 0 next), so every register
// index is static and the buffer never lands in scratch memory.
struct Stream {
    uint32_t key0, key1, particle, round, tag;
    uint32_t k;
    Words4 buf;

    __device__ inline void start(uint64_t seed, uint32_t p, uint32_t r, uint32_t t)
    {
        key0 = (uint32_t)seed;
        key1 = (uint32_t)(seed >> 32);
        particle = p;
        round = r;
        tag = t;
        k = 0;
    }

    __device__ inline uint32_t next()
    {
        if ((k & 3u) == 0u) buf = philox10(k >> 2, particle, round, tag, key0, key1);
        k += 1u;
        const uint32_t w = buf.w0;
        buf.w0 = buf.w1;
        buf.w1 = buf.w2;
        buf.w2 = buf.w3;
        return w;
    }

    __device__ inline double uniform() { return word_to_uniform(next()); }

    __host__ __device__ static inline double word_to_uniform(uint32_t w)
    {
        // (2w + 1) 2^-33: exact, strictly inside (0, 1)
        return ((double)w * 2.0 + 1.0) * 0x1p-33;
    }
};

// ---------------------------------------------------------------------------
// Pinned FP64 elementary functions.
// ---------------------------------------------------------------------------
namespace fn {

// ln 2 split as a 24-bit head (exact products with small integers) and tail.
constexpr double kLn2Head = 0.693147182464599609375;
constexpr double kLn2Tail = -1.904654299957767878541823431924e-9;
constexpr double kLog2e = 1.442695040888963407359924681001892137427;
constexpr double kRoot2 = 1.41421356237309504880168872420969807857;
constexpr double kTau = 6.283185307179586476925286766559005768394;   // 2 pi

// a * b + c rounded once, with the constant c read from scalar registers: the
// compiler's own form of a polynomial step first copies c into the vector
// registers it accumulates in (two extra vector moves per step). Same operation
// and rounding as __builtin_fma.
__device__ inline double fma_sc(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// a * b + c rounded once, with the constant b read from scalar registers.
__device__ inline double fma_vsv(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// One polynomial step. kScalarCoef: the coefficient is read from scalar
// registers (fma_sc), which keeps it out of the vector register file and the
// vector instruction stream - the better placement where many wavefronts share
// each SIMD. Otherwise the compiler places it (vector registers, hoisted where
// registers allow), which is faster for a lone long chain of dependent steps
// with little else resident. Same value either way.
template <bool kScalarCoef>
__device__ inline double coef_fma(double a, double b, double c)
{
    if constexpr (kScalarCoef) return fma_sc(a, b, c);
    else return __builtin_fma(a, b, c);
}

// a / b correctly rounded, for operands kept in range by the caller: 2^-900 <
// |b| < 2^900, and a = 0 or 2^-900 < |a| < 2^900, with a normal quotient. The
// reciprocal estimate is refined by two Newton steps and the quotient corrected
// once with its exact residual: the steps of the compiler's IEEE division,
// without the operand scaling and special-case fix-up that this range never
// takes (three instructions fewer, same bits).
__device__ inline double div_in_range(double a, double b)
{
    double y = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = a * y;
    const double r = __builtin_fma(-b, q, a);
    return __builtin_fma(r, y, q);
}

__device__ inline double two_to(int n)   // 2^n, -1022 <= n <= 1023
{
    return __longlong_as_double((long long)(n + 1023) << 52);
}

// exp: x = n ln2 + r with n = rint(x log2 e) and r reduced in two steps
// (head, tail); e^r from its degree-13 Taylor polynomial (Horner, fma);
// result scaled by 2^n. Below -708 the result is flushed to +0, above 709 it
// is +inf.
template <bool kSc = true>
__device__ inline double exp(double x)
{
    if (x != x) return x;
    if (x > 709.0) return __builtin_huge_val();
    if (x < -708.0) return 0.0;
    const double n = __builtin_rint(x * kLog2e);
    const double r = (x - n * kLn2Head) - n * kLn2Tail;
    double p = 1.0 / 6227020800.0;
    p = coef_fma<kSc>(p, r, 1.0 / 479001600.0);
    p = coef_fma<kSc>(p, r, 1.0 / 39916800.0);
    p = coef_fma<kSc>(p, r, 1.0 / 3628800.0);
    p = coef_fma<kSc>(p, r, 1.0 / 362880.0);
    p = coef_fma<kSc>(p, r, 1.0 / 40320.0);
    p = coef_fma<kSc>(p, r, 1.0 / 5040.0);
    p = coef_fma<kSc>(p, r, 1.0 / 720.0);
    p = coef_fma<kSc>(p, r, 1.0 / 120.0);
    p = coef_fma<kSc>(p, r, 1.0 / 24.0);
    p = coef_fma<kSc>(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return p * two_to((int)n);
}

// log: x = 2^k m, m in [sqrt(2)/2, sqrt(2)); with f = m - 1 and s = f / (2 + f),
// log m = 2 atanh s = 2s + 2s * z * R(z), z = s^2, R(z) = sum_{j<10} z^j / (2j + 3);
// log x = k ln2_head + (k ln2_tail + log m).
template <bool kSc = true>
__device__ inline double log(double x)
{
    int k = 0;
    // one class test (positive normal: mask bit 8) keeps the special cases off
    // the common path
    if (!__builtin_amdgcn_class(x, 0x100)) {
        if (x != x) return x;
        if (x < 0.0) return __builtin_nan("");
        if (x == 0.0) return -__builtin_huge_val();
        if (x == __builtin_huge_val()) return x;
        x = x * 0x1p54;  // positive subnormal
        k = -54;
    }
    const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    k += (int)((bits >> 52) & 0x7ffull) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > kRoot2) {
        m = m * 0.5;
        k += 1;
    }
    const double f = m - 1.0;
    const double s = div_in_range(f, 2.0 + f);  // |f| < 0.42, 2 + f in [1.7, 2.5)
    const double z = s * s;
    double R = 1.0 / 21.0;
    R = coef_fma<kSc>(R, z, 1.0 / 19.0);
    R = coef_fma<kSc>(R, z, 1.0 / 17.0);
    R = coef_fma<kSc>(R, z, 1.0 / 15.0);
    R = coef_fma<kSc>(R, z, 1.0 / 13.0);
    R = coef_fma<kSc>(R, z, 1.0 / 11.0);
    R = coef_fma<kSc>(R, z, 1.0 / 9.0);
    R = coef_fma<kSc>(R, z, 1.0 / 7.0);
    R = coef_fma<kSc>(R, z, 1.0 / 5.0);
    R = coef_fma<kSc>(R, z, 1.0 / 3.0);
    const double s2 = 2.0 * s;
    const double log_m = __builtin_fma(s2, z * R, s2);
    const double kd = (double)k;
    return kd * kLn2Head + (kd * kLn2Tail + log_m);
}

// cos(2 pi u): quadrant q = rint(4u); t = u - q/4 (exact) in [-1/8, 1/8];
// theta = 2 pi t; sin and cos of theta from their Taylor series in theta^2.
template <bool kSc = true>
__device__ inline double cos2pi(double u)
{
    const double q = __builtin_rint(4.0 * u);
    const double t = u - q * 0.25;
    const double th = t * kTau;
    const double z = th * th;
    double S = 1.0 / 355687428096000.0;
    S = coef_fma<kSc>(S, z, -1.0 / 1307674368000.0);
    S = coef_fma<kSc>(S, z, 1.0 / 6227020800.0);
    S = coef_fma<kSc>(S, z, -1.0 / 39916800.0);
    S = coef_fma<kSc>(S, z, 1.0 / 362880.0);
    S = coef_fma<kSc>(S, z, -1.0 / 5040.0);
    S = coef_fma<kSc>(S, z, 1.0 / 120.0);
    S = coef_fma<kSc>(S, z, -1.0 / 6.0);
    S = __builtin_fma(S, z, 1.0);
    const double sn = th * S;
    double C = -1.0 / 6402373705728000.0;
    C = coef_fma<kSc>(C, z, 1.0 / 20922789888000.0);
    C = coef_fma<kSc>(C, z, -1.0 / 87178291200.0);
    C = coef_fma<kSc>(C, z, 1.0 / 479001600.0);
    C = coef_fma<kSc>(C, z, -1.0 / 3628800.0);
    C = coef_fma<kSc>(C, z, 1.0 / 40320.0);
    C = coef_fma<kSc>(C, z, -1.0 / 720.0);
    C = coef_fma<kSc>(C, z, 1.0 / 24.0);
    C = __builtin_fma(C, z, -0.5);
    C = __builtin_fma(C, z, 1.0);
    const int quadrant = ((int)q) & 3;
    double out = C;
    out = (quadrant == 1) ? -sn : out;
    out = (quadrant == 2) ? -C : out;
    out = (quadrant == 3) ? sn : out;
    return out;
}

// Correctly rounded square root.
__device__ inline double sqrt(double x) { return __builtin_sqrt(x); }

constexpr double kEventCap = 10000.0;
constexpr int kMaxInversionSteps = 10000;

}  // namespace fn

// ---------------------------------------------------------------------------
// Samplers.
// ---------------------------------------------------------------------------
template <bool kSc = true>
__device__ inline double draw_exponential(Stream& s, double rate) { return -fn::log<kSc>(s.uniform()) / rate; }
template <bool kSc = true>
__device__ inline double draw_gamma1(Stream& s, double scale) { return -scale * fn::log<kSc>(s.uniform()); }
__device__ inline double draw_uniform(Stream& s, double a, double b) { return a + (b - a) * s.uniform(); }
__device__ inline bool draw_bernoulli(Stream& s, double p) { return s.uniform() < p; }

// Box-Muller, cosine branch: sqrt(-2 log u1) cos(2 pi u2).
template <bool kSc = true>
__device__ inline double normal_from(double u1, double u2)
{
    const double radius = fn::sqrt(-2.0 * fn::log<kSc>(u1));
    return radius * fn::cos2pi<kSc>(u2);
}

template <bool kSc = true>
__device__ inline double draw_normal(Stream& s)
{
    const double u1 = s.uniform();
    const double u2 = s.uniform();
    return normal_from<kSc>(u1, u2);
}

template <bool kSc = true>
__device__ inline double draw_lognormal(Stream& s, double mu_ln, double sigma)
{
    const double z = draw_normal<kSc>(s);
    return fn::exp<kSc>(mu_ln + sigma * z);
}

// Poisson(m): inversion of the CDF, with m split into ceil(m/32) equal chunks
// (one uniform per chunk; the chunk counts add up). Returns -1 when m exceeds
// the event cap or is not a number.
__device__ inline int draw_poisson(Stream& s, double m)
{
    if (!(m >= 0.0) || m > fn::kEventCap) return -1;
    if (m == 0.0) return 0;
    const int chunks = (int)__builtin_ceil(m / 32.0);
    // a division by 1 is exact: with one chunk (m <= 32, nearly every draw)
    // the FP64 division is skipped
    const double mc = chunks == 1 ? m : m / (double)chunks;
    const double p0 = fn::exp(-mc);
    int total = 0;
    for (int c = 0; c < chunks; ++c) {
        const double u = s.uniform();
        double p = p0;
        double F = p;
        int k = 0;
        while (u > F && k < fn::kMaxInversionSteps) {
            k += 1;
            // p * mc stays above 2^-80 before the inverted CDF passes u (mc <= 32,
            // u <= 1 - 2^-33) and 1 <= k <= 10^4: inside div_in_range's range
            p = fn::div_in_range(p * mc, (double)k);
            F = F + p;
        }
        total += k;
    }
    return total;
}

// ---------------------------------------------------------------------------
// Samplers of the vector-borne disease model. The paper names the
// distributions, not the algorithms; the pinned readings:
//  - log k!: the sum of log i for k < 16, else the Stirling series in
//    x = k + 1 up to the x^-7 term;
//  - Gamma(a, 1), a >= 1: Marsaglia and Tsang (2000) without the squeeze;
//  - Beta(a, b) = X / (X + Y) with X ~ Gamma(a), Y ~ Gamma(b);
//  - Binomial(n, p): 0 for n = 0 or p = 0 and n for p = 1 (no draw);
//    n - Binomial(n, 1 - p) for p > 1/2; inversion by sequential search when
//    n p < 10; otherwise Hoermann's (1993) transformed rejection with squeeze
//    (BTRS), two uniforms per try.
// Rejection loops stop after kMaxTries tries (probability below 1e-100) and
// return the stated fallback.
// ---------------------------------------------------------------------------
constexpr int kMaxTries = 256;

__device__ __forceinline__ double log_factorial(long long k)
{
    if (k < 2) return 0.0;
    if (k < 16) {
        // log i for i < 16 are compile-time constants (the compiler folds the
        // compiler-placed form of log on constant arguments); they are added
        // in order, each times 1 (i <= k) or 0 (adds nothing), with the
        // constant read from scalar registers.
        double s = 0.0;
#pragma unroll
        for (int i = 2; i < 16; ++i) s = fn::fma_vsv(i <= k ? 1.0 : 0.0, fn::log<false>((double)i), s);
        return s;
    }
    const double x = (double)(k + 1);
    const double x2 = x * x;
    // x >= 17: every quotient is inside div_in_range's range
    const double series = fn::div_in_range(
        1.0 / 12.0 - fn::div_in_range(1.0 / 360.0 - fn::div_in_range(1.0 / 1260.0 - fn::div_in_range(1.0, 1680.0 * x2), x2), x2),
        x);
    return ((x - 0.5) * fn::log(x) - x) + (0.5 * fn::log<false>(fn::kTau) + series);  // a folded constant
}

// log k! - [(k + 1/2) log(k + 1) - (k + 1) + log(2 pi) / 2]
__device__ inline double stirling_tail(long long k)
{
    const double x = (double)(k + 1);
    return log_factorial(k) - ((((double)k + 0.5) * fn::log(x) - x) + 0.5 * fn::log<false>(fn::kTau));
}

__device__ inline double draw_gamma(Stream& s, double a)
{
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / fn::sqrt(9.0 * d);
    for (int it = 0; it < kMaxTries; ++it) {
        const double z = draw_normal(s);
        const double w = 1.0 + c * z;
        if (w <= 0.0) continue;
        const double v = w * w * w;
        const double u = s.uniform();
        if (fn::log(u) < 0.5 * z * z + d - d * v + d * fn::log(v)) return d * v;
    }
    return d;
}

__device__ inline double draw_beta(Stream& s, double a, double b)
{
    const double x = draw_gamma(s, a);
    const double y = draw_gamma(s, b);
    return x / (x + y);
}

__device__ inline long long binomial_small(Stream& s, long long n, double p)
{
    const double q = 1.0 - p;
    double pk = fn::exp((double)n * fn::log(q));
    const double ratio = p / q;
    double u = s.uniform();
    long long k = 0;
    while (u > pk && k < n) {
        u = u - pk;
        k += 1;
        pk = pk * (fn::div_in_range((double)(n - k + 1), (double)k) * ratio);
    }
    return k;
}

__device__ inline long long binomial_btrs(Stream& s, long long n, double p)
{
    const double q = 1.0 - p;
    const double spq = fn::sqrt((double)n * p * q);
    const double b = 1.15 + 2.53 * spq;
    const double a = -0.0873 + 0.0248 * b + 0.01 * p;
    const double c = (double)n * p + 0.5;
    const double v_r = 0.92 - fn::div_in_range(4.2, b);
    const double r = fn::div_in_range(p, q);
    const double alpha = (2.83 + fn::div_in_range(5.1, b)) * spq;
    const long long m = (long long)__builtin_floor((double)(n + 1) * p);
    const double h = ((double)m + 0.5) * fn::log(fn::div_in_range((double)m + 1.0, r * (double)(n - m + 1))) +
                     (stirling_tail(m) + stirling_tail(n - m));
    for (int it = 0; it < kMaxTries; ++it) {
        const double u = s.uniform() - 0.5;
        const double v = s.uniform();
        const double us = 0.5 - __builtin_fabs(u);
        const double kf = __builtin_floor((fn::div_in_range(2.0 * a, us) + b) * u + c);
        if (us >= 0.07 && v <= v_r) return (long long)kf;
        if (kf < 0.0 || kf > (double)n) continue;
        const long long k = (long long)kf;
        const double lv = fn::log(fn::div_in_range(v * alpha, fn::div_in_range(a, us * us) + b));
        const double bound = h + ((double)(n + 1) * fn::log(fn::div_in_range((double)(n - m + 1), (double)(n - k + 1))) +
                                  ((double)k + 0.5) * fn::log(fn::div_in_range(r * (double)(n - k + 1), (double)k + 1.0))) -
                             (stirling_tail(k) + stirling_tail(n - k));
        if (lv <= bound) return k;
    }
    return (long long)__builtin_floor(c);
}

__device__ inline long long draw_binomial(Stream& s, long long n, double p)
{
    if (n <= 0 || !(p > 0.0)) return 0;
    if (p >= 1.0) return n;
    const bool flip = p > 0.5;
    const double pp = flip ? 1.0 - p : p;
    const long long k = (double)n * pp < 10.0 ? binomial_small(s, n, pp) : binomial_btrs(s, n, pp);
    return flip ? n - k : k;
}

// Delayed sampling under Gamma(a, th) posteriors (shape, scale):
// the Negative Binomial predictive of a Poisson(rate t) count, by inversion
// (-1 beyond the event cap), and the Lomax predictive of an
// Exponential(rate) lifetime, by inversion.
__device__ inline long long draw_neg_binomial(Stream& s, double a, double th, double t)
{
    const double lq = fn::log(1.0 + th * t);
    double pk = fn::exp(-a * lq);
    const double q = th * t / (1.0 + th * t);
    double u = s.uniform();
    long long k = 0;
    while (u > pk) {
        if (k >= fn::kMaxInversionSteps) return -1;
        u = u - pk;
        k += 1;
        pk = pk * (((double)(k - 1) + a) / (double)k * q);
    }
    return k;
}

__device__ inline double draw_lomax(Stream& s, double a, double th)
{
    const double u = s.uniform();
    return (fn::exp(-fn::log(u) / a) - 1.0) / th;
}

// log of the Binomial(z, p) probability of y, with 0 log 0 = 0.
__device__ __forceinline__ double log_binomial_pmf(long long y, long long z, double p)
{
    if (y < 0 || y > z) return -__builtin_huge_val();
    double lw = log_factorial(z) - (log_factorial(y) + log_factorial(z - y));
    if (y > 0) lw = lw + (double)y * fn::log(p);
    if (z - y > 0) lw = lw + (double)(z - y) * fn::log(1.0 - p);
    return lw;
}

}  // namespace pcfg
