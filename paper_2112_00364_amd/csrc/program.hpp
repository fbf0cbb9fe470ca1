// Compiled programs (Sec. 4): bytecode of PCFG blocks produced by the host
// compiler (Algorithm 2 for the block split, explicit stack frames of
// Sec. 4.1), its opcodes, and the samplers and observation densities the
// bytecode calls. The interpreter loop itself is in kernels.hip; the
// instruction set is documented in include/pcfgsmc.h.
#pragma once

#include "models.hpp"

namespace pcfg {

enum ProgOp : uint32_t {
    kOpFrame = 1, kOpConst = 2, kOpImm = 3, kOpMov = 4, kOpLdf = 5, kOpStf = 6,
    kOpAdd = 7, kOpSub = 8, kOpMul = 9, kOpDiv = 10, kOpLt = 11, kOpLe = 12, kOpEq = 13, kOpNe = 14,
    kOpNeg = 15, kOpNot = 16, kOpLog = 17, kOpExp = 18, kOpSqrt = 19, kOpFloor = 20,
    kOpData = 21, kOpLen = 22, kOpSample = 23, kOpObserve = 24, kOpWeight = 25,
    kOpJz = 26, kOpJmp = 27, kOpCallFrame = 28, kOpStn = 29, kOpAddr = 30, kOpPush = 31,
    kOpStret = 32, kOpGoto = 33, kOpCkpt = 34, kOpJret = 35, kOpFault = 36,
    kOpCount = 37
};

enum ProgDist : uint32_t {
    kDistUniform = 0, kDistNormal = 1, kDistExponential = 2, kDistGamma = 3, kDistBeta = 4,
    kDistBernoulli = 5, kDistPoisson = 6, kDistBinomial = 7, kDistCount = 8
};

constexpr int kProgRegs = 16;
constexpr uint32_t kProgMaxBlocks = 254;
constexpr uint32_t kProgMaxCode = 1u << 20;
constexpr uint32_t kProgMaxStack = 4096;
// Instructions one particle may execute in one round; beyond it the particle
// faults. Bounds the work of a launch whatever the program does.
constexpr uint32_t kProgInstrBudget = 1u << 20;
constexpr double kHalfLog2Pi = 0.918938533204672741780329736406;
constexpr double kCountLimit = 2147483648.0;

__device__ inline bool is_count(double v) { return v >= 0.0 && v < kCountLimit && v == __builtin_floor(v); }

// One draw; fault = true (value 0) for arguments outside the sampler's domain.
__device__ inline double prog_draw(uint32_t dist, double a, double b, Stream& s, bool& fault)
{
    switch (dist) {
    case kDistUniform: return draw_uniform(s, a, b);
    case kDistNormal: return a + b * draw_normal(s);
    case kDistExponential: return draw_exponential(s, a);
    case kDistGamma:
        if (!(a >= 1.0)) break;
        return b * draw_gamma(s, a);
    case kDistBeta:
        if (!(a >= 1.0 && b >= 1.0)) break;
        return draw_beta(s, a, b);
    case kDistBernoulli: return draw_bernoulli(s, a) ? 1.0 : 0.0;
    case kDistPoisson: {
        const int c = draw_poisson(s, a);
        if (c < 0) break;
        return (double)c;
    }
    case kDistBinomial:
        if (!(is_count(a) && b >= 0.0 && b <= 1.0)) break;
        return (double)draw_binomial(s, (long long)a, b);
    default: break;
    }
    fault = true;
    return 0.0;
}

// Log-density of v; fault = true for parameters outside the family's domain.
// Operation order is part of the definition (results are compared bit for
// bit with an independent implementation).
__device__ inline double prog_logpdf(uint32_t dist, double a, double b, double v, bool& fault)
{
    const double ninf = -__builtin_huge_val();
    switch (dist) {
    case kDistUniform:
        if (!(b > a)) break;
        return (v >= a && v <= b) ? -fn::log(b - a) : ninf;
    case kDistNormal: {
        if (!(b > 0.0)) break;
        const double z = (v - a) / b;
        const double q = (-0.5 * z) * z;
        return (q - fn::log(b)) - kHalfLog2Pi;
    }
    case kDistExponential:
        if (!(a > 0.0)) break;
        return v >= 0.0 ? fn::log(a) - a * v : ninf;
    case kDistBernoulli:
        if (!(a >= 0.0 && a <= 1.0)) break;
        if (v == 1.0) return fn::log(a);
        return v == 0.0 ? fn::log(1.0 - a) : ninf;
    case kDistPoisson:
        if (!(a >= 0.0 && a < __builtin_huge_val())) break;
        if (!is_count(v)) return ninf;
        if (v == 0.0) return -a;
        return (v * fn::log(a) - a) - log_factorial((long long)v);
    case kDistBinomial:
        if (!(is_count(a) && b >= 0.0 && b <= 1.0)) break;
        if (!(is_count(v) && v <= a)) return ninf;
        return log_binomial_pmf((long long)v, (long long)a, b);
    default: break;
    }
    fault = true;
    return 0.0;
}

}  // namespace pcfg
