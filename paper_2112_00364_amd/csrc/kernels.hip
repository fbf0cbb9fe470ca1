// Round kernels for SMC over PCFGs on gfx950.
//
// One round of Algorithm 1 (Sec. 3.2) is three launches over a table of
// (run, tile) work-groups, so one launch serves any number of runs:
//   k_propagate  Alg. 1 step 2: each lane takes one particle slot j, gathers
//                its (block, state) from the ancestor chosen by the previous
//                resampling (the duplication step of Sec. 3.3, done on read),
//                runs blocks until a checkpoint or b_stop and writes block,
//                state and log-weight; each work-group folds its partial (max
//                log-weight key, active count, block steps) into one of
//                kPartialGroups slots of its run with two device atomics on
//                distinct addresses.
//   k_reduce     reads its run's group slots (M = max lw, NaN flag), then
//                sums exp(lw - M) (for log Z) and the grid-quantised weights of
//                its tile; tile 0 publishes M, the counts and the round's
//                offset word.
//   k_scan_anc   folds the tile sums of its run (total mass, tile offset),
//                scans the quantised weights inside the tile exactly, turns
//                cumulative mass into offspring counts by integer comparison
//                and writes the ancestor of every output slot it owns
//                (systematic resampling, Sec. 3.3); tile 0 updates log Z,
//                decides termination and advances the round.
// Runs above kMaxFusedRedTiles reduction tiles fold the tile sums in a
// one-work-group kernel (k_fold_sums) instead. Sums that decide anything are
// exact (integers, or maxima), so no result depends on the order of atomics.
// Memory is structure-of-arrays (Sec. 3.3): consecutive lanes touch
// consecutive elements of each field.
#include <type_traits>

#include "engine.hpp"
#include "launch.hpp"
#include "program.hpp"

namespace pcfg {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ inline unsigned long long order_key(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline double key_value(unsigned long long k)
{
    const unsigned long long b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

__device__ inline int grid_bits(uint32_t n)
{
    const int cl = n <= 1 ? 0 : 32 - __builtin_clz(n - 1);  // ceil(log2 n), n <= 2^24
    const int g = 53 - cl;
    return g < 32 ? g : 32;
}

// 64 x 64 -> 128-bit product.
struct U128 {
    unsigned long long hi, lo;
};
__device__ inline U128 mul128(unsigned long long a, unsigned long long b)
{
    return U128{__umul64hi(a, b), a * b};
}
__device__ inline bool less128(U128 a, U128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ inline U128 add128(U128 a, U128 b)
{
    const unsigned long long lo = a.lo + b.lo;
    return U128{a.hi + b.hi + (lo < a.lo ? 1ull : 0ull), lo};
}

// ESS-triggered resampling (adaptive resampling is listed among RootPPL's
// features in Sec. 3.3; the rule is this library's reading). With q the
// quantised weights of the resampling step, ESS = (sum q)^2 / sum q^2, and the
// round resamples iff ESS < t N / 2^16, decided exactly:
//   2^16 (sum q)^2 < t N sum q^2.
// sum q <= N 2^G <= 2^53 and sum q^2 <= 2^G sum q <= 2^85, so with t <= 2^16
// and N <= 2^24 both sides stay below 2^126. t = 0 always resamples.
__device__ inline bool ess_says_resample(uint32_t t, uint32_t N, double qtot, U128 q2)
{
    if (t == 0) return true;
    const unsigned long long s1 = (unsigned long long)qtot;
    const U128 sq = mul128(s1, s1);
    const U128 lhs{(sq.hi << 16) | (sq.lo >> 48), sq.lo << 16};
    const unsigned long long k = (unsigned long long)t * N;  // <= 2^40
    const U128 lo_part = mul128(q2.lo, k);
    const U128 rhs{lo_part.hi + q2.hi * k, lo_part.lo};
    return less128(lhs, rhs);
}

// Number of output slots j in [0, N) whose systematic position lies below
// cumulative mass W (grid units): #{ j : (j 2^32 + U) Qtot < N W 2^32 }, i.e.
// the number of integers j < y = N W / Qtot - U 2^-32. The FP64 estimate of y
// is within 1e-8 of y, so away from integers its ceiling is exact; within
// 2^-20 of an integer the count is settled by exact 128-bit comparisons.
__device__ inline uint32_t offspring_before(double W, double Qtot, double rQ, uint32_t U, uint32_t N)
{
    const double y = (double)N * (W * rQ) - (double)U * 0x1p-32;
    const double fl = __builtin_floor(y);
    const double frac = y - fl;
    if (frac > 0x1p-20 && frac < 1.0 - 0x1p-20) {
        const double c = fl + 1.0;
        return c <= 0.0 ? 0u : (c >= (double)N ? N : (uint32_t)c);
    }
    const unsigned long long w = (unsigned long long)W;
    const unsigned long long qt = (unsigned long long)Qtot;
    const U128 nw = mul128((unsigned long long)N, w);  // < 2^78
    const U128 rhs = U128{(nw.hi << 32) | (nw.lo >> 32), nw.lo << 32};
    auto below = [&](uint32_t j) {
        const unsigned long long pos = ((unsigned long long)j << 32) | (unsigned long long)U;
        return less128(mul128(pos, qt), rhs);
    };
    const double cf = __builtin_ceil(y);
    uint32_t c = cf <= 0.0 ? 0u : (cf >= (double)N ? N : (uint32_t)cf);
    while (c > 0 && !below(c - 1)) c -= 1;
    while (c < N && below(c)) c += 1;
    return c;
}

// Values every lane of a work-group reads from a run's control block are
// uniform; moving them to scalar registers keeps the address arithmetic that
// depends on them (the parity-selected particle buffer, for one) out of
// vector registers.
__device__ inline uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ inline int32_t uniform_i32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline unsigned long long uniform_u64(unsigned long long v)
{
    return ((unsigned long long)uniform_u32((uint32_t)(v >> 32)) << 32) | uniform_u32((uint32_t)v);
}

// Wavefront-wide scans and reductions with DPP row operations (the data moves
// between lanes inside the VALU, with no LDS round trip). Inclusive scan:
// shifts by 1, 2, 4, 8 within each row of 16 lanes, then the total of row r
// is added to row r + 1 (row_bcast:15) and the total of rows 0-1 to rows 2-3
// (row_bcast:31). Lanes outside the row mask or reading past a row start get
// the identity (0). The combination order is fixed, so results are
// reproducible. Every lane of the wavefront must be active.
enum : int { kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118,
             kRowBcast15 = 0x142, kRowBcast31 = 0x143 };

template <int kCtrl, int kRowMask>
__device__ inline uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, true);
}
template <int kCtrl, int kRowMask>
__device__ inline unsigned long long dpp_u64(unsigned long long v)
{
    const uint32_t lo = dpp_u32<kCtrl, kRowMask>((uint32_t)v);
    const uint32_t hi = dpp_u32<kCtrl, kRowMask>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
template <int kCtrl, int kRowMask>
__device__ inline double dpp_f64(double v)
{
    return __longlong_as_double((long long)dpp_u64<kCtrl, kRowMask>((unsigned long long)__double_as_longlong(v)));
}

struct OpAddF64 {
    static __device__ inline double op(double a, double b) { return a + b; }
    template <int C, int M>
    static __device__ inline double mv(double v) { return dpp_f64<C, M>(v); }
};
struct OpAddU32 {
    static __device__ inline uint32_t op(uint32_t a, uint32_t b) { return a + b; }
    template <int C, int M>
    static __device__ inline uint32_t mv(uint32_t v) { return dpp_u32<C, M>(v); }
};
struct OpMaxU32 {
    static __device__ inline uint32_t op(uint32_t a, uint32_t b) { return a > b ? a : b; }
    template <int C, int M>
    static __device__ inline uint32_t mv(uint32_t v) { return dpp_u32<C, M>(v); }
};
struct OpMaxU64 {
    static __device__ inline unsigned long long op(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
    template <int C, int M>
    static __device__ inline unsigned long long mv(unsigned long long v) { return dpp_u64<C, M>(v); }
};

struct OpAddU128 {
    static __device__ inline U128 op(U128 a, U128 b) { return add128(a, b); }
    template <int C, int M>
    static __device__ inline U128 mv(U128 v) { return U128{dpp_u64<C, M>(v.hi), dpp_u64<C, M>(v.lo)}; }
};

template <class Op, class T>
__device__ inline T wave_incl_scan(T v)
{
    v = Op::op(v, Op::template mv<kRowShr1, 0xf>(v));
    v = Op::op(v, Op::template mv<kRowShr2, 0xf>(v));
    v = Op::op(v, Op::template mv<kRowShr4, 0xf>(v));
    v = Op::op(v, Op::template mv<kRowShr8, 0xf>(v));
    v = Op::op(v, Op::template mv<kRowBcast15, 0xa>(v));
    v = Op::op(v, Op::template mv<kRowBcast31, 0xc>(v));
    return v;
}

__device__ inline uint32_t lane63_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }
__device__ inline unsigned long long lane63_u64(unsigned long long v)
{
    return ((unsigned long long)lane63_u32((uint32_t)(v >> 32)) << 32) | lane63_u32((uint32_t)v);
}

// Totals, the same in every lane.
__device__ inline double wave_sum(double v)
{
    v = wave_incl_scan<OpAddF64>(v);
    return __longlong_as_double((long long)lane63_u64((unsigned long long)__double_as_longlong(v)));
}
__device__ inline uint32_t wave_sum(uint32_t v) { return lane63_u32(wave_incl_scan<OpAddU32>(v)); }
__device__ inline unsigned long long wave_max_u64(unsigned long long v)
{
    return lane63_u64(wave_incl_scan<OpMaxU64>(v));
}
__device__ inline uint32_t wave_min_u32(uint32_t v) { return ~lane63_u32(wave_incl_scan<OpMaxU32>(~v)); }
__device__ inline U128 wave_sum(U128 v)
{
    v = wave_incl_scan<OpAddU128>(v);
    return U128{lane63_u64(v.hi), lane63_u64(v.lo)};
}

// Key stored for a tile that produced a NaN or +inf log-weight: above every
// order_key of a non-NaN double, so a max over tile keys flags the round.
constexpr unsigned long long kBadKey = ~0ull;

// Partial of a set of particles: max key, active count, NaN flag, block steps.
struct Partial {
    unsigned long long key;
    uint32_t act, bad, steps;
};

__device__ inline Partial combine(Partial a, Partial b)
{
    return Partial{a.key > b.key ? a.key : b.key, a.act + b.act, a.bad | b.bad, a.steps + b.steps};
}

__device__ inline Partial wave_partial(Partial p)
{
    p.key = wave_max_u64(p.key);
    p.act = wave_sum(p.act);
    p.bad = __ballot(p.bad != 0) ? 1u : 0u;
    p.steps = wave_sum(p.steps);
    return p;
}

// Work-group reduction of a Partial (fixed order); every thread gets the result.
template <int kThreads>
__device__ inline Partial block_partial(Partial p)
{
    __shared__ Partial s_part[kThreads / 64];
    p = wave_partial(p);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s_part[wave] = p;
    __syncthreads();
    Partial r = s_part[0];
    for (int w = 1; w < kThreads / 64; ++w) r = combine(r, s_part[w]);
    return r;
}

// Folds a work-group's partial into its group slot (device-scope atomics on
// distinct addresses; work-groups finish spread over the launch, so the slots
// see little contention).
__device__ inline void publish_group(const RunDev& R, uint32_t tile, const Partial& r)
{
    GroupPartials* g = R.groups;
    const uint32_t slot = tile & (kPartialGroups - 1u);
    const unsigned long long key = r.bad ? kBadKey : r.key;
    const unsigned long long counts = (unsigned long long)r.act | ((unsigned long long)r.steps << 32);
    if (key) atomicMax(&g->key[slot], key);
    if (counts) atomicAdd(&g->counts[slot], counts);
}

// The propagation's partials of a run from its group slots: each wavefront
// reads all kPartialGroups of them (kPartialGroups / 64 per lane, loads
// issued together); every thread gets the result. Counts are exact integer
// sums (a run's active particles and block steps per round stay below 2^32).
__device__ inline Partial fold_groups(const RunDev& R)
{
    constexpr int kPer = (int)(kPartialGroups / 64);
    static_assert(kPartialGroups % 64 == 0, "whole wavefronts of slots");
    const GroupPartials* g = R.groups;
    const int lane = threadIdx.x & 63;
    unsigned long long kv[kPer], cv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        kv[i] = g->key[lane + 64 * i];
        cv[i] = g->counts[lane + 64 * i];
    }
    unsigned long long key = 0, counts = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        key = kv[i] > key ? kv[i] : key;
        counts += cv[i];
    }
    key = wave_max_u64(key);
    const uint32_t act = wave_sum((uint32_t)counts);
    const uint32_t steps = wave_sum((uint32_t)(counts >> 32));
    return Partial{key, act, key == kBadKey ? 1u : 0u, steps};
}

// Work-group partial with no closing barrier: each wavefront leaves its
// partial in LDS and counts itself in; the last to arrive combines the
// partials in wavefront order and writes the tile's record. Wavefronts that
// finish early exit at once and free their slots for the next work-group.
// *arrived must be zero before any wavefront gets here.
template <int kThreads>
__device__ inline void publish_tile_partial(const RunDev& R, uint32_t tile, Partial p, uint32_t* arrived)
{
    __shared__ Partial s_part[kThreads / 64];
    p = wave_partial(p);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane != 0) return;
    s_part[wave] = p;
    __threadfence_block();
    if (atomicAdd(arrived, 1u) != (uint32_t)(kThreads / 64 - 1)) return;
    __threadfence_block();
    Partial r = s_part[0];
    for (int w = 1; w < kThreads / 64; ++w) r = combine(r, s_part[w]);
    publish_group(R, tile, r);
}

// ---------------------------------------------------------------------------
// Propagation (Alg. 1 step 2) with gather-on-read of the previous resampling.
// ---------------------------------------------------------------------------
template <class Real>
__device__ inline double load_real(const void* p, uint32_t i)
{
    return (double)static_cast<const Real*>(p)[i];
}
template <class Real>
__device__ inline void store_real(void* p, uint32_t i, double v)
{
    static_cast<Real*>(p)[i] = (Real)v;
}

// CRBD frame stacks: registers on the fast path, LDS for the rare deep particle.
template <bool kDeep>
struct CrbdStack {
    using type = typename std::conditional<kDeep, LdsFrames<CrbdFrame>, RegFrames<CrbdFrame, kRegFrames>>::type;
};

// Bytes of one wavefront's LDS stack for the deep pass.
constexpr int kDeepStackBytes = kMaxDepthCap * sizeof(CrbdFrame);

// One particle slot j of round `round`: gather (block, state) from the
// ancestor, run blocks until a checkpoint or b_stop, store the results.
// Returns false (storing nothing) when a register stack overflowed. Forced
// inline: an out-of-line call (taken once the kernel has several
// instantiations) costs the SEIR propagation about 6 %.
template <int Kind, class Real, bool kDeep>
__device__ __forceinline__ bool run_particle(const RunDev& R, const ModelDev& m, uint64_t seed, uint32_t j, uint32_t round,
                                    uint32_t src, double lw0, uint8_t& blk, double& lw, uint32_t& steps,
                                    void* lds_stack)
{
    const ParticleBuf& out = R.buf[round & 1u];
    const ParticleBuf& in = R.buf[(round & 1u) ^ 1u];
    blk = round > 0 ? in.blk[src] : 0;
    lw = lw0;
    steps = 0;
    Stream s;
    s.start(seed, j, round, kTagPropagate);
    bool overflow = false;
    if constexpr (Kind == 0) {
        Geometric::State st{round > 0 ? in.ints[0][src] : 0};
        while (blk != kStop) {
            bool ck = false;
            blk = Geometric::sim(m, round, blk, st, lw, s, ck);
            steps += 1;
            if (ck) break;
        }
        out.ints[0][j] = st.flips;
    } else if constexpr (Kind == 1) {
        typename Lgssm<Real>::State st{round > 0 ? load_real<Real>(in.real[0], src) : 0.0};
        while (blk != kStop) {
            bool ck = false;
            blk = Lgssm<Real>::sim(m, round, blk, st, lw, s, ck);
            steps += 1;
            if (ck) break;
        }
        store_real<Real>(out.real[0], j, st.x);
    } else if constexpr (Kind == 2) {
        using Stack = typename CrbdStack<kDeep>::type;
        Stack stack;
        if constexpr (kDeep) stack.base = static_cast<CrbdFrame*>(lds_stack);
        typename Crbd<Real>::State st{0.0, 0.0};
        if (round > 0) {
            st.lambda = load_real<Real>(in.real[0], src);
            st.mu = load_real<Real>(in.real[1], src);
        }
        while (blk != kStop) {
            bool ck = false;
            blk = Crbd<Real>::template sim<Stack>(m, round, blk, st, lw, s, ck, overflow, stack);
            if (overflow) return false;
            steps += 1;
            if (ck) break;
        }
        store_real<Real>(out.real[0], j, st.lambda);
        store_real<Real>(out.real[1], j, st.mu);
    } else if constexpr (Kind == 5) {
        using Stack = typename CrbdStack<kDeep>::type;
        Stack stack;
        if constexpr (kDeep) stack.base = static_cast<CrbdFrame*>(lds_stack);
        typename CrbdDs<Real>::State st{0.0, 0.0, 0.0, 0.0};
        if (round > 0) {
            st.a_l = load_real<Real>(in.real[0], src);
            st.th_l = load_real<Real>(in.real[1], src);
            st.a_mu = load_real<Real>(in.real[2], src);
            st.th_mu = load_real<Real>(in.real[3], src);
        }
        while (blk != kStop) {
            bool ck = false;
            blk = CrbdDs<Real>::template sim<Stack>(m, round, blk, st, lw, s, ck, overflow, stack);
            if (overflow) return false;
            steps += 1;
            if (ck) break;
        }
        store_real<Real>(out.real[0], j, st.a_l);
        store_real<Real>(out.real[1], j, st.th_l);
        store_real<Real>(out.real[2], j, st.a_mu);
        store_real<Real>(out.real[3], j, st.th_mu);
    } else if constexpr (Kind == 4) {
        typename Seir<Real>::State st{};
        if (round > 0) {
#pragma unroll
            for (int f = 0; f < Seir<Real>::kReal; ++f) st.r[f] = load_real<Real>(in.real[f], src);
#pragma unroll
            for (int f = 0; f < Seir<Real>::kInt; ++f) st.c[f] = in.ints[f][src];
        }
        while (blk != kStop) {
            bool ck = false;
            blk = Seir<Real>::sim(m, round, blk, st, lw, s, ck);
            steps += 1;
            if (ck) break;
        }
#pragma unroll
        for (int f = 0; f < Seir<Real>::kReal; ++f) store_real<Real>(out.real[f], j, st.r[f]);
#pragma unroll
        for (int f = 0; f < Seir<Real>::kInt; ++f) out.ints[f][j] = (int32_t)st.c[f];
    } else {
        using Stack = ClaDSGlobalFrames;
        const uint64_t levels = (uint64_t)kMaxDepthCap * R.n;
        Stack stack{static_cast<double*>(R.side_stack), static_cast<double*>(R.side_stack) + levels,
                    reinterpret_cast<uint8_t*>(static_cast<double*>(R.side_stack) + 2 * levels), (uint64_t)R.n, j};
        typename Clads<Real>::State st{0.0, 0.0, 0.0, 0.0};
        if (round > 0) {
            st.lambda = load_real<Real>(in.real[0], src);
            st.eps = load_real<Real>(in.real[1], src);
            st.alpha = load_real<Real>(in.real[2], src);
            st.sigma = load_real<Real>(in.real[3], src);
        }
        typename Clads<Real>::StackIO io{static_cast<const Real*>(in.stack), static_cast<Real*>(out.stack),
                                         (uint64_t)R.n, src, j};
        while (blk != kStop) {
            bool ck = false;
            blk = Clads<Real>::template sim<Stack>(m, round, blk, st, lw, s, ck, io, overflow, stack);
            if (overflow) return false;
            steps += 1;
            if (ck) break;
        }
        store_real<Real>(out.real[0], j, st.lambda);
        store_real<Real>(out.real[1], j, st.eps);
        store_real<Real>(out.real[2], j, st.alpha);
        store_real<Real>(out.real[3], j, st.sigma);
    }
    out.blk[j] = blk;
    R.lw[j] = lw;
    return true;
}

// ---------------------------------------------------------------------------
// Compiled programs (Sec. 4): each lane interprets the bytecode blocks of its
// particle until a checkpoint or b_stop. The particle's state is its block,
// its stack pointer sp and a stack of FP64 words stored level-major (word w
// of slot j at w * N + j), so lanes touching the same word touch consecutive
// addresses. The gather of the previous resampling copies only the live part
// [0, sp) of the ancestor's stack (Sec. 3.3).
//
// Scheduling: every step executes the instruction at the smallest program
// counter among the wavefront's running lanes, for the lanes at that counter.
// Opcode and operands are then wavefront-uniform (one scalar load, scalar
// branches, LDS register addresses off a scalar offset), and since jumps
// inside a block only go forward, lanes split by a branch rejoin where the
// branches meet. Registers live in LDS (lane-interleaved: no bank conflicts).
// Every stack and data access is in range by construction: the host checks
// operand bounds, frame sizes and jump targets; the kernel checks sp against
// frame sizes and the capacity, and the stored return blocks, return-value
// locations and data indices, faulting the particle (weight -inf) otherwise.
// ---------------------------------------------------------------------------
// Slot a propagation lane takes: its position, or the position's entry of the
// bucketing permutation (clamped, so a malformed entry cannot leave the run).
__device__ inline uint32_t lane_slot(const RunDev& R, uint32_t idx)
{
    if (!R.perm || idx >= R.n) return idx;
    const uint32_t j = R.perm[idx];
    return j < R.n ? j : idx;
}

template <int kThreads>
__device__ __forceinline__ void program_body(const RunDev& R, uint32_t tile)
{
    const uint32_t j = lane_slot(R, tile * kThreads + threadIdx.x);
    const bool valid = j < R.n;
    RunCtl* ctl = R.ctl;
    const int32_t status = uniform_i32(ctl->status);
    const uint32_t round = uniform_u32(ctl->round);
    const uint64_t seed = uniform_u64(ctl->seed);
    const bool carry = uniform_u32(ctl->carry) != 0;
    const uint32_t ancestor = valid ? R.anc[j] : 0u;
    if (status != 0) return;  // uniform over the work-group
    const uint32_t src = (round > 0 && !carry) ? ancestor : j;
    const double lw0 = (carry && valid) ? R.lw[j] : 0.0;
    __shared__ uint32_t s_arrived;
    __shared__ double s_reg[kProgRegs * kThreads];
    if (threadIdx.x == 0) s_arrived = 0;
    __syncthreads();
    const ProgramDev P = R.model->prog;
    const ParticleBuf& out = R.buf[round & 1u];
    const ParticleBuf& in = R.buf[(round & 1u) ^ 1u];
    const uint64_t n = R.n;
    double* __restrict__ st = static_cast<double*>(out.stack);
    const double* __restrict__ st_in = static_cast<const double*>(in.stack);
    double* __restrict__ reg = s_reg + threadIdx.x;  // register r at reg[r * kThreads]
    // The bytecode is read-only for the whole launch: in the constant address
    // space its wavefront-uniform reads can be scalar loads.
    using ConstWord = const __attribute__((address_space(4))) unsigned long long;
    ConstWord* code = (ConstWord*)P.code;

    uint32_t blk = kStop, sp = 0;
    double lw = lw0;
    if (valid) {
        blk = round > 0 ? in.blk[src] : 0u;
        sp = round > 0 ? (uint32_t)in.ints[0][src] : 0u;
    }
    if (sp > P.stack_words) {  // never written by this kernel; keeps every access in range
        sp = 0;
        blk = kStop;
        lw = -__builtin_huge_val();
    }
    // Live-prefix gather, 16 words in flight per lane (all loads before the
    // stores). Apart from the top frame, the copied words are read again only
    // by the next round's gather, so the stores are non-temporal.
    uint32_t w0 = 0;
    for (; w0 + 16 <= sp; w0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = st_in[(uint64_t)(w0 + u) * n + src];
#pragma unroll
        for (int u = 0; u < 16; ++u) __builtin_nontemporal_store(v[u], &st[(uint64_t)(w0 + u) * n + j]);
    }
    for (; w0 < sp; ++w0) st[(uint64_t)w0 * n + j] = st_in[(uint64_t)w0 * n + src];

    bool live = valid && blk != kStop;
    uint32_t pc = live ? P.block_start[blk] : 0u;
    uint32_t fp = 0, steps = live ? 1u : 0u, executed = 0;
    Stream s;
    s.start(seed, j, round, kTagPropagate);
    for (;;) {
        const uint32_t sel = wave_min_u32(live ? pc : 0xffffffffu);
        if (sel == 0xffffffffu) break;  // uniform: no lane of the wavefront is running
        // The fetch address must stay the wavefront-uniform sel: under the
        // branch on pc == sel the compiler would otherwise substitute the
        // lane's own pc and fetch and decode per lane. An empty asm statement
        // with a scalar-register operand makes the copy opaque, so the word
        // comes by one scalar load and the dispatch below is scalar.
        uint32_t at = sel;
        asm volatile("" : "+s"(at));
        const unsigned long long word = code[at];
        const uint32_t lo = (uint32_t)word;
        const uint32_t op = lo & 255u, x = (lo >> 8) & 255u, y = (lo >> 16) & 255u, z = lo >> 24;
        const uint32_t imm = (uint32_t)(word >> 32);
        if (!(live && pc == sel)) continue;
        double* rx = reg + x * kThreads;
        const double ry = reg[y * kThreads], rz = reg[z * kThreads];
        pc = sel + 1;
        bool fault = ++executed > kProgInstrBudget;
        if (!fault) {
            switch (op) {
            case kOpFrame:
                if (sp < imm) fault = true;
                else fp = sp - imm;
                break;
            case kOpConst: *rx = P.consts[imm]; break;
            case kOpImm: *rx = (double)(int32_t)imm; break;
            case kOpMov: *rx = ry; break;
            case kOpLdf: *rx = st[(uint64_t)(fp + imm) * n + j]; break;
            case kOpStf: st[(uint64_t)(fp + imm) * n + j] = *rx; break;
            case kOpAdd: *rx = ry + rz; break;
            case kOpSub: *rx = ry - rz; break;
            case kOpMul: *rx = ry * rz; break;
            case kOpDiv: *rx = ry / rz; break;
            case kOpLt: *rx = ry < rz ? 1.0 : 0.0; break;
            case kOpLe: *rx = ry <= rz ? 1.0 : 0.0; break;
            case kOpEq: *rx = ry == rz ? 1.0 : 0.0; break;
            case kOpNe: *rx = ry != rz ? 1.0 : 0.0; break;
            case kOpNeg: *rx = -ry; break;
            case kOpNot: *rx = ry == 0.0 ? 1.0 : 0.0; break;
            case kOpLog: *rx = fn::log(ry); break;
            case kOpExp: *rx = fn::exp(ry); break;
            case kOpSqrt: *rx = fn::sqrt(ry); break;
            case kOpFloor: *rx = __builtin_floor(ry); break;
            case kOpData: {
                const uint32_t a0 = P.array_start[imm], a1 = P.array_start[imm + 1];
                if (!(ry >= 0.0 && ry < (double)(a1 - a0) && ry == __builtin_floor(ry))) fault = true;
                else *rx = P.data[a0 + (uint32_t)ry];
                break;
            }
            case kOpLen: *rx = (double)(P.array_start[imm + 1] - P.array_start[imm]); break;
            case kOpSample: {
                const double v = prog_draw(imm, ry, rz, s, fault);
                if (!fault) *rx = v;
                break;
            }
            case kOpObserve: {
                const double d = prog_logpdf(imm, ry, rz, *rx, fault);
                if (!fault) lw = lw + d;
                break;
            }
            case kOpWeight: lw = lw + *rx; break;
            case kOpJz:
                if (*rx == 0.0) pc = imm;
                break;
            case kOpJmp: pc = imm; break;
            case kOpCallFrame:
                if (imm > P.stack_words - sp) fault = true;
                break;
            case kOpStn: st[(uint64_t)(sp + imm) * n + j] = *rx; break;
            case kOpAddr: *rx = (double)(fp + imm); break;
            case kOpPush: sp += imm; break;
            case kOpStret: {
                const double loc = st[(uint64_t)(fp + 1u) * n + j];
                if (!(loc >= 0.0 && loc < (double)sp && loc == __builtin_floor(loc))) fault = true;
                else st[(uint64_t)loc * n + j] = *rx;
                break;
            }
            case kOpGoto:
            case kOpCkpt:
            case kOpJret: {
                uint32_t next = imm;
                if (op == kOpJret) {
                    const double ra = st[(uint64_t)fp * n + j];
                    if (ra == (double)kStop) {
                        next = kStop;
                    } else if (ra >= 0.0 && ra < (double)P.n_blocks && ra == __builtin_floor(ra)) {
                        next = (uint32_t)ra;
                    } else {
                        fault = true;
                        break;
                    }
                    sp -= imm;
                }
                blk = next;
                if (next == kStop || op == kOpCkpt) {
                    live = false;
                } else {
                    steps += 1;
                    pc = P.block_start[next];
                }
                break;
            }
            default: fault = true; break;  // kOpFault
            }
        }
        if (fault) {
            lw = -__builtin_huge_val();
            blk = kStop;
            sp = 0;
            live = false;
        }
    }
    if (valid) {
        out.blk[j] = (uint8_t)blk;
        out.ints[0][j] = (int32_t)sp;
        R.lw[j] = lw;
    }
    Partial p{0ull, 0u, 0u, 0u};
    if (valid) {
        if (lw != lw || lw == __builtin_huge_val()) p.bad = 1;
        else p.key = order_key(lw);
        p.act = blk != kStop ? 1u : 0u;
        p.steps = steps;
    }
    publish_tile_partial<kThreads>(R, tile, p, &s_arrived);
}

// Hidden-lineage stacks live in registers (kRegFrames frames). A particle that
// needs more is recomputed, in the same work-group, one lane of its wavefront
// at a time with a kMaxDepthCap-frame stack in LDS; its random stream is
// counter-based, so the recomputation draws the same words.
template <int Kind, class Real, int kThreads>
__device__ __forceinline__ void builtin_body(const RunDev& R, uint32_t tile)
{
    const uint32_t j = lane_slot(R, tile * kThreads + threadIdx.x);
    const bool valid = j < R.n;
    RunCtl* ctl = R.ctl;
    const int32_t status = uniform_i32(ctl->status);
    const uint32_t round = uniform_u32(ctl->round);
    const uint64_t seed = uniform_u64(ctl->seed);
    const bool carry = uniform_u32(ctl->carry) != 0;
    // The ancestor index is loaded before the control block is consumed, so
    // the two loads overlap (at round 0 the value is not used).
    const uint32_t ancestor = valid ? R.anc[j] : 0u;
    if (status != 0) return;  // uniform over the work-group
    // After a round that kept its weights (ESS rule) the particle continues in
    // its own slot from its carried log-weight; otherwise it starts from its
    // ancestor with weight 0.
    const uint32_t src = (round > 0 && !carry) ? ancestor : j;
    const double lw0 = (carry && valid) ? R.lw[j] : 0.0;
    __shared__ uint32_t s_arrived;
    if (threadIdx.x == 0) s_arrived = 0;
    __syncthreads();
    const ModelDev& m = *R.model;
    uint8_t blk = kStop;
    double lw = 0.0;
    uint32_t steps = 0;
    bool deep = false;
    if (valid) deep = !run_particle<Kind, Real, false>(R, m, seed, j, round, src, lw0, blk, lw, steps, nullptr);
    if constexpr (Kind == 2 || Kind == 5) {
        __shared__ __align__(16) unsigned char s_stack[kThreads / 64][kDeepStackBytes];
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        unsigned long long pending = __ballot(deep);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            if (lane == leader)
                run_particle<Kind, Real, true>(R, m, seed, j, round, src, lw0, blk, lw, steps, s_stack[wave]);
            pending &= pending - 1;
        }
    }
    Partial p{0ull, 0u, 0u, 0u};
    if (valid) {
        if (lw != lw || lw == __builtin_huge_val()) p.bad = 1;
        else p.key = order_key(lw);
        p.act = blk != kStop ? 1u : 0u;
        p.steps = steps;
    }
    publish_tile_partial<kThreads>(R, tile, p, &s_arrived);
}

template <int Kind, class Real, int kThreads>
__device__ __forceinline__ void propagate_body(const RunDev& R, uint32_t tile)
{
    if constexpr (Kind == 6) program_body<kThreads>(R, tile);
    else builtin_body<Kind, Real, kThreads>(R, tile);
}

// Entry points: one run (its record is a kernel argument, tile = work-group)
// or a batch (work-group -> (run, tile) table).
template <int Kind, class Real, int kThreads>
__global__ __launch_bounds__(kThreads) void k_propagate_one(const RunDev R)
{
    propagate_body<Kind, Real, kThreads>(R, blockIdx.x);
}

template <int Kind, class Real, int kThreads>
__global__ __launch_bounds__(kThreads) void k_propagate(const RunDev* __restrict__ runs,
                                                        const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    propagate_body<Kind, Real, kThreads>(runs[tr.run], tr.tile);
}

// ---------------------------------------------------------------------------
// Block bucketing (optional). Before a propagation, a stable counting sort of
// the particle slots by the block each resumes at (the ancestor's block, or
// its own after a round that kept its weights; 255 = b_stop sorts last), so
// the lanes of a wavefront mostly run the same block. Three launches over
// kTileRed-slot tiles: per-tile counts (block-major), an exclusive scan of
// each block's counts over the tiles, and a scatter that ranks every slot
// among the equal keys before it (rows of 64 slots, ranked with ballots).
// Slots keep their random streams, so the results do not depend on it.
// ---------------------------------------------------------------------------
__device__ inline uint32_t resume_key(const RunDev& R, uint32_t j, uint32_t round, bool carry)
{
    if (round == 0) return 0u;
    const ParticleBuf& in = R.buf[(round & 1u) ^ 1u];
    return in.blk[carry ? j : R.anc[j]];
}

// Inclusive scan of one value per thread over a kRedThreads work-group.
__device__ inline uint32_t block_incl_scan_u32(uint32_t v)
{
    __shared__ uint32_t s_wave[kRedThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_incl_scan<OpAddU32>(v);
    if (lane == 63) s_wave[wave] = v;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    __syncthreads();
    return v + before;
}

__global__ __launch_bounds__(kRedThreads) void k_bucket_count(const RunDev R)
{
    RunCtl* ctl = R.ctl;
    if (uniform_i32(ctl->status) != 0) return;
    const uint32_t round = uniform_u32(ctl->round);
    const bool carry = uniform_u32(ctl->carry) != 0;
    __shared__ uint32_t s_hist[kBuckets];
    s_hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kTileRed;
    for (int i = 0; i < kRedItems; ++i) {
        const uint32_t j = base + threadIdx.x + i * kRedThreads;
        if (j < R.n) atomicAdd(&s_hist[resume_key(R, j, round, carry)], 1u);
    }
    __syncthreads();
    R.bucket_hist[threadIdx.x * R.red_tiles + blockIdx.x] = s_hist[threadIdx.x];
}

// One work-group per block: exclusive prefix of its counts over the tiles.
__global__ __launch_bounds__(kRedThreads) void k_bucket_scan(const RunDev R)
{
    if (uniform_i32(R.ctl->status) != 0) return;
    uint32_t* col = R.bucket_hist + (uint64_t)blockIdx.x * R.red_tiles;
    const uint32_t T = R.red_tiles;
    const uint32_t per = (T + kRedThreads - 1) / kRedThreads;
    const uint32_t lo = threadIdx.x * per;
    const uint32_t hi = lo + per < T ? lo + per : T;
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i) sum += col[i];
    const uint32_t incl = block_incl_scan_u32(sum);
    uint32_t run = incl - sum;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = col[i];
        col[i] = run;
        run += v;
    }
    if (threadIdx.x == kRedThreads - 1) R.bucket_total[blockIdx.x] = incl;
}

__global__ __launch_bounds__(kRedThreads) void k_bucket_scatter(const RunDev R)
{
    RunCtl* ctl = R.ctl;
    if (uniform_i32(ctl->status) != 0) return;
    const uint32_t round = uniform_u32(ctl->round);
    const bool carry = uniform_u32(ctl->carry) != 0;
    constexpr int kRows = kTileRed / 64;
    __shared__ uint32_t s_base[kBuckets];
    __shared__ uint32_t s_row[kRows][kBuckets];
    const uint32_t t = threadIdx.x;
    const uint32_t tot = R.bucket_total[t];
    const uint32_t incl = block_incl_scan_u32(tot);
    s_base[t] = (incl - tot) + R.bucket_hist[t * R.red_tiles + blockIdx.x];
    for (int r = 0; r < kRows; ++r) s_row[r][t] = 0;
    __syncthreads();
    const int wave = t >> 6, lane = t & 63;
    constexpr int kRowsPerWave = kRows / (kRedThreads / 64);
    uint32_t key[kRowsPerWave];
    bool valid[kRowsPerWave];
    for (int q = 0; q < kRowsPerWave; ++q) {
        const int row = wave + (kRedThreads / 64) * q;
        const uint32_t j = blockIdx.x * kTileRed + row * 64 + lane;
        valid[q] = j < R.n;
        key[q] = valid[q] ? resume_key(R, j, round, carry) : 0u;
        unsigned long long todo = __ballot(valid[q]);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)key[q], leader);
            const unsigned long long mask = __ballot(valid[q] && key[q] == lk);
            if (lane == leader) s_row[row][lk] = (uint32_t)__popcll(mask);
            todo &= ~mask;
        }
    }
    __syncthreads();
    uint32_t run = 0;
    for (int r = 0; r < kRows; ++r) {
        const uint32_t c = s_row[r][t];
        s_row[r][t] = run;
        run += c;
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int q = 0; q < kRowsPerWave; ++q) {
        const int row = wave + (kRedThreads / 64) * q;
        const uint32_t j = blockIdx.x * kTileRed + row * 64 + lane;
        unsigned long long todo = __ballot(valid[q]);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)key[q], leader);
            const unsigned long long mask = __ballot(valid[q] && key[q] == lk);
            if (valid[q] && key[q] == lk) {
                const uint32_t pos = s_base[lk] + s_row[row][lk] + (uint32_t)__popcll(mask & below);
                if (pos < R.n) R.perm[pos] = j;
            }
            todo &= ~mask;
        }
    }
}

// ---------------------------------------------------------------------------
// Reduction: M, then per-tile sums of exp(lw - M) and grid units.
// ---------------------------------------------------------------------------
constexpr int kFoldThreads = 512;

// Publishes the round's fold of the propagation partials (one writer per run).
__device__ inline void publish_fold(const RunDev& R, RunCtl* ctl, const Partial& f)
{
    ctl->maxkey = f.key;
    ctl->bad = f.bad;
    ctl->active = f.act;
    ctl->block_steps += f.steps;
    const uint32_t round = ctl->round;
    const uint64_t seed = ctl->seed;
    ctl->u = philox10(0u, 0u, round, kTagResample, (uint32_t)seed, (uint32_t)(seed >> 32)).w0;
}

__device__ __forceinline__ void reduce_body(const RunDev& R, const TileRef tr)
{
    // The status, the tile's log-weights and the propagation partials are all
    // requested before any of them is used, so their latencies overlap.
    RunCtl* ctl = R.ctl;
    const int32_t status = uniform_i32(ctl->status);
    double x[kRedItems];
    const uint32_t base = tr.tile * kTileRed + threadIdx.x * kRedItems;
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) x[k] = base + k < R.n ? R.lw[base + k] : 0.0;
    // one wavefront folds the run's group slots for the whole work-group
    __shared__ Partial s_fold;
    if (threadIdx.x < 64) {
        const Partial g = fold_groups(R);
        if (threadIdx.x == 0) s_fold = g;
    }
    __syncthreads();
    const Partial f = s_fold;
    if (status != 0) return;  // uniform over the work-group
    if (tr.tile == 0 && threadIdx.x == 0) publish_fold(R, ctl, f);
    const unsigned long long key = f.key;
    const double M = key_value(key);
    if (key == kBadKey || key == 0 || M == -__builtin_huge_val()) return;  // uniform over the work-group
    const double scale = (double)(1ull << grid_bits(R.n));
    const bool ess = R.ess_t != 0;  // uniform
    double sq = 0.0, se = 0.0;
    U128 sq2{0ull, 0ull};
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) {
        if (base + k < R.n) {
            const double e = fn::exp(x[k] - M);
            const double q = __builtin_rint(e * scale);
            se += e;
            sq += q;
            if (ess) sq2 = add128(sq2, mul128((unsigned long long)q, (unsigned long long)q));
        }
    }
    sq = wave_sum(sq);
    se = wave_sum(se);
    if (ess) sq2 = wave_sum(sq2);
    __shared__ double s_q[kRedThreads / 64], s_e[kRedThreads / 64];
    __shared__ U128 s_q2[kRedThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_q[wave] = sq;
        s_e[wave] = se;
        s_q2[wave] = sq2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double q = s_q[0], e = s_e[0];
        U128 q2 = s_q2[0];
        for (int w = 1; w < kRedThreads / 64; ++w) {
            q += s_q[w];
            e += s_e[w];
            q2 = add128(q2, s_q2[w]);
        }
        R.part_q[tr.tile] = q;
        R.part_e[tr.tile] = e;
        if (ess) {
            R.part_q2[2 * tr.tile] = q2.lo;
            R.part_q2[2 * tr.tile + 1] = q2.hi;
        }
    }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_one(const RunDev R)
{
    reduce_body(R, TileRef{0u, blockIdx.x});
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const RunDev* __restrict__ runs,
                                                         const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    reduce_body(runs[tr.run], tr);
}

// log Z update, termination and the next round (one writer per run). active:
// some particle is not at b_stop; resample: the round resamples (always when
// active without an ESS threshold). A round that keeps its weights leaves
// log Z alone and marks the carry for the next propagation.
__device__ inline void finish_round(const RunDev& R, RunCtl* ctl, bool bad, bool usable, double M, double S,
                                    bool active, bool resample)
{
    if (bad) {
        ctl->status = -5;  // SMC_ERR_NAN
    } else if (!usable) {
        ctl->log_z = -__builtin_huge_val();
        ctl->status = -6;  // SMC_DEGENERATE
    } else if (!active) {
        ctl->log_z = ctl->log_z + ((M + fn::log(S)) - fn::log((double)R.n));
        ctl->status = 1;  // SMC_FINISHED
    } else if (resample) {
        ctl->log_z = ctl->log_z + ((M + fn::log(S)) - fn::log((double)R.n));
        ctl->round = ctl->round + 1;
        ctl->carry = 0;
        ctl->resamples = ctl->resamples + 1;
    } else {
        ctl->round = ctl->round + 1;
        ctl->carry = 1;
    }
}

// Fold-kernel path (large runs): one work-group per run folds the reduction's
// tile sums and writes the tile offsets.
// Tiles folded per thread: kFoldPer x kFoldThreads tiles of kTileRed particles
// cover the largest run (2^24 particles).
constexpr uint32_t kFoldPer = 32;
static_assert((unsigned long long)kFoldPer * kFoldThreads * kTileRed >= (1ull << 24), "fold covers 2^24 particles");

__device__ __forceinline__ void fold_sums_body(const RunDev& R)
{
    if (R.fused) return;  // this run's scan folds its own tile sums
    RunCtl* ctl = R.ctl;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t T = R.red_tiles;
    const bool ess = R.ess_t != 0;
    // Tile t sits in row t / kFoldThreads, column t % kFoldThreads: thread c
    // holds column c, so every load of a row is one coalesced access. All tile
    // sums are requested at once, before the control block is consumed (zeros
    // past the last tile leave every sum unchanged: they are non-negative).
    double qv[kFoldPer];
    double e_local = 0.0;
#pragma unroll
    for (uint32_t i = 0; i < kFoldPer; ++i) {
        const uint32_t t = i * kFoldThreads + threadIdx.x;
        qv[i] = t < T ? R.part_q[t] : 0.0;
        e_local += t < T ? R.part_e[t] : 0.0;
    }
    if (ctl->status != 0) return;
    const bool bad = ctl->bad != 0;
    const double M = key_value(ctl->maxkey);
    const bool usable = !bad && ctl->maxkey != 0 && M != -__builtin_huge_val();
    U128 q2_local{0ull, 0ull};
    if (!usable) {
#pragma unroll
        for (uint32_t i = 0; i < kFoldPer; ++i) qv[i] = 0.0;
        e_local = 0.0;
    }
    if (usable && ess)
        for (uint32_t t = threadIdx.x; t < T; t += kFoldThreads)
            q2_local = add128(q2_local, U128{R.part_q2[2 * t + 1], R.part_q2[2 * t]});
    // Exclusive prefix of every tile in row-major order: the rows before it,
    // the wavefronts before it in its row, the lanes before it in its
    // wavefront. The q sums are integer-valued and below 2^53, so every
    // partial sum is exact and the order of the additions does not matter.
    constexpr int kWaves = kFoldThreads / 64;
    __shared__ double s_row_wave[kFoldPer][kWaves];  // wavefront totals per row
    __shared__ double s_ew[kWaves];
    __shared__ U128 s_q2w[kWaves];
#pragma unroll
    for (uint32_t i = 0; i < kFoldPer; ++i) {
        const double incl = wave_incl_scan<OpAddF64>(qv[i]);
        if (lane == 63) s_row_wave[i][wave] = incl;
        qv[i] = incl - qv[i];  // exclusive within the wavefront (exact)
    }
    const double e_wave = wave_sum(e_local);
    const U128 q2_wave = ess ? wave_sum(q2_local) : U128{0ull, 0ull};
    if (lane == 0) {
        s_ew[wave] = e_wave;
        s_q2w[wave] = q2_wave;
    }
    __syncthreads();
    // one lane per row: the wavefront totals become offsets within the row
    __shared__ double s_row_total[kFoldPer];
    if (threadIdx.x < kFoldPer) {
        const uint32_t i = threadIdx.x;
        double run = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            const double x = s_row_wave[i][w];
            s_row_wave[i][w] = run;
            run += x;
        }
        s_row_total[i] = run;
    }
    __syncthreads();
    double q_all = 0.0, e_all = 0.0;
    U128 q2_all{0ull, 0ull};
    for (uint32_t i = 0; i < kFoldPer; ++i) q_all += s_row_total[i];
    for (int w = 0; w < kWaves; ++w) {
        e_all += s_ew[w];
        q2_all = add128(q2_all, s_q2w[w]);
    }
    const bool active = ctl->active != 0;
    const bool resample = active && ess_says_resample(R.ess_t, R.n, q_all, q2_all);
    if (usable && resample) {
        double row_base = 0.0;
#pragma unroll
        for (uint32_t i = 0; i < kFoldPer; ++i) {
            const uint32_t t = i * kFoldThreads + threadIdx.x;
            if (t < T) R.prefix[t] = row_base + s_row_wave[i][wave] + qv[i];
            row_base += s_row_total[i];
        }
    }
    if (threadIdx.x == 0) {
        ctl->m_cur = M;
        ctl->qtot = q_all;
        finish_round(R, ctl, bad, usable, M, e_all, active, resample);
    }
}

__global__ __launch_bounds__(kFoldThreads) void k_fold_sums(const RunDev* __restrict__ runs)
{
    fold_sums_body(runs[blockIdx.x]);
}

__global__ __launch_bounds__(kFoldThreads) void k_fold_sums_one(const RunDev R)
{
    fold_sums_body(R);
}

// ---------------------------------------------------------------------------
// Exact scan + systematic ancestors for the output slots owned by each tile.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scan_anc_body(const RunDev& R, const TileRef tr)
{
    // Stable during this kernel (written by k_reduce / k_fold_* of this round).
    // Only tile 0 writes the control block here, and nothing it writes is read
    // by the other tiles except status, whose change (run finished or failed)
    // also tells them to do nothing.
    RunCtl* ctl = R.ctl;
    const int32_t status = uniform_i32(ctl->status);
    const unsigned long long key = uniform_u64(ctl->maxkey);
    const bool bad = uniform_u32(ctl->bad) != 0;
    const bool active = uniform_u32(ctl->active) != 0;
    const bool carry = uniform_u32(ctl->carry) != 0;  // large runs: the fold kernel's decision
    const uint32_t U = uniform_u32(ctl->u);
    const uint32_t N = R.n;
    const bool ess = R.ess_t != 0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ double s_wave[kRedThreads / 64];
    __shared__ double s_wave2[kRedThreads / 64];
    __shared__ double s_wave3[kRedThreads / 64];

    // The tile's log-weights and the tile sums are requested before the control
    // block is consumed, so all these loads are in flight together; when the
    // round turns out not to resample they are simply not used.
    const uint32_t tile0 = tr.tile * kTileRed;
    const uint32_t first = tile0 + threadIdx.x * kRedItems;
    double x[kRedItems];
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) x[k] = first + k < N ? R.lw[first + k] : 0.0;
    constexpr int kPer = (int)(kMaxFusedRedTiles / kRedThreads);
    double qv[kPer], ev[kPer];
    U128 q2v[kPer];
    if (R.fused) {
        const uint32_t T = R.red_tiles;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const uint32_t t = threadIdx.x + (uint32_t)i * kRedThreads;
            qv[i] = t < T ? R.part_q[t] : 0.0;
            ev[i] = (tr.tile == 0 && t < T) ? R.part_e[t] : 0.0;
            q2v[i] = (ess && t < T) ? U128{R.part_q2[2 * t + 1], R.part_q2[2 * t]} : U128{0ull, 0ull};
        }
    }

    if (status != 0) return;  // uniform over the work-group
    // The propagation partials of this round have been read (by the
    // reduction): clear the group slots for the next round.
    if (tr.tile == 0)
        for (uint32_t i = threadIdx.x; i < kPartialGroups; i += kRedThreads) {
            R.groups->key[i] = 0ull;
            R.groups->counts[i] = 0ull;
        }
    const double M = key_value(key);
    const bool usable = !bad && key != 0 && M != -__builtin_huge_val();

    double base = 0.0, Qtot = 0.0;
    bool resample = active;
    if (R.fused) {
        // every work-group folds the run's tile sums: total mass and own offset
        // (the sums are meaningless when the round is not usable)
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            qv[i] = usable ? qv[i] : 0.0;
            ev[i] = usable ? ev[i] : 0.0;
        }
        double q_all = 0.0, q_before = 0.0, e_all = 0.0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const uint32_t t = threadIdx.x + (uint32_t)i * kRedThreads;
            q_all += qv[i];
            if (t < tr.tile) q_before += qv[i];
            e_all += ev[i];
        }
        q_all = wave_sum(q_all);
        q_before = wave_sum(q_before);
        e_all = wave_sum(e_all);
        if (lane == 0) {
            s_wave[wave] = q_all;
            s_wave2[wave] = q_before;
            s_wave3[wave] = e_all;
        }
        __syncthreads();
        double S = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) {
            Qtot += s_wave[w];
            base += s_wave2[w];
            S += s_wave3[w];
        }
        if (ess && usable && active) {
            // every work-group reaches the same (exact) decision
            U128 q2{0ull, 0ull};
#pragma unroll
            for (int i = 0; i < kPer; ++i) q2 = add128(q2, q2v[i]);
            q2 = wave_sum(q2);
            __shared__ U128 s_q2[kRedThreads / 64];
            if (lane == 0) s_q2[wave] = q2;
            __syncthreads();
            U128 Q2{0ull, 0ull};
            for (int w = 0; w < kRedThreads / 64; ++w) Q2 = add128(Q2, s_q2[w]);
            resample = ess_says_resample(R.ess_t, N, Qtot, Q2);
        }
        if (tr.tile == 0 && threadIdx.x == 0) finish_round(R, ctl, bad, usable, M, S, active, resample);
        __syncthreads();  // s_wave is reused below
    } else {
        Qtot = ctl->qtot;
        base = usable ? R.prefix[tr.tile] : 0.0;
        resample = active && !carry;
    }
    if (!usable || !resample) return;  // uniform over the work-group

    const double scale = (double)(1ull << grid_bits(N));
    const double rQ = 1.0 / Qtot;
    double q[kRedItems];
    double tsum = 0.0;
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) {
        q[k] = first + k < N ? __builtin_rint(fn::exp(x[k] - M) * scale) : 0.0;
        tsum += q[k];
    }
    // inclusive scan of thread sums across the work-group (exact: integer-valued)
    const double incl = wave_incl_scan<OpAddF64>(tsum);
    __shared__ uint32_t s_c[kTileRed];
    __shared__ uint32_t s_o0;
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    double before = base;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    double W = before + (incl - tsum);  // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) {
        W += q[k];
        s_c[threadIdx.x * kRedItems + k] = offspring_before(W, Qtot, rQ, U, N);
    }
    if (threadIdx.x == 0) s_o0 = offspring_before(base, Qtot, rQ, U, N);
    __syncthreads();
    const uint32_t count = (N - tile0) < (uint32_t)kTileRed ? (N - tile0) : (uint32_t)kTileRed;
    const uint32_t o0 = s_o0;
    const uint32_t o1 = s_c[count - 1];
    // Output slot jj descends from the first particle of the tile whose
    // running offspring count exceeds jj. Each particle with offspring marks
    // the first slot of its range with its index + 1 in an LDS window of up
    // to kWindow slots; an inclusive prefix maximum over the window then
    // gives every slot its ancestor (a slot between two marks belongs to the
    // last particle that started at or before it), and the window is copied
    // out with coalesced stores. The work is the same for every thread
    // whatever the weights. A tile with more slots than the window takes
    // several windows, each starting from the last ancestor of the previous.
    constexpr uint32_t kWindow = 4096;
    __shared__ uint32_t s_win[kWindow + kWindow / 16];
    __shared__ uint32_t s_segmax[kRedThreads / 64];
    auto at = [](uint32_t i) { return i + (i >> 4); };  // padding against bank conflicts
    uint32_t prev = 0;  // ancestor (+ 1) of the slot before the window
    for (uint32_t w0 = o0; w0 < o1; w0 += kWindow) {
        const uint32_t len = (o1 - w0) < kWindow ? (o1 - w0) : kWindow;
        for (uint32_t i = threadIdx.x; i < len; i += kRedThreads) s_win[at(i)] = 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRedItems; ++k) {
            const uint32_t idx = threadIdx.x * kRedItems + (uint32_t)k;
            if (idx < count) {
                const uint32_t before = idx == 0 ? o0 : s_c[idx - 1];
                const uint32_t after = s_c[idx];
                if (after > before && before >= w0 && before - w0 < len) s_win[at(before - w0)] = idx + 1u;
            }
        }
        __syncthreads();
        // thread t scans slots [t seg, (t + 1) seg) of the window
        const uint32_t seg = (len + kRedThreads - 1) / kRedThreads;
        const uint32_t s0 = threadIdx.x * seg;
        uint32_t m = 0;
        for (uint32_t j = 0; j < seg; ++j)
            if (s0 + j < len) m = s_win[at(s0 + j)] > m ? s_win[at(s0 + j)] : m;
        const uint32_t incl = wave_incl_scan<OpMaxU32>(m);
        if (lane == 63) s_segmax[wave] = incl;
        __syncthreads();
        uint32_t run = prev;
        for (int w = 0; w < wave; ++w) run = s_segmax[w] > run ? s_segmax[w] : run;
        const uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, 64);
        if (lane > 0) run = excl > run ? excl : run;
        for (uint32_t j = 0; j < seg; ++j)
            if (s0 + j < len) {
                const uint32_t v = s_win[at(s0 + j)];
                run = v > run ? v : run;
                s_win[at(s0 + j)] = run;
            }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < len; i += kRedThreads) R.anc[w0 + i] = tile0 + s_win[at(i)] - 1u;
        prev = s_win[at(len - 1)];
        __syncthreads();  // the window is reused
    }
}

__global__ __launch_bounds__(kRedThreads) void k_scan_anc_one(const RunDev R)
{
    scan_anc_body(R, TileRef{0u, blockIdx.x});
}

__global__ __launch_bounds__(kRedThreads) void k_scan_anc(const RunDev* __restrict__ runs,
                                                           const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    scan_anc_body(runs[tr.run], tr);
}

// ---------------------------------------------------------------------------
// Batched runs owned by one work-group each.
// ---------------------------------------------------------------------------
// A run of at most kOwnedMaxParticles particles is advanced by one work-group
// through every round of a tick: its propagation tiles, then its reduction
// tiles, then its scan tiles, one after another with the work-group's
// barriers between them, so the run moves at its own pace and costs no launch
// per round. The steps are the bodies the segmented launches run, in an order
// they accept (tile 0, which writes the control block, last), so every run
// gets the same bits either way.
template <int Kind, class Real>
__global__ __launch_bounds__(kRedThreads) void k_batch_owned(const RunDev* __restrict__ runs,
                                                             const uint32_t* __restrict__ ids, uint32_t rounds)
{
    const uint32_t run = ids[blockIdx.x];
    const RunDev& R = runs[run];
    const uint32_t prop_tiles = (R.n + kRedThreads - 1) / kRedThreads;
    for (uint32_t k = 0; k < rounds; ++k) {
        if (uniform_i32(R.ctl->status) != 0) break;  // uniform over the work-group
        for (uint32_t t = 0; t < prop_tiles; ++t) {
            propagate_body<Kind, Real, kRedThreads>(R, t);
            __syncthreads();
        }
        // The group slots were updated by device-scope atomics in L2: drop
        // this compute unit's cached copies before the reduction reads them.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (uint32_t t = R.red_tiles; t-- > 0;) {
            reduce_body(R, TileRef{run, t});
            __syncthreads();
        }
        for (uint32_t t = R.red_tiles; t-- > 0;) {
            scan_anc_body(R, TileRef{run, t});
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Standalone pieces: max of a given weight vector, reads, self-tests, setup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void maxkey_body(const RunDev& R, const TileRef tr)
{
    const uint32_t i = tr.tile * kMaxkeyThreads + threadIdx.x;
    Partial p{0ull, 0u, 0u, 0u};
    if (i < R.n) {
        const double x = R.lw[i];
        if (x != x || x == __builtin_huge_val()) p.bad = 1;
        else p.key = order_key(x);
        p.act = 1;  // standalone resampling always resamples
    }
    const Partial r = block_partial<kMaxkeyThreads>(p);
    if (threadIdx.x == 0) publish_group(R, tr.tile, r);
}

__global__ __launch_bounds__(kMaxkeyThreads) void k_maxkey(const RunDev* __restrict__ runs,
                                                          const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    maxkey_body(runs[tr.run], tr);
}

__global__ __launch_bounds__(kMaxkeyThreads) void k_maxkey_one(const RunDev R)
{
    maxkey_body(R, TileRef{0u, blockIdx.x});
}

// Standalone resampling with caller-provided control memory: the control
// block starts as a fresh run at `round` under `seed`, and the propagation
// group slots start cleared (a kernel, not a memset, so nothing here depends
// on what an earlier call left behind).
__global__ __launch_bounds__(kPartialGroups) void k_resample_prepare(const RunDev R, uint32_t round, uint64_t seed)
{
    R.groups->key[threadIdx.x] = 0ull;
    R.groups->counts[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) {
        RunCtl c{};
        c.round = round;
        c.seed = seed;
        *R.ctl = c;
    }
}

__global__ void k_store_log_z(const RunCtl* __restrict__ ctl, double* __restrict__ out)
{
    if (threadIdx.x == 0) *out = ctl->log_z;
}

// Gathered copy of one array: dst[j] = src[anc[j]] for `levels` level-major rows.
template <class T>
__global__ void k_gather(const T* __restrict__ src, const uint32_t* __restrict__ anc, T* __restrict__ dst,
                         uint64_t n, uint64_t levels, uint64_t stride)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint64_t s = anc ? anc[j] : j;
    for (uint64_t k = 0; k < levels; ++k) dst[k * stride + j] = src[k * stride + s];
}

__global__ void k_selftest_math(int op, const double* __restrict__ in, double* __restrict__ out, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = 0.0;
    switch (op) {
    case 0: r = fn::exp(in[i]); break;
    case 1: r = fn::log(in[i]); break;
    case 2: r = fn::cos2pi(in[i]); break;
    case 3: r = fn::sqrt(in[i]); break;
    case 4: r = Stream::word_to_uniform((uint32_t)in[i]); break;
    case 5:
        r = normal_from(Stream::word_to_uniform((uint32_t)in[2 * i]), Stream::word_to_uniform((uint32_t)in[2 * i + 1]));
        break;
    case 6: {
        Stream s;
        s.start((uint64_t)in[2 * i + 1], (uint32_t)i, 0u, kTagPropagate);
        r = (double)draw_poisson(s, in[2 * i]);
        break;
    }
    case 7: {  // in: (n, p, seed) -> first Binomial(n, p) draw of stream (seed, particle 0)
        Stream s;
        s.start((uint64_t)in[3 * i + 2], 0u, 0u, kTagPropagate);
        r = (double)draw_binomial(s, (long long)in[3 * i], in[3 * i + 1]);
        break;
    }
    case 8: {  // in: (a, b, seed) -> Gamma(a) if b < 0, else Beta(a, b)
        Stream s;
        s.start((uint64_t)in[3 * i + 2], 0u, 0u, kTagPropagate);
        r = in[3 * i + 1] < 0.0 ? draw_gamma(s, in[3 * i]) : draw_beta(s, in[3 * i], in[3 * i + 1]);
        break;
    }
    case 11: {  // in: (a, th, seed) -> Negative Binomial predictive of a Poisson(rate) count, rate ~ Gamma(a, th)
        Stream s;
        s.start((uint64_t)in[3 * i + 2], 0u, 0u, kTagPropagate);
        r = (double)draw_neg_binomial(s, in[3 * i], in[3 * i + 1], 1.0);
        break;
    }
    case 12: {  // in: (a, th, seed) -> Lomax predictive of an Exponential(rate) lifetime
        Stream s;
        s.start((uint64_t)in[3 * i + 2], 0u, 0u, kTagPropagate);
        r = draw_lomax(s, in[3 * i], in[3 * i + 1]);
        break;
    }
    case 13: r = fn::exp<false>(in[i]); break;
    case 14: r = fn::log<false>(in[i]); break;
    case 15: r = fn::cos2pi<false>(in[i]); break;
    case 9: r = log_factorial((long long)in[i]); break;
    case 10: r = log_binomial_pmf((long long)in[3 * i], (long long)in[3 * i + 1], in[3 * i + 2]); break;
    default: r = 0.0;
    }
    out[i] = r;
}

__global__ void k_selftest_philox(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                                  uint32_t* __restrict__ out, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Words4 w = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[2 * i], key[2 * i + 1]);
    out[4 * i] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
}

// Algorithm 1 step 1 again on existing buffers: round 0, zero log Z, new seed.
// (A kernel rather than a memset so that it can sit inside a captured graph.)
__global__ void k_reset(RunDev* run, uint64_t seed)
{
    if (blockIdx.x != 0) return;
    for (uint32_t i = threadIdx.x; i < kPartialGroups; i += blockDim.x) {
        run->groups->key[i] = 0ull;
        run->groups->counts[i] = 0ull;
    }
    if (threadIdx.x != 0) return;
    RunCtl* c = run->ctl;
    c->seed = seed;
    c->maxkey = 0;
    c->block_steps = 0;
    c->log_z = 0.0;
    c->m_cur = 0.0;
    c->qtot = 0.0;
    c->u = 0;
    c->round = 0;
    c->status = 0;
    c->active = 0;
    c->bad = 0;
    c->carry = 0;
    c->resamples = 0;
}

// Derived model constants, computed with the pinned device functions so that
// every weight term has the same bits as on any other conforming evaluator.
__global__ void k_model_setup(ModelDev* m)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    m->ln2 = fn::log(2.0);
    if (m->kind == 0) m->log_w = fn::log(m->p[1]);
    if (m->kind == 1) {
        m->obs_var = m->p[3] * m->p[3];
        m->obs_c = -0.5 * fn::log(fn::kTau * m->obs_var);
    }
    m->ln10 = fn::log(10.0);
    if (m->kind == 2 || m->kind == 3 || m->kind == 5) {
        const int tips = (m->n_nodes + 1) / 2;
        m->log_rho = fn::log(m->p[0]);
        double log_fact = 0.0;
        for (int k = 2; k <= tips; ++k) log_fact = log_fact + fn::log((double)k);
        m->corr = (double)(tips - 1) * m->ln2 - log_fact;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int Kind, class Real>
static hipError_t launch_table_sized(int lanes, const RunDev* runs, const TileRef* tiles, uint32_t n_tiles,
                                     hipStream_t st)
{
    if (lanes == 256) hipLaunchKernelGGL((k_propagate<Kind, Real, 256>), dim3(n_tiles), dim3(256), 0, st, runs, tiles);
    else hipLaunchKernelGGL((k_propagate<Kind, Real, 128>), dim3(n_tiles), dim3(128), 0, st, runs, tiles);
    return hipGetLastError();
}

hipError_t launch_propagate(int kind, int precision, int lanes, const RunDev* runs, const TileRef* tiles,
                            uint32_t n_tiles, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    const bool f32 = precision == 32;
    switch (kind) {
    case 0: return launch_table_sized<0, double>(lanes, runs, tiles, n_tiles, st);
    case 1: return f32 ? launch_table_sized<1, float>(lanes, runs, tiles, n_tiles, st)
                       : launch_table_sized<1, double>(lanes, runs, tiles, n_tiles, st);
    case 2: return f32 ? launch_table_sized<2, float>(lanes, runs, tiles, n_tiles, st)
                       : launch_table_sized<2, double>(lanes, runs, tiles, n_tiles, st);
    case 3: return f32 ? launch_table_sized<3, float>(lanes, runs, tiles, n_tiles, st)
                       : launch_table_sized<3, double>(lanes, runs, tiles, n_tiles, st);
    case 4: return f32 ? launch_table_sized<4, float>(lanes, runs, tiles, n_tiles, st)
                       : launch_table_sized<4, double>(lanes, runs, tiles, n_tiles, st);
    case 6: return launch_table_sized<6, double>(lanes, runs, tiles, n_tiles, st);
    default: return f32 ? launch_table_sized<5, float>(lanes, runs, tiles, n_tiles, st)
                        : launch_table_sized<5, double>(lanes, runs, tiles, n_tiles, st);
    }
}

hipError_t launch_owned(int kind, int precision, const RunDev* runs, const uint32_t* ids, uint32_t n_runs,
                        uint32_t rounds, hipStream_t st)
{
    if (n_runs == 0 || rounds == 0) return hipSuccess;
    const bool f32 = precision == 32;
    const dim3 g(n_runs), b(kRedThreads);
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_batch_owned<0, double>), g, b, 0, st, runs, ids, rounds); break;
    case 1:
        if (f32) hipLaunchKernelGGL((k_batch_owned<1, float>), g, b, 0, st, runs, ids, rounds);
        else hipLaunchKernelGGL((k_batch_owned<1, double>), g, b, 0, st, runs, ids, rounds);
        break;
    case 2:
        if (f32) hipLaunchKernelGGL((k_batch_owned<2, float>), g, b, 0, st, runs, ids, rounds);
        else hipLaunchKernelGGL((k_batch_owned<2, double>), g, b, 0, st, runs, ids, rounds);
        break;
    case 3:
        if (f32) hipLaunchKernelGGL((k_batch_owned<3, float>), g, b, 0, st, runs, ids, rounds);
        else hipLaunchKernelGGL((k_batch_owned<3, double>), g, b, 0, st, runs, ids, rounds);
        break;
    case 4:
        if (f32) hipLaunchKernelGGL((k_batch_owned<4, float>), g, b, 0, st, runs, ids, rounds);
        else hipLaunchKernelGGL((k_batch_owned<4, double>), g, b, 0, st, runs, ids, rounds);
        break;
    case 5:
        if (f32) hipLaunchKernelGGL((k_batch_owned<5, float>), g, b, 0, st, runs, ids, rounds);
        else hipLaunchKernelGGL((k_batch_owned<5, double>), g, b, 0, st, runs, ids, rounds);
        break;
    default: return hipErrorInvalidValue;  // compiled programs take the segmented path
    }
    return hipGetLastError();
}

template <int Kind, class Real>
static hipError_t launch_one_sized(const RunDev& run, hipStream_t st)
{
    const dim3 g(run.prop_tiles);
    if (run.lanes == 256) hipLaunchKernelGGL((k_propagate_one<Kind, Real, 256>), g, dim3(256), 0, st, run);
    else hipLaunchKernelGGL((k_propagate_one<Kind, Real, 128>), g, dim3(128), 0, st, run);
    return hipGetLastError();
}

hipError_t launch_propagate_one(int kind, int precision, const RunDev& run, hipStream_t st)
{
    const bool f32 = precision == 32;
    switch (kind) {
    case 0: return launch_one_sized<0, double>(run, st);
    case 1: return f32 ? launch_one_sized<1, float>(run, st) : launch_one_sized<1, double>(run, st);
    case 2: return f32 ? launch_one_sized<2, float>(run, st) : launch_one_sized<2, double>(run, st);
    case 3: return f32 ? launch_one_sized<3, float>(run, st) : launch_one_sized<3, double>(run, st);
    case 4: return f32 ? launch_one_sized<4, float>(run, st) : launch_one_sized<4, double>(run, st);
    case 6: return launch_one_sized<6, double>(run, st);
    default: return f32 ? launch_one_sized<5, float>(run, st) : launch_one_sized<5, double>(run, st);
    }
}

hipError_t launch_bucket(const RunDev& run, hipStream_t st)
{
    hipLaunchKernelGGL(k_bucket_count, dim3(run.red_tiles), dim3(kRedThreads), 0, st, run);
    hipLaunchKernelGGL(k_bucket_scan, dim3(kBuckets), dim3(kRedThreads), 0, st, run);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(run.red_tiles), dim3(kRedThreads), 0, st, run);
    return hipGetLastError();
}

hipError_t launch_resample_one(const RunDev& run, const RunDev* run_dev, hipStream_t st, int part)
{
    // part: 1 = reduction (+ fold), 2 = scan and ancestors, 3 = both
    if (part & 1) {
        hipLaunchKernelGGL(k_reduce_one, dim3(run.red_tiles), dim3(kRedThreads), 0, st, run);
        if (!run.fused) hipLaunchKernelGGL(k_fold_sums, dim3(1), dim3(kFoldThreads), 0, st, run_dev);
    }
    if (part & 2) hipLaunchKernelGGL(k_scan_anc_one, dim3(run.red_tiles), dim3(kRedThreads), 0, st, run);
    return hipGetLastError();
}

hipError_t launch_reduce(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, uint32_t n_runs,
                         bool any_unfused, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n_tiles), dim3(kRedThreads), 0, st, runs, tiles);
    if (any_unfused) hipLaunchKernelGGL(k_fold_sums, dim3(n_runs), dim3(kFoldThreads), 0, st, runs);
    return hipGetLastError();
}

hipError_t launch_scan_anc(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_anc, dim3(n_tiles), dim3(kRedThreads), 0, st, runs, tiles);
    return hipGetLastError();
}

hipError_t launch_maxkey(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_maxkey, dim3(n_tiles), dim3(kMaxkeyThreads), 0, st, runs, tiles);
    return hipGetLastError();
}

hipError_t launch_resample_weights_one(const RunDev& run, uint32_t round, uint64_t seed, double* log_z_out,
                                       hipStream_t st)
{
    hipLaunchKernelGGL(k_resample_prepare, dim3(1), dim3(kPartialGroups), 0, st, run, round, seed);
    hipLaunchKernelGGL(k_maxkey_one, dim3(run.prop_tiles), dim3(kMaxkeyThreads), 0, st, run);
    hipLaunchKernelGGL(k_reduce_one, dim3(run.red_tiles), dim3(kRedThreads), 0, st, run);
    if (!run.fused) hipLaunchKernelGGL(k_fold_sums_one, dim3(1), dim3(kFoldThreads), 0, st, run);
    hipLaunchKernelGGL(k_scan_anc_one, dim3(run.red_tiles), dim3(kRedThreads), 0, st, run);
    hipLaunchKernelGGL(k_store_log_z, dim3(1), dim3(64), 0, st, run.ctl, log_z_out);
    return hipGetLastError();
}

hipError_t launch_gather(int elem_bytes, const void* src, const uint32_t* anc, void* dst, uint64_t n,
                         uint64_t levels, uint64_t stride, hipStream_t st)
{
    const dim3 b(256), g((unsigned)((n + 255) / 256));
    if (elem_bytes == 1)
        hipLaunchKernelGGL(k_gather<uint8_t>, g, b, 0, st, (const uint8_t*)src, anc, (uint8_t*)dst, n, levels, stride);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_gather<uint32_t>, g, b, 0, st, (const uint32_t*)src, anc, (uint32_t*)dst, n, levels, stride);
    else
        hipLaunchKernelGGL(k_gather<uint64_t>, g, b, 0, st, (const uint64_t*)src, anc, (uint64_t*)dst, n, levels, stride);
    return hipGetLastError();
}

hipError_t launch_selftest_math(int op, const double* in, double* out, uint64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_selftest_math, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, op, in, out, n);
    return hipGetLastError();
}

hipError_t launch_selftest_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_selftest_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ctr, key, out, n);
    return hipGetLastError();
}

hipError_t launch_reset(RunDev* run, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, run, seed);
    return hipGetLastError();
}

hipError_t launch_model_setup(ModelDev* m, hipStream_t st)
{
    hipLaunchKernelGGL(k_model_setup, dim3(1), dim3(64), 0, st, m);
    return hipGetLastError();
}

}  // namespace pcfg
