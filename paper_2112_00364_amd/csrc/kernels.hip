// Round kernels for SMC over PCFGs on gfx950.
//
// One round of Algorithm 1 (Sec. 3.2) is three launches over a table of
// (run, tile) work-groups, so one launch serves any number of runs:
//   k_propagate  Alg. 1 step 2: each lane takes one particle slot j, gathers
//                its (block, state) from the ancestor chosen by the previous
//                resampling (the duplication step of Sec. 3.3 done on read),
//                runs blocks until a checkpoint or b_stop and writes block,
//                state and log-weight; work-group maxima feed the run's max.
//   k_reduce     sum of exp(lw - M) (for log Z) and of the grid-quantised
//                weights per tile; the last work-group of a run folds the
//                partials in a fixed order, updates log Z (Sec. 3.3), decides
//                termination and prepares the exclusive tile offsets.
//   k_scan_anc   exact FP64 inclusive scan of the quantised weights inside the
//                tile, offspring counts by integer comparison, and the
//                ancestor indices of every output slot the tile owns
//                (systematic resampling, Sec. 3.3).
// Memory is structure-of-arrays (Sec. 3.3): consecutive lanes touch
// consecutive elements of each field.
#include <type_traits>

#include "engine.hpp"
#include "launch.hpp"

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
    int cl = 0;
    while ((1u << cl) < n) cl += 1;  // n <= 2^24
    const int g = 53 - cl;
    return g < 32 ? g : 32;
}

// Grid-quantised weight of log-weight x against the maximum M.
__device__ inline double quantised(double x, double M, double scale)
{
    const double e = fn::exp(x - M);
    return __builtin_rint(e * scale);
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

// Number of output slots j in [0, N) whose systematic position lies below
// cumulative mass W (grid units): #{ j : (j 2^32 + U) Qtot < N W 2^32 }.
__device__ inline uint32_t offspring_before(double W, double Qtot, uint32_t U, uint32_t N)
{
    const unsigned long long w = (unsigned long long)W;
    const unsigned long long qt = (unsigned long long)Qtot;
    const U128 nw = mul128((unsigned long long)N, w);  // < 2^78
    const U128 rhs = U128{(nw.hi << 32) | (nw.lo >> 32), nw.lo << 32};
    auto below = [&](uint32_t j) {
        const unsigned long long pos = ((unsigned long long)j << 32) | (unsigned long long)U;
        return less128(mul128(pos, qt), rhs);
    };
    double y = (double)N * (W / Qtot) - (double)U * 0x1p-32;
    double cf = __builtin_ceil(y);
    uint32_t c = cf <= 0.0 ? 0u : (cf >= (double)N ? N : (uint32_t)cf);
    while (c > 0 && !below(c - 1)) c -= 1;
    while (c < N && below(c)) c += 1;
    return c;
}

template <class T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
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

// One particle slot j of round `round`: gather (block, state) from the
// ancestor src, run blocks until a checkpoint or b_stop, store the results.
// Returns false (storing nothing) when the hidden-lineage stack overflowed.
template <int Kind, class Real, bool kFast>
__device__ inline bool run_particle(const RunDev& R, const ModelDev& m, uint32_t j, uint32_t round, uint8_t& blk,
                                    double& lw, uint32_t& steps)
{
    const ParticleBuf& out = R.buf[round & 1u];
    const ParticleBuf& in = R.buf[(round & 1u) ^ 1u];
    const uint32_t src = round > 0 ? R.anc[j] : j;
    blk = round > 0 ? in.blk[src] : 0;
    lw = 0.0;
    steps = 0;
    Stream s;
    s.start(R.seed, j, round, kTagPropagate);
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
        using Stack = typename std::conditional<kFast, RegFrames<CrbdFrame, kRegFrames>, ArrayFrames<CrbdFrame>>::type;
        typename Crbd<Real>::State st{0.0, 0.0};
        if (round > 0) {
            st.lambda = load_real<Real>(in.real[0], src);
            st.mu = load_real<Real>(in.real[1], src);
        }
        while (blk != kStop) {
            bool ck = false;
            blk = Crbd<Real>::template sim<Stack>(m, round, blk, st, lw, s, ck, overflow);
            if (overflow) return false;
            steps += 1;
            if (ck) break;
        }
        store_real<Real>(out.real[0], j, st.lambda);
        store_real<Real>(out.real[1], j, st.mu);
    } else {
        using Stack =
            typename std::conditional<kFast, RegFrames<ClaDSPending, kRegFrames>, ArrayFrames<ClaDSPending>>::type;
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
            blk = Clads<Real>::template sim<Stack>(m, round, blk, st, lw, s, ck, io, overflow);
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

// Fast pass over every particle: hidden-lineage stacks live in registers. A
// particle whose stack would need more frames is appended to the run's
// overflow list instead and recomputed by k_propagate_deep (its random stream
// is counter-based, so the recomputation draws the same words).
template <int Kind, class Real>
__global__ __launch_bounds__(kPropThreads) void k_propagate(const RunDev* __restrict__ runs,
                                                             const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    const RunDev& R = runs[tr.run];
    RunCtl* ctl = R.ctl;
    if (ctl->status != 0) return;  // uniform over the work-group
    const uint32_t round = ctl->round;
    const ModelDev& m = *R.model;
    const uint32_t j = tr.tile * kPropThreads + threadIdx.x;
    bool counted = false;
    uint8_t blk = kStop;
    double lw = 0.0;
    uint32_t steps = 0;
    if (j < R.n) {
        if (run_particle<Kind, Real, true>(R, m, j, round, blk, lw, steps)) {
            counted = true;
        } else {
            const uint32_t slot = atomicAdd(&ctl->deep_count, 1u);
            R.deep_list[slot] = j;
        }
    }

    // work-group reduction: max key, bad flag, active count, block steps
    unsigned long long key = 0;
    uint32_t bad = 0, act = 0;
    if (counted) {
        if (lw != lw || lw == __builtin_huge_val()) bad = 1;
        else key = order_key(lw);
        act = blk != kStop ? 1u : 0u;
    } else {
        steps = 0;
    }
    key = wave_max_u64(key);
    bad = wave_sum(bad);
    act = wave_sum(act);
    steps = wave_sum(steps);
    __shared__ unsigned long long s_key[kPropThreads / 64];
    __shared__ uint32_t s_bad[kPropThreads / 64], s_act[kPropThreads / 64], s_steps[kPropThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_key[wave] = key;
        s_bad[wave] = bad;
        s_act[wave] = act;
        s_steps[wave] = steps;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = s_key[0];
        uint32_t b = s_bad[0], a = s_act[0], st = s_steps[0];
        for (int w = 1; w < kPropThreads / 64; ++w) {
            k = s_key[w] > k ? s_key[w] : k;
            b += s_bad[w];
            a += s_act[w];
            st += s_steps[w];
        }
        // per-tile partials, folded by k_fold_max (no same-address atomics)
        R.part_key[tr.tile] = k;
        R.part_cnt[tr.tile] = a | (b ? 0x80000000u : 0u);
        R.part_steps[tr.tile] = st;
    }
}

// Particles handed over by the fast pass, recomputed with a stack of
// kMaxDepthCap frames. kDeepGroups work-groups per run stride over the run's
// overflow list (usually a few dozen entries, often none).
constexpr int kDeepGroups = 4;

template <int Kind, class Real>
__global__ __launch_bounds__(kPropThreads) void k_propagate_deep(const RunDev* __restrict__ runs)
{
    const RunDev& R = runs[blockIdx.x / kDeepGroups];
    RunCtl* ctl = R.ctl;
    if (ctl->status != 0 || R.model->kind != Kind || R.model->precision != (int)(8 * sizeof(Real))) return;
    const uint32_t count = ctl->deep_count;
    if (count == 0) return;  // uniform: k_fold_max ignores the deep partials then
    const uint32_t round = ctl->round;
    const uint32_t g = blockIdx.x % kDeepGroups;
    unsigned long long key = 0;
    uint32_t bad = 0, act = 0, steps_all = 0;
    for (uint32_t i = g * kPropThreads + threadIdx.x; i < count; i += kDeepGroups * kPropThreads) {
        const uint32_t j = R.deep_list[i];
        uint8_t blk;
        double lw;
        uint32_t steps;
        run_particle<Kind, Real, false>(R, *R.model, j, round, blk, lw, steps);
        if (lw != lw || lw == __builtin_huge_val()) bad = 1;
        else {
            const unsigned long long kk = order_key(lw);
            key = kk > key ? kk : key;
        }
        act += blk != kStop ? 1u : 0u;
        steps_all += steps;
    }
    key = wave_max_u64(key);
    bad = wave_sum(bad);
    act = wave_sum(act);
    steps_all = wave_sum(steps_all);
    __shared__ unsigned long long s_key[kPropThreads / 64];
    __shared__ uint32_t s_bad[kPropThreads / 64], s_act[kPropThreads / 64], s_steps[kPropThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_key[wave] = key;
        s_bad[wave] = bad;
        s_act[wave] = act;
        s_steps[wave] = steps_all;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = s_key[0];
        uint32_t b = s_bad[0], a = s_act[0], st = s_steps[0];
        for (int w = 1; w < kPropThreads / 64; ++w) {
            k = s_key[w] > k ? s_key[w] : k;
            b += s_bad[w];
            a += s_act[w];
            st += s_steps[w];
        }
        ctl->deep_key[g] = k;
        ctl->deep_cnt[g] = a | (b ? 0x80000000u : 0u);
        ctl->deep_steps[g] = st;
    }
}

// One work-group per run folds the propagation partials: M (as a key), the
// NaN flag, the number of active particles and the block steps of the round.
constexpr int kFoldThreads = 1024;

__global__ __launch_bounds__(kFoldThreads) void k_fold_max(const RunDev* __restrict__ runs)
{
    const RunDev& R = runs[blockIdx.x];
    RunCtl* ctl = R.ctl;
    if (ctl->status != 0) return;
    unsigned long long key = 0;
    uint32_t bad = 0, act = 0, steps = 0;
    for (uint32_t t = threadIdx.x; t < R.prop_tiles; t += kFoldThreads) {
        const unsigned long long k = R.part_key[t];
        const uint32_t c = R.part_cnt[t];
        key = k > key ? k : key;
        act += c & 0x7fffffffu;
        bad |= c >> 31;
        steps += R.part_steps[t];
    }
    if (ctl->deep_count > 0 && threadIdx.x < kDeepGroups) {
        const unsigned long long k = ctl->deep_key[threadIdx.x];
        const uint32_t c = ctl->deep_cnt[threadIdx.x];
        key = k > key ? k : key;
        act += c & 0x7fffffffu;
        bad |= c >> 31;
        steps += ctl->deep_steps[threadIdx.x];
    }
    key = wave_max_u64(key);
    bad = wave_sum(bad);
    act = wave_sum(act);
    steps = wave_sum(steps);
    __shared__ unsigned long long s_key[kFoldThreads / 64];
    __shared__ uint32_t s_bad[kFoldThreads / 64], s_act[kFoldThreads / 64], s_steps[kFoldThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_key[wave] = key;
        s_bad[wave] = bad;
        s_act[wave] = act;
        s_steps[wave] = steps;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = 0;
        uint32_t b = 0, a = 0;
        unsigned long long st = 0;
        for (int w = 0; w < kFoldThreads / 64; ++w) {
            k = s_key[w] > k ? s_key[w] : k;
            b += s_bad[w];
            a += s_act[w];
            st += s_steps[w];
        }
        ctl->maxkey = k;
        ctl->bad = b ? 1u : 0u;
        ctl->active = a;
        ctl->block_steps += st;
    }
}

// ---------------------------------------------------------------------------
// Reduction: per-tile sums, then the run's last work-group finalises.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRedThreads) void k_reduce(const RunDev* __restrict__ runs,
                                                         const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    const RunDev& R = runs[tr.run];
    const RunCtl* ctl = R.ctl;
    if (ctl->status != 0 || ctl->bad != 0) return;
    const double M = key_value(ctl->maxkey);
    if (ctl->maxkey == 0 || M == -__builtin_huge_val()) return;
    const double scale = (double)(1ull << grid_bits(R.n));
    double sq = 0.0, se = 0.0;
    const uint32_t base = tr.tile * kTileRed + threadIdx.x * kRedItems;
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) {
        const uint32_t i = base + k;
        if (i < R.n) {
            const double e = fn::exp(R.lw[i] - M);
            se += e;
            sq += __builtin_rint(e * scale);
        }
    }
    sq = wave_sum(sq);
    se = wave_sum(se);
    __shared__ double s_q[kRedThreads / 64], s_e[kRedThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_q[wave] = sq;
        s_e[wave] = se;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double q = s_q[0], e = s_e[0];
        for (int w = 1; w < kRedThreads / 64; ++w) {
            q += s_q[w];
            e += s_e[w];
        }
        R.part_q[tr.tile] = q;
        R.part_e[tr.tile] = e;
    }
}

// One work-group per run: fold the tile sums in tile order, write each tile's
// exclusive offset in grid units (exact in FP64), update log Z (Sec. 3.3),
// decide termination and draw the round's resampling offset word.
__global__ __launch_bounds__(kFoldThreads) void k_fold_sums(const RunDev* __restrict__ runs)
{
    const RunDev& R = runs[blockIdx.x];
    RunCtl* ctl = R.ctl;
    if (ctl->status != 0) return;
    const bool bad = ctl->bad != 0;
    const double M = key_value(ctl->maxkey);
    const bool usable = !bad && ctl->maxkey != 0 && M != -__builtin_huge_val();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t T = R.red_tiles;
    const uint32_t per = (T + kFoldThreads - 1) / kFoldThreads;
    const uint32_t t0 = threadIdx.x * per;
    const uint32_t t1 = t0 + per < T ? t0 + per : T;
    double q_local = 0.0, e_local = 0.0;
    if (usable)
        for (uint32_t t = t0; t < t1; ++t) {
            q_local += R.part_q[t];
            e_local += R.part_e[t];
        }
    double q_incl = q_local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(q_incl, off, 64);
        if (lane >= off) q_incl += o;
    }
    const double e_wave = wave_sum(e_local);
    __shared__ double s_qw[kFoldThreads / 64], s_ew[kFoldThreads / 64];
    if (lane == 63) s_qw[wave] = q_incl;
    if (lane == 0) s_ew[wave] = e_wave;
    __syncthreads();
    double q_before = 0.0, q_all = 0.0, e_all = 0.0;
    for (int w = 0; w < kFoldThreads / 64; ++w) {
        if (w < wave) q_before += s_qw[w];
        q_all += s_qw[w];
        e_all += s_ew[w];
    }
    if (usable) {
        double run = q_before + (q_incl - q_local);
        for (uint32_t t = t0; t < t1; ++t) {
            R.prefix[t] = run;
            run += R.part_q[t];
        }
    }
    if (threadIdx.x == 0) {
        const uint32_t round = ctl->round;
        if (bad) {
            ctl->status = -5;  // SMC_ERR_NAN
        } else if (!usable) {
            ctl->log_z = -__builtin_huge_val();
            ctl->status = -6;  // SMC_DEGENERATE
        } else {
            ctl->log_z = ctl->log_z + ((M + fn::log(e_all)) - fn::log((double)R.n));
            if (ctl->active == 0) {
                ctl->status = 1;  // SMC_FINISHED
            } else {
                ctl->m_cur = M;
                ctl->qtot = q_all;
                ctl->u = philox10(0u, 0u, round, kTagResample, (uint32_t)R.seed, (uint32_t)(R.seed >> 32)).w0;
                ctl->round = round + 1;
            }
        }
        ctl->deep_count = 0;
    }
}

// ---------------------------------------------------------------------------
// Exact scan + systematic ancestors for the output slots owned by each tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRedThreads) void k_scan_anc(const RunDev* __restrict__ runs,
                                                           const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    const RunDev& R = runs[tr.run];
    const RunCtl* ctl = R.ctl;
    if (ctl->status != 0) return;
    const double M = ctl->m_cur;
    const double Qtot = ctl->qtot;
    const uint32_t U = ctl->u;
    const uint32_t N = R.n;
    const double scale = (double)(1ull << grid_bits(N));
    const double base = R.prefix[tr.tile];
    const uint32_t tile0 = tr.tile * kTileRed;
    const uint32_t first = tile0 + threadIdx.x * kRedItems;

    double q[kRedItems];
    double tsum = 0.0;
#pragma unroll
    for (int k = 0; k < kRedItems; ++k) {
        const uint32_t i = first + k;
        q[k] = i < N ? quantised(R.lw[i], M, scale) : 0.0;
        tsum += q[k];
    }
    // inclusive scan of thread sums across the work-group
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double incl = tsum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    __shared__ double s_wave[kRedThreads / 64];
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
        s_c[threadIdx.x * kRedItems + k] = offspring_before(W, Qtot, U, N);
    }
    if (threadIdx.x == 0) s_o0 = offspring_before(base, Qtot, U, N);
    __syncthreads();
    const uint32_t count = (N - tile0) < (uint32_t)kTileRed ? (N - tile0) : (uint32_t)kTileRed;
    const uint32_t o0 = s_o0;
    const uint32_t o1 = s_c[count - 1];
    for (uint32_t j = o0 + threadIdx.x; j < o1; j += kRedThreads) {
        uint32_t lo = 0, hi = count - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_c[mid] > j) hi = mid;
            else lo = mid + 1;
        }
        R.anc[j] = tile0 + lo;
    }
}

// ---------------------------------------------------------------------------
// Standalone pieces: max of a given weight vector, reads, self-tests.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPropThreads) void k_maxkey(const RunDev* __restrict__ runs,
                                                          const TileRef* __restrict__ tiles)
{
    const TileRef tr = tiles[blockIdx.x];
    const RunDev& R = runs[tr.run];
    const uint32_t i = tr.tile * kPropThreads + threadIdx.x;
    unsigned long long key = 0;
    uint32_t bad = 0;
    if (i < R.n) {
        const double x = R.lw[i];
        if (x != x || x == __builtin_huge_val()) bad = 1;
        else key = order_key(x);
    }
    key = wave_max_u64(key);
    bad = wave_sum(bad);
    __shared__ unsigned long long s_key[kPropThreads / 64];
    __shared__ uint32_t s_bad[kPropThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s_key[wave] = key;
        s_bad[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = 0;
        uint32_t b = 0;
        for (int w = 0; w < kPropThreads / 64; ++w) {
            k = s_key[w] > k ? s_key[w] : k;
            b += s_bad[w];
        }
        R.part_key[tr.tile] = k;
        R.part_cnt[tr.tile] = 1u | (b ? 0x80000000u : 0u);  // standalone resampling always resamples
        R.part_steps[tr.tile] = 0;
    }
}

// Gathered copy of one array: dst[j] = src[anc[j]] (elements of `bytes` bytes).
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
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    run->seed = seed;
    RunCtl* c = run->ctl;
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
    c->deep_count = 0;
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
    if (m->kind == 2 || m->kind == 3) {
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
hipError_t launch_propagate(int kind, int precision, const RunDev* runs, const TileRef* tiles, uint32_t n_tiles,
                            hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    dim3 g(n_tiles), b(kPropThreads);
    if (kind == 0) hipLaunchKernelGGL((k_propagate<0, double>), g, b, 0, st, runs, tiles);
    else if (kind == 1 && precision == 32) hipLaunchKernelGGL((k_propagate<1, float>), g, b, 0, st, runs, tiles);
    else if (kind == 1) hipLaunchKernelGGL((k_propagate<1, double>), g, b, 0, st, runs, tiles);
    else if (kind == 2 && precision == 32) hipLaunchKernelGGL((k_propagate<2, float>), g, b, 0, st, runs, tiles);
    else if (kind == 2) hipLaunchKernelGGL((k_propagate<2, double>), g, b, 0, st, runs, tiles);
    else if (kind == 3 && precision == 32) hipLaunchKernelGGL((k_propagate<3, float>), g, b, 0, st, runs, tiles);
    else hipLaunchKernelGGL((k_propagate<3, double>), g, b, 0, st, runs, tiles);
    return hipGetLastError();
}

hipError_t launch_propagate_deep(int kind, int precision, const RunDev* runs, uint32_t n_runs, hipStream_t st)
{
    // only the birth-death models have hidden-lineage stacks
    if (n_runs == 0 || kind < 2) return hipSuccess;
    dim3 g(n_runs * kDeepGroups), b(kPropThreads);
    if (kind == 2 && precision == 32) hipLaunchKernelGGL((k_propagate_deep<2, float>), g, b, 0, st, runs);
    else if (kind == 2) hipLaunchKernelGGL((k_propagate_deep<2, double>), g, b, 0, st, runs);
    else if (precision == 32) hipLaunchKernelGGL((k_propagate_deep<3, float>), g, b, 0, st, runs);
    else hipLaunchKernelGGL((k_propagate_deep<3, double>), g, b, 0, st, runs);
    return hipGetLastError();
}

hipError_t launch_fold_max(const RunDev* runs, uint32_t n_runs, hipStream_t st)
{
    if (n_runs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_max, dim3(n_runs), dim3(kFoldThreads), 0, st, runs);
    return hipGetLastError();
}

hipError_t launch_reduce(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, uint32_t n_runs, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n_tiles), dim3(kRedThreads), 0, st, runs, tiles);
    hipLaunchKernelGGL(k_fold_sums, dim3(n_runs), dim3(kFoldThreads), 0, st, runs);
    return hipGetLastError();
}

hipError_t launch_scan_anc(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_anc, dim3(n_tiles), dim3(kRedThreads), 0, st, runs, tiles);
    return hipGetLastError();
}

hipError_t launch_resample(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, uint32_t n_runs, hipStream_t st)
{
    hipError_t e = launch_reduce(runs, tiles, n_tiles, n_runs, st);
    if (e != hipSuccess) return e;
    return launch_scan_anc(runs, tiles, n_tiles, st);
}

hipError_t launch_maxkey(const RunDev* runs, const TileRef* tiles, uint32_t n_tiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_maxkey, dim3(n_tiles), dim3(kPropThreads), 0, st, runs, tiles);
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
