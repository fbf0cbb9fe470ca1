// Built-in PCFG block tables (Sec. 3.1): for each model, the blocks B, the
// per-particle state S (held in registers while a block runs) and sim, which
// runs one block and returns the successor plus whether a checkpoint follows.
//
// All tree/observation cursors advance exactly once per checkpoint for every
// particle alike, so they are the round number and are not stored per
// particle.
#pragma once

#include "devmath.hpp"

namespace pcfg {

constexpr uint8_t kStop = 255;  // b_stop

// A compiled program (SMC_MODEL_PROGRAM): bytecode blocks, constants and
// data arrays; stack_words is each particle's stack capacity.
struct ProgramDev {
    const unsigned long long* code;
    const uint32_t* block_start;
    const double* consts;
    const double* data;
    const uint32_t* array_start;
    uint32_t n_blocks, n_arrays, stack_words, n_consts;
};

// Constant model data on the device (uploaded by smc_model_register).
struct ModelDev {
    int32_t kind, precision, checkpoint, n_nodes, T, stack_depth;
    const int32_t* parent;
    const int32_t* left;
    const double* age;
    const double* y;
    const int32_t* sp_before;  // ClaDS: pending-stack size when node r is visited
    double p[16];
    // constants derived on the device with the pinned functions
    double ln2, log_rho, corr, log_w, obs_c, obs_var, ln10;
    ProgramDev prog;
};

// ---------------------------------------------------------------------------
// Weighted geometric program (Sec. 2, Fig. 2). State: flips (int).
// ---------------------------------------------------------------------------
struct Geometric {
    static constexpr int kReal = 0, kInt = 1;
    struct State {
        int flips;
    };
    __device__ static inline uint8_t sim(const ModelDev& m, uint32_t /*round*/, uint8_t /*b*/, State& st,
                                         double& lw, Stream& s, bool& ckpt)
    {
        const bool heads = draw_bernoulli(s, m.p[0]);
        st.flips += 1;
        if (heads) {
            lw = lw + m.log_w;
            ckpt = m.checkpoint != 0;
            return 0;
        }
        ckpt = true;
        return kStop;
    }
};

// ---------------------------------------------------------------------------
// Linear-Gaussian state-space model (eq. (2), Fig. 4). State: x.
// Block 0 draws x_0 and jumps to block 1 without a checkpoint; block 1 moves x,
// observes y_t, and checkpoints (b_stop after the last observation).
// ---------------------------------------------------------------------------
template <class Real>
struct Lgssm {
    static constexpr int kReal = 1, kInt = 0;
    struct State {
        double x;
    };
    __device__ static inline uint8_t sim(const ModelDev& m, uint32_t round, uint8_t b, State& st, double& lw,
                                         Stream& s, bool& ckpt)
    {
        if (b == 0) {
            const double z = draw_normal(s);
            st.x = (double)(Real)(m.p[4] + m.p[5] * z);
            ckpt = false;
            return 1;
        }
        const double z = draw_normal(s);
        st.x = (double)(Real)((m.p[0] * st.x + m.p[1]) + m.p[2] * z);
        const double d = m.y[round] - st.x;
        lw = lw + (m.obs_c - (d * d) / (2.0 * m.obs_var));
        ckpt = true;
        return (int)round + 1 == m.T ? kStop : 1;
    }
};

// ---------------------------------------------------------------------------
// Constant-rate birth-death (Appendix B listing). State: lambda, mu.
// Block 0 draws the rates and adds the correction weight; block 1 handles the
// observed branch above node `round` (preorder, left subtree first).
// ---------------------------------------------------------------------------
constexpr int kMaxDepthCap = 32;
constexpr int kRegFrames = 3;  // frames held in registers on the fast path

// Outcome of simulating one hidden lineage.
enum Hidden : int { kDetected = 0, kUndetected = 1, kOverflow = 2 };

// Depth-first frame stacks. RegFrames keeps the K innermost frames in
// registers (every index is a compile-time constant, so no scratch memory is
// needed) and reports full() when a K+1-th frame is asked for; LdsFrames
// holds all kMaxDepthCap frames in LDS.
template <class Frame, int K>
struct RegFrames {
    Frame f[K];
    int depth = 0;
    __device__ inline bool full() const { return depth == K; }
    __device__ inline Frame& top() { return f[0]; }
    __device__ inline void push(const Frame& x)
    {
#pragma unroll
        for (int i = K - 1; i > 0; --i) f[i] = f[i - 1];
        f[0] = x;
        depth += 1;
    }
    __device__ inline void pop()
    {
#pragma unroll
        for (int i = 0; i < K - 1; ++i) f[i] = f[i + 1];
        depth -= 1;
    }
};

// LdsFrames holds up to kMaxDepthCap frames in a caller-provided LDS region
// (one region per wavefront; used for one lane at a time).
template <class Frame>
struct LdsFrames {
    Frame* base;
    int depth = 0;
    __device__ inline bool full() const { return false; }
    __device__ inline Frame& top() { return base[depth - 1]; }
    __device__ inline void push(const Frame& x) { base[depth++] = x; }
    __device__ inline void pop() { depth -= 1; }
};

struct CrbdFrame {
    int remaining;
    double start, length;
};

struct CrbdSim {
    double lambda, mu, rho;
    int events, max_events, max_depth;

    // A hidden lineage born at age t0 goes undetected (crbdGoesUndetected): its
    // lifetime is Exponential(mu); if it outlives the present it is detected
    // with probability rho; along its life it speciates Poisson(lambda * life)
    // times, and each daughter (born at a uniform time) must go undetected too.
    // Evaluated depth-first with an explicit frame stack; any detection, or
    // exceeding the depth or event budget, answers kDetected. kOverflow means
    // the stack ran out of registers before any budget did (the caller then
    // recomputes the particle with a deeper stack).
    template <class Stack>
    __device__ inline int undetected(Stream& s, double t0, Stack& stack)
    {
        stack.depth = 0;
        double enter_at = t0;
        bool entering = true;
        while (true) {
            if (entering) {
                if (stack.depth + 1 > max_depth) return kDetected;
                const double life = draw_exponential(s, mu);
                if (life > enter_at) {
                    if (draw_bernoulli(s, rho)) return kDetected;
                }
                const double len = life < enter_at ? life : enter_at;
                const int n = draw_poisson(s, lambda * len);
                if (n < 0) return kDetected;
                // a lineage without daughters needs no frame: it is done at once
                if (n > 0) {
                    if (stack.full()) return kOverflow;
                    stack.push(CrbdFrame{n, enter_at, len});
                } else if (stack.depth == 0) {
                    return kUndetected;
                }
                entering = false;
            }
            CrbdFrame& top = stack.top();
            if (top.remaining == 0) {
                stack.pop();
                if (stack.depth == 0) return kUndetected;
                continue;
            }
            top.remaining -= 1;
            if (events >= max_events) return kDetected;
            events += 1;
            const double a = top.start - top.length;
            enter_at = draw_uniform(s, a, top.start);
            entering = true;
        }
    }
};

template <class Real>
struct Crbd {
    static constexpr int kReal = 2, kInt = 0;
    struct State {
        double lambda, mu;
    };

    // What a branch block knows before its hidden events are simulated.
    struct Branch {
        double tp, tc;  // ages of the parent and of the node
        double ln1;     // -mu (t_p - t_c): no extinction along the branch
        double ln2;     // log lambda (speciation at an internal node) or log rho (sampled tip)
        int n;          // hidden speciations on the branch (-1: beyond the event cap)
    };

    // First part of a block: the init block entirely, or a branch block up to
    // (and including) the Poisson draw of its hidden speciations.
    __device__ static inline uint8_t begin(const ModelDev& m, uint32_t round, uint8_t b, State& st, double& lw,
                                           Stream& s, Branch& br)
    {
        if (b == 0) {
            const double lambda = m.p[3] > 0.0 ? m.p[3] : draw_gamma1(s, m.p[1]);
            const double mu = m.p[4] >= 0.0 ? m.p[4] : draw_gamma1(s, m.p[2]);
            st.lambda = (double)(Real)lambda;
            st.mu = (double)(Real)mu;
            lw = lw + m.corr;
            br.n = 0;
            br.ln1 = br.ln2 = 0.0;
            return m.n_nodes > 1 ? 1 : kStop;
        }
        const int node = (int)round;
        br.tp = m.age[m.parent[node]];
        br.tc = m.age[node];
        br.ln1 = -st.mu * (br.tp - br.tc);
        br.ln2 = m.left[node] >= 0 ? fn::log(st.lambda) : m.log_rho;
        br.n = draw_poisson(s, st.lambda * (br.tp - br.tc));
        return node + 1 < m.n_nodes ? 1 : kStop;
    }

    // Second part of a branch block (simBranch): the n hidden speciations in
    // order, each at a uniform time on the branch, each side lineage required
    // to go undetected; returns ln3 (or sets overflow).
    template <class Stack>
    __device__ static inline double events(const ModelDev& m, double lambda, double mu, const Branch& br, Stream& s,
                                           bool& overflow, Stack& stack)
    {
        if (br.n < 0) return -__builtin_huge_val();
        double ln3 = 0.0;
        CrbdSim sim{lambda, mu, m.p[0], 0, (int)m.p[5], (int)m.p[6]};
        for (int e = 0; e < br.n; ++e) {
            if (sim.events >= sim.max_events) return -__builtin_huge_val();
            sim.events += 1;
            const double t = draw_uniform(s, br.tc, br.tp);
            const int h = sim.template undetected<Stack>(s, t, stack);
            if (h == kOverflow) {
                overflow = true;
                return 0.0;
            }
            if (h == kDetected) return -__builtin_huge_val();
            ln3 = ln3 + m.ln2;
        }
        return ln3;
    }

    // The whole block: lw += ln1 + (ln2 + ln3).
    template <class Stack>
    __device__ static inline uint8_t sim(const ModelDev& m, uint32_t round, uint8_t b, State& st, double& lw,
                                         Stream& s, bool& ckpt, bool& overflow, Stack& stack)
    {
        ckpt = true;
        Branch br;
        const uint8_t next = begin(m, round, b, st, lw, s, br);
        if (b == 0) return next;
        const double ln3 = events<Stack>(m, st.lambda, st.mu, br, s, overflow, stack);
        if (overflow) return b;
        lw = lw + (br.ln1 + (br.ln2 + ln3));
        return next;
    }
};

// ---------------------------------------------------------------------------
// CRBD with static delayed sampling (the paper's CRBD experiment with
// variance-reducing techniques, Sec. 5.3; the derivation is this library's
// reading). lambda and mu are never sampled: each particle carries their
// Gamma posteriors (shape a, scale th). Branch survival weighs
// -a_mu log(1 + th_mu t), an observed speciation log(a_l th_l); hidden
// speciation counts come from the Negative Binomial predictive and hidden
// lifetimes from the Lomax predictive; each is followed by its conjugate
// update. Program order, caps and detection as in Crbd.
// ---------------------------------------------------------------------------
struct CrbdDsSim {
    double a_l, th_l, a_mu, th_mu, rho;
    int events, max_events, max_depth;

    template <class Stack>
    __device__ inline int undetected(Stream& s, double t0, Stack& stack)
    {
        stack.depth = 0;
        double enter_at = t0;
        bool entering = true;
        while (true) {
            if (entering) {
                if (stack.depth + 1 > max_depth) return kDetected;
                const double life = draw_lomax(s, a_mu, th_mu);
                a_mu = a_mu + 1.0;
                th_mu = th_mu / (1.0 + th_mu * life);
                if (life > enter_at) {
                    if (draw_bernoulli(s, rho)) return kDetected;
                }
                const double len = life < enter_at ? life : enter_at;
                const long long n = draw_neg_binomial(s, a_l, th_l, len);
                if (n < 0) return kDetected;
                a_l = a_l + (double)n;
                th_l = th_l / (1.0 + th_l * len);
                if (n > 0) {
                    if (stack.full()) return kOverflow;
                    stack.push(CrbdFrame{(int)n, enter_at, len});
                } else if (stack.depth == 0) {
                    return kUndetected;
                }
                entering = false;
            }
            CrbdFrame& top = stack.top();
            if (top.remaining == 0) {
                stack.pop();
                if (stack.depth == 0) return kUndetected;
                continue;
            }
            top.remaining -= 1;
            if (events >= max_events) return kDetected;
            events += 1;
            const double a = top.start - top.length;
            enter_at = draw_uniform(s, a, top.start);
            entering = true;
        }
    }
};

template <class Real>
struct CrbdDs {
    static constexpr int kReal = 4, kInt = 0;
    struct State {
        double a_l, th_l, a_mu, th_mu;
    };

    template <class Stack>
    __device__ static inline uint8_t sim(const ModelDev& m, uint32_t round, uint8_t b, State& st, double& lw,
                                         Stream& s, bool& ckpt, bool& overflow, Stack& stack)
    {
        ckpt = true;
        if (b == 0) {
            st.a_l = (double)(Real)1.0;
            st.th_l = (double)(Real)m.p[1];
            st.a_mu = (double)(Real)1.0;
            st.th_mu = (double)(Real)m.p[2];
            lw = lw + m.corr;
            return m.n_nodes > 1 ? 1 : kStop;
        }
        const int node = (int)round;
        CrbdDsSim c{st.a_l, st.th_l, st.a_mu, st.th_mu, m.p[0], 0, (int)m.p[5], (int)m.p[6]};
        const double tp = m.age[m.parent[node]], tc = m.age[node];
        const double len = tp - tc;
        const double ln1 = -c.a_mu * fn::log(1.0 + c.th_mu * len);
        c.th_mu = c.th_mu / (1.0 + c.th_mu * len);
        double ln2 = m.log_rho;
        if (m.left[node] >= 0) {
            ln2 = fn::log(c.a_l * c.th_l);
            c.a_l = c.a_l + 1.0;
        }
        const long long n = draw_neg_binomial(s, c.a_l, c.th_l, len);
        double ln3 = 0.0;
        if (n < 0) {
            ln3 = -__builtin_huge_val();
        } else {
            c.a_l = c.a_l + (double)n;
            c.th_l = c.th_l / (1.0 + c.th_l * len);
            for (long long e = 0; e < n; ++e) {
                if (c.events >= c.max_events) {
                    ln3 = -__builtin_huge_val();
                    break;
                }
                c.events += 1;
                const double t = draw_uniform(s, tc, tp);
                const int h = c.template undetected<Stack>(s, t, stack);
                if (h == kOverflow) {
                    overflow = true;
                    return b;
                }
                if (h == kDetected) {
                    ln3 = -__builtin_huge_val();
                    break;
                }
                ln3 = ln3 + m.ln2;
            }
        }
        st.a_l = (double)(Real)c.a_l;
        st.th_l = (double)(Real)c.th_l;
        st.a_mu = (double)(Real)c.a_mu;
        st.th_mu = (double)(Real)c.th_mu;
        lw = lw + (ln1 + (ln2 + ln3));
        return node + 1 < m.n_nodes ? 1 : kStop;
    }
};

// ---------------------------------------------------------------------------
// Birth-death with cladogenetic rate shifts (ClaDS-style). State: current
// lineage rate lambda, eps, alpha, sigma, plus a stack of pending right-
// daughter rates (its size is the same for every particle: sp_before[round]).
// ---------------------------------------------------------------------------
struct ClaDSPending {
    double start, rate;
    int depth;
};

// ClaDS pending side lineages in device memory: level k of particle slot j at
// k * stride + j (start time and rate in FP64, depth in a byte). Side-lineage
// recursion under ClaDS is routinely deep, so every lane keeps a full
// kMaxDepthCap-level stack here and no lane waits for another.
struct ClaDSGlobalFrames {
    double* start;
    double* rate;
    uint8_t* dep;
    uint64_t stride;
    uint32_t j;
    int depth = 0;
    __device__ inline bool full() const { return false; }
    __device__ inline ClaDSPending top() const
    {
        const uint64_t at = (uint64_t)(depth - 1) * stride + j;
        return ClaDSPending{start[at], rate[at], (int)dep[at]};
    }
    __device__ inline void push(const ClaDSPending& x)
    {
        const uint64_t at = (uint64_t)depth * stride + j;
        start[at] = x.start;
        rate[at] = x.rate;
        dep[at] = (uint8_t)x.depth;
        depth += 1;
    }
    __device__ inline void pop() { depth -= 1; }
};

struct ClaDSSide {
    double eps, log_alpha, sigma, rho;
    int events, max_events, max_depth;

    // A side lineage born at age t0 with rate r0 must die out unobserved: events
    // arrive at rate r (1 + eps); an event is a speciation with probability
    // 1/(1+eps) (both daughters get r * LogNormal(log alpha, sigma)) and an
    // extinction otherwise; reaching the present is detection with prob. rho.
    // Depth-first: the second daughter waits on a stack while the first one's
    // subtree is simulated. Returns kUndetected, kDetected or kOverflow.
    template <class Stack>
    __device__ inline int undetected(Stream& s, double t0, double r0, Stack& stack)
    {
        stack.depth = 0;
        double start = t0, rate = r0;
        int depth = 1;
        while (true) {
            bool lineage_done = false;
            if (depth > max_depth) return kDetected;
            if (events >= max_events) return kDetected;
            events += 1;
            const double w = draw_exponential<false>(s, rate * (1.0 + eps));
            if (start - w <= 0.0) {
                if (draw_bernoulli(s, rho)) return kDetected;
                lineage_done = true;
            } else {
                const double t = start - w;
                if (s.uniform() < 1.0 / (1.0 + eps)) {
                    if (stack.full()) return kOverflow;
                    const double d1 = rate * draw_lognormal<false>(s, log_alpha, sigma);
                    const double d2 = rate * draw_lognormal<false>(s, log_alpha, sigma);
                    stack.push(ClaDSPending{t, d2, depth + 1});
                    start = t;
                    rate = d1;
                    depth = depth + 1;
                } else {
                    lineage_done = true;
                }
            }
            if (lineage_done) {
                if (stack.depth == 0) return kUndetected;
                const ClaDSPending p = stack.top();
                stack.pop();
                start = p.start;
                rate = p.rate;
                depth = p.depth;
            }
        }
    }
};

template <class Real>
struct Clads {
    static constexpr int kReal = 4, kInt = 0;
    struct State {
        double lambda, eps, alpha, sigma;
    };
    // Stack access for the particle: level k of this particle's pending rates.
    struct StackIO {
        const Real* in;   // gathered source (previous buffer, particle src), may be null in round 0
        Real* out;        // this particle's column in the output buffer
        uint64_t stride;  // particles per level
        uint32_t src, dst;
    };
    template <class Stack>
    __device__ static inline uint8_t sim(const ModelDev& m, uint32_t round, uint8_t b, State& st, double& lw,
                                         Stream& s, bool& ckpt, const StackIO& io, bool& overflow, Stack& stack)
    {
        ckpt = true;
        if (b == 0) {
            const double l0 = m.p[9] > 0.0 ? m.p[9] : draw_gamma1<false>(s, m.p[1]);
            const double eps = m.p[10] >= 0.0 ? m.p[10] : draw_uniform(s, m.p[2], m.p[3]);
            const double alpha = m.p[11] > 0.0 ? m.p[11] : draw_uniform(s, m.p[4], m.p[5]);
            const double sigma = m.p[12] >= 0.0 ? m.p[12] : draw_gamma1<false>(s, m.p[6]);
            st.eps = (double)(Real)eps;
            st.alpha = (double)(Real)alpha;
            st.sigma = (double)(Real)sigma;
            lw = lw + m.corr;
            const double log_alpha = fn::log<false>(st.alpha);
            const double left = l0 * draw_lognormal<false>(s, log_alpha, st.sigma);
            const double right = l0 * draw_lognormal<false>(s, log_alpha, st.sigma);
            io.out[io.dst] = (Real)right;  // level 0
            st.lambda = (double)(Real)left;
            return m.n_nodes > 1 ? 1 : kStop;
        }
        const int node = (int)round;
        const int sp = m.sp_before[node];
        const double log_alpha = fn::log<false>(st.alpha);
        ClaDSSide side{st.eps, log_alpha, st.sigma, m.p[0], 0, (int)m.p[7], (int)m.p[8]};
        double lambda = st.lambda;
        double t = m.age[m.parent[node]];
        const double tc = m.age[node];
        double w_acc = lw;
        bool dead = false;
        while (true) {
            if (side.events >= side.max_events) {
                dead = true;
                break;
            }
            side.events += 1;
            const double w = draw_exponential<false>(s, lambda);
            if (t - w <= tc) {
                w_acc = w_acc + (-(st.eps * lambda) * (t - tc));
                break;
            }
            w_acc = w_acc + (-(st.eps * lambda) * w);
            t = t - w;
            const double cont = lambda * draw_lognormal<false>(s, log_alpha, st.sigma);
            const double sider = lambda * draw_lognormal<false>(s, log_alpha, st.sigma);
            const int h = side.template undetected<Stack>(s, t, sider, stack);
            if (h == kOverflow) {
                overflow = true;
                return b;
            }
            if (h == kDetected) {
                dead = true;
                break;
            }
            w_acc = w_acc + m.ln2;
            lambda = cont;
        }
        const bool internal = m.left[node] >= 0;
        // carry the live part of the stack (levels below sp) to this slot
        for (int k = 0; k < sp; ++k) io.out[(uint64_t)k * io.stride + io.dst] = io.in[(uint64_t)k * io.stride + io.src];
        if (dead) {
            w_acc = -__builtin_huge_val();
            if (internal) {
                io.out[(uint64_t)sp * io.stride + io.dst] = (Real)lambda;
                st.lambda = (double)(Real)lambda;
            } else if (sp > 0) {
                st.lambda = (double)io.in[(uint64_t)(sp - 1) * io.stride + io.src];
            }
        } else if (internal) {
            w_acc = w_acc + fn::log<false>(lambda);
            const double left = lambda * draw_lognormal<false>(s, log_alpha, st.sigma);
            const double right = lambda * draw_lognormal<false>(s, log_alpha, st.sigma);
            io.out[(uint64_t)sp * io.stride + io.dst] = (Real)right;
            st.lambda = (double)(Real)left;
        } else {
            w_acc = w_acc + m.log_rho;
            if (sp > 0) st.lambda = (double)io.in[(uint64_t)(sp - 1) * io.stride + io.src];
        }
        lw = w_acc;
        return node + 1 < m.n_nodes ? 1 : kStop;
    }
};

// ---------------------------------------------------------------------------
// Vector-borne disease (SEIR) model of the Appendix listing: human and
// mosquito susceptible / exposed / infectious / recovered counts per day; new
// human cases are observed as Binomial(z, rho), z counting the humans that
// became infectious since the last observed day. Block 0 draws the rates
// (Beta priors, or fixed by the parameters) and the initial counts and
// conditions on y_0; block 1 simulates day t = round and conditions on y_t;
// the last day is followed by b_stop. Reals (storage precision): hLambda,
// hDelta, hGamma, mLambda, mDelta, rho. Counts: hS, hE, hI, hR, mS, mE, mI,
// mR, z. params = {n humans, six fixed rates (< 0 draws), fixed initial hE,
// hI, hR, mS (< 0 draws)}.
// ---------------------------------------------------------------------------
template <class Real>
struct Seir {
    static constexpr int kReal = 6, kInt = 9;
    struct State {
        double r[kReal];
        long long c[kInt];
    };

    __device__ static inline double rate(Stream& s, double fixed, double a, double b)
    {
        return fixed >= 0.0 ? fixed : draw_beta(s, a, b);
    }

    // the listing's condition: accumulate new infectious humans; an observed
    // day weighs Binomial(z, rho) at y_t and restarts the count
    __device__ static inline void condition(const ModelDev& m, int t, State& st, long long new_infectious, double& lw)
    {
        long long z = st.c[8] + new_infectious;
        const long long y = (long long)m.y[t];
        if (y != -1) {
            lw = lw + log_binomial_pmf(y, z, st.r[5]);
            z = 0;
        }
        st.c[8] = z;
    }

    __device__ static inline uint8_t sim(const ModelDev& m, uint32_t round, uint8_t b, State& st, double& lw,
                                         Stream& s, bool& ckpt)
    {
        ckpt = true;
        const long long n = (long long)m.p[0];
        if (b == 0) {
            st.r[0] = (double)(Real)rate(s, m.p[1], 1.0, 1.0);
            st.r[1] = (double)(Real)rate(s, m.p[2], 1.0 + 2.0 / 4.4, 3.0 - 2.0 / 4.4);
            st.r[2] = (double)(Real)rate(s, m.p[3], 1.0 + 2.0 / 4.5, 3.0 - 2.0 / 4.5);
            st.r[3] = (double)(Real)rate(s, m.p[4], 1.0, 1.0);
            st.r[4] = (double)(Real)rate(s, m.p[5], 1.0 + 2.0 / 6.5, 3.0 - 2.0 / 6.5);
            st.r[5] = (double)(Real)rate(s, m.p[6], 1.0, 1.0);
            const long long hI = m.p[8] >= 0.0 ? (long long)m.p[8] : 1 + (long long)draw_poisson(s, 5.0);
            const long long hE = m.p[7] >= 0.0 ? (long long)m.p[7] : (long long)draw_poisson(s, 5.0);
            const long long hR = m.p[9] >= 0.0
                                     ? (long long)m.p[9]
                                     : (long long)__builtin_floor(draw_uniform(s, 0.0, (double)(n - hI - hE + 1)));
            const long long mS = m.p[10] >= 0.0
                                     ? (long long)m.p[10]
                                     : (long long)__builtin_floor((double)n * fn::exp(draw_uniform(s, -1.0, 2.0) * m.ln10));
            st.c[0] = n - hE - hI - hR;
            st.c[1] = hE;
            st.c[2] = hI;
            st.c[3] = hR;
            st.c[4] = mS;
            st.c[5] = st.c[6] = st.c[7] = 0;
            st.c[8] = 0;
            condition(m, 0, st, hI, lw);
            return m.T > 1 ? 1 : kStop;
        }
        const int t = (int)round;
        const double hLambda = st.r[0], hDelta = st.r[1], hGamma = st.r[2];
        const double mLambda = st.r[3], mDelta = st.r[4];
        const double mNu = 1.0 / 7.0, mMu = 6.0 / 7.0, mGamma = 0.0;
        const long long hSP = st.c[0], hEP = st.c[1], hIP = st.c[2], hRP = st.c[3];
        const long long mSP = st.c[4], mEP = st.c[5], mIP = st.c[6], mRP = st.c[7];
        // humans
        const long long hN = hSP + hEP + hIP + hRP;
        const long long hTau = draw_binomial(s, hSP, 1.0 - fn::exp(-((double)mIP / (double)hN)));
        const long long hDeltaE = draw_binomial(s, hTau, hLambda);
        const long long hDeltaI = draw_binomial(s, hEP, hDelta);
        const long long hDeltaR = draw_binomial(s, hIP, hGamma);
        st.c[0] = hSP - hDeltaE;
        st.c[1] = hEP + hDeltaE - hDeltaI;
        st.c[2] = hIP + hDeltaI - hDeltaR;
        st.c[3] = hRP + hDeltaR;
        // mosquitoes
        const long long mTau = draw_binomial(s, mSP, 1.0 - fn::exp(-((double)hIP / (double)hN)));
        const long long mN = mSP + mEP + mIP + mRP;
        const long long mDeltaE = draw_binomial(s, mTau, mLambda);
        const long long mDeltaI = draw_binomial(s, mEP, mDelta);
        const long long mDeltaR = draw_binomial(s, mIP, mGamma);
        long long mS = mSP - mDeltaE;
        long long mE = mEP + mDeltaE - mDeltaI;
        long long mI = mIP + mDeltaI - mDeltaR;
        long long mR = mRP + mDeltaR;
        mS = draw_binomial(s, mS, mMu);
        mE = draw_binomial(s, mE, mMu);
        mI = draw_binomial(s, mI, mMu);
        mR = draw_binomial(s, mR, mMu);
        const long long mDeltaS = draw_binomial(s, mN, mNu);
        st.c[4] = mS + mDeltaS;
        st.c[5] = mE;
        st.c[6] = mI;
        st.c[7] = mR;
        condition(m, t, st, hDeltaI, lw);
        return t + 1 < m.T ? 1 : kStop;
    }
};

}  // namespace pcfg
