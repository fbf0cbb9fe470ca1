"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds no part of the SMC method: it only builds the data a run is
conditioned on (observed trees, observation series, request streams) and the
plain model specifications (dicts of parameters) that both the GPU binding and
the CPU checker accept. Random numbers here come from NumPy's PCG64 generator
and never from the method's own Philox streams.

Model specifications (``params`` positions are part of the C interface):

* ``geometric`` (Sec. 2, Fig. 2): params = [p_heads, weight factor];
  ``checkpoint`` = resample after every heads (else one importance-sampling pass).
* ``lgssm`` (eq. (2), Fig. 4): params = [a, b, q_sd, r_sd, m0, s0_sd];
  x_0 ~ N(m0, s0), x_t = a x_{t-1} + b + N(0, q), y_t ~ N(x_t, r).
* ``crbd`` (Appendix B listing): params = [rho, lambda scale, mu scale,
  fixed lambda (>0 fixes it), fixed mu (>=0 fixes it), max hidden events,
  max recursion depth]; priors lambda ~ Gamma(1, scale), mu ~ Gamma(1, scale).
* ``clads``: params = [rho, lambda0 scale, eps lo, eps hi, alpha lo, alpha hi,
  sigma scale, max events, max depth, fixed lambda0 (>0), fixed eps (>=0),
  fixed alpha (>0), fixed sigma (>=0)].

Trees are binary, ultrametric, in preorder with the root at index 0 and the
left subtree before the right one; ``age`` is time before the present.
"""
from __future__ import annotations

import math

import numpy as np

MAX_EVENTS = 10_000
MAX_DEPTH = 32


def yule_tree(n_tips: int, seed: int) -> dict:
    """Rate-1 Yule tree with ``n_tips`` tips, scaled to root age 1.0.

    Forward in time from a root split into two lineages: while there are k < n
    lineages, wait Exp(rate k) and split a uniformly chosen lineage (its left
    daughter keeps the lineage's slot); then wait a final Exp(rate n) to the
    present. Ages are measured back from the present and divided by the root
    age. Returned arrays are in preorder (root 0, left subtree first).
    """
    if n_tips < 2:
        raise ValueError("a tree needs at least two tips")
    rng = np.random.default_rng(seed)
    time = [0.0]                 # birth time of each node's lineage split (internal) / present (tips)
    children: list[tuple[int, int] | None] = [None]
    active = []
    for _ in range(2):
        time.append(0.0)
        children.append(None)
        active.append(len(time) - 1)
    children[0] = (active[0], active[1])
    t = 0.0
    while len(active) < n_tips:
        k = len(active)
        t += rng.exponential(1.0 / k)
        idx = int(rng.integers(k))
        node = active[idx]
        time[node] = t
        a = len(time); time.append(0.0); children.append(None)
        b = len(time); time.append(0.0); children.append(None)
        children[node] = (a, b)
        active[idx] = a
        active.append(b)
    t += rng.exponential(1.0 / n_tips)
    for node in active:
        time[node] = t
    root_age = t - time[0]
    # preorder relabelling
    order = []
    stack = [0]
    while stack:
        v = stack.pop()
        order.append(v)
        ch = children[v]
        if ch is not None:
            stack.append(ch[1])
            stack.append(ch[0])
    new_id = {v: i for i, v in enumerate(order)}
    n_nodes = len(order)
    parent = np.full(n_nodes, -1, dtype=np.int32)
    left = np.full(n_nodes, -1, dtype=np.int32)
    right = np.full(n_nodes, -1, dtype=np.int32)
    age = np.zeros(n_nodes, dtype=np.float64)
    for v in order:
        i = new_id[v]
        age[i] = (t - time[v]) / root_age
        ch = children[v]
        if ch is not None:
            left[i] = new_id[ch[0]]
            right[i] = new_id[ch[1]]
            parent[new_id[ch[0]]] = i
            parent[new_id[ch[1]]] = i
    age[left < 0] = 0.0
    age[0] = 1.0
    return {"parent": parent, "left": left, "right": right, "age": age, "tips": n_tips}


def tree_from_newick_like(spec) -> dict:
    """Tree from nested tuples ``(left, right, age)`` with tips given as ``0.0``
    (their age). Used for tiny hand-made test trees."""
    nodes = []

    def visit(node, par):
        i = len(nodes)
        if isinstance(node, tuple):
            nodes.append([par, -1, -1, float(node[2])])
            nodes[i][1] = visit(node[0], i)
            nodes[i][2] = visit(node[1], i)
        else:
            nodes.append([par, -1, -1, float(node)])
        return i

    visit(spec, -1)
    parent = np.array([n[0] for n in nodes], dtype=np.int32)
    left = np.array([n[1] for n in nodes], dtype=np.int32)
    right = np.array([n[2] for n in nodes], dtype=np.int32)
    age = np.array([n[3] for n in nodes], dtype=np.float64)
    return {"parent": parent, "left": left, "right": right, "age": age,
            "tips": int((left < 0).sum())}


def lgssm_data(T: int, seed: int, a=0.9, b=0.0, q=1.0, r=0.5, m0=0.0, s0=None) -> np.ndarray:
    """Simulate y_1..y_T from the linear-Gaussian model (x_0 ~ N(m0, s0))."""
    if s0 is None:
        s0 = math.sqrt(q * q / (1.0 - a * a))
    rng = np.random.default_rng(seed)
    x = m0 + s0 * rng.standard_normal()
    y = np.empty(T, dtype=np.float64)
    for t in range(T):
        x = a * x + b + q * rng.standard_normal()
        y[t] = x + r * rng.standard_normal()
    return y


def geometric_spec(checkpoint=True, p=0.5, w=1.5) -> dict:
    return {"kind": "geometric", "precision": 64, "checkpoint": bool(checkpoint),
            "params": [p, w]}


def lgssm_spec(y, precision=32, a=0.9, b=0.0, q=1.0, r=0.5, m0=0.0, s0=None) -> dict:
    if s0 is None:
        s0 = math.sqrt(q * q / (1.0 - a * a))
    return {"kind": "lgssm", "precision": precision, "y": np.asarray(y, dtype=np.float64),
            "params": [a, b, q, r, m0, s0]}


def crbd_spec(tree, precision=64, rho=1.0, scale_lambda=1.0, scale_mu=0.5,
              fixed_lambda=0.0, fixed_mu=-1.0, max_events=MAX_EVENTS, max_depth=MAX_DEPTH) -> dict:
    return {"kind": "crbd", "precision": precision, "tree": tree,
            "params": [rho, scale_lambda, scale_mu, fixed_lambda, fixed_mu,
                       float(max_events), float(max_depth)]}


def crbd_ds_spec(tree, precision=64, rho=1.0, scale_lambda=1.0, scale_mu=0.5,
                 max_events=MAX_EVENTS, max_depth=MAX_DEPTH) -> dict:
    """CRBD with static delayed sampling: the Gamma(1, scale) priors of lambda
    and mu are carried as posteriors instead of being sampled. Parameter
    positions as for CRBD (fixed-rate entries unused)."""
    return {"kind": "crbd_ds", "precision": precision, "tree": tree,
            "params": [rho, scale_lambda, scale_mu, -1.0, -1.0, float(max_events), float(max_depth)]}


def clads_spec(tree, precision=32, rho=1.0, scale_l0=1.0, eps=(0.0, 1.0), alpha=(0.8, 1.1),
               scale_sigma=0.2, max_events=MAX_EVENTS, max_depth=MAX_DEPTH,
               fixed_l0=0.0, fixed_eps=-1.0, fixed_alpha=0.0, fixed_sigma=-1.0) -> dict:
    return {"kind": "clads", "precision": precision, "tree": tree,
            "params": [rho, scale_l0, eps[0], eps[1], alpha[0], alpha[1], scale_sigma,
                       float(max_events), float(max_depth), fixed_l0, fixed_eps,
                       fixed_alpha, fixed_sigma]}


SEIR_HUMANS = 7370


def seir_data(T: int, seed: int, n=SEIR_HUMANS, hLambda=0.35, hDelta=0.3, hGamma=0.35, mLambda=0.35,
              mDelta=0.3, rho=0.6, hE=5, hI=6, hR=0, mS=12000, missing=0.05) -> np.ndarray:
    """Synthetic daily counts of reported new cases (the vector-borne disease
    model's observations): one forward simulation of the SEIR dynamics with
    NumPy's generator at the given parameters; a fraction of days is missing
    (-1). Input preparation only, independent of the samplers under test."""
    rng = np.random.default_rng(seed)
    bi = rng.binomial
    hS = n - hE - hI - hR
    mE = mI = mR = 0
    y = np.empty(T, dtype=np.float64)
    z = hI
    for t in range(T):
        if t > 0:
            hN = hS + hE + hI + hR
            hTau = bi(hS, 1.0 - math.exp(-mI / hN))
            dE = bi(hTau, hLambda)
            dI = bi(hE, hDelta)
            dR = bi(hI, hGamma)
            mTau = bi(mS, 1.0 - math.exp(-hI / hN))
            mN = mS + mE + mI + mR
            mdE = bi(mTau, mLambda)
            mdI = bi(mE, mDelta)
            hS, hE, hI, hR = hS - dE, hE + dE - dI, hI + dI - dR, hR + dR
            mS, mE, mI = mS - mdE, mE + mdE - mdI, mI + mdI
            mS, mE, mI, mR = bi(mS, 6 / 7), bi(mE, 6 / 7), bi(mI, 6 / 7), bi(mR, 6 / 7)
            mS += bi(mN, 1 / 7)
            z += dI
        if rng.random() < missing and t > 0:
            y[t] = -1.0
        else:
            y[t] = float(bi(z, rho))
            z = 0
    return y


def seir_spec(y, precision=32, n=SEIR_HUMANS, fixed_rates=None, initial=None) -> dict:
    """Vector-borne disease model (SEIR, Appendix listing). params: n humans,
    fixed rates (hLambda, hDelta, hGamma, mLambda, mDelta, rho; -1 draws from
    the Beta priors), fixed initial (hE, hI, hR, mS; -1 draws them)."""
    rates = list(fixed_rates) if fixed_rates is not None else [-1.0] * 6
    init = list(initial) if initial is not None else [-1.0] * 4
    return {"kind": "seir", "precision": precision, "y": np.asarray(y, dtype=np.float64),
            "params": [float(n)] + [float(v) for v in rates] + [float(v) for v in init]}


def request_stream(n_requests: int, seed: int, rate_per_s: float,
                   tips=(16, 512), log2_particles=(10, 18)) -> list[dict]:
    """Serving workload: Poisson arrivals; each request is CRBD or ClaDS (1/2 each)
    on a fresh Yule tree with round(2^U(log2 lo, log2 hi)) tips and
    N = 2^k particles, k uniform on the integer range."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log2(tips[0]), math.log2(tips[1])
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        kind = "crbd" if rng.random() < 0.5 else "clads"
        n_tips = int(round(2.0 ** rng.uniform(lo, hi)))
        n_tips = min(max(n_tips, tips[0]), tips[1])
        k = int(rng.integers(log2_particles[0], log2_particles[1] + 1))
        tree_seed = int(rng.integers(1 << 31))
        run_seed = int(rng.integers(1 << 62))
        out.append({"id": i, "arrival": t, "kind": kind, "tips": n_tips, "n": 1 << k,
                    "tree_seed": tree_seed, "seed": run_seed})
    return out


# ---------------------------------------------------------------------------
# Compiled-program workloads (source text for ppl.compile_program). Numbers are
# written with repr, so both readers of the text get the same doubles.
# ---------------------------------------------------------------------------
def _num(v) -> str:
    return repr(float(v))


def geometric_program(p=0.5, w=1.5) -> str:
    """Sec. 2 / Fig. 2's weighted geometric program, written recursively with
    a resample after every heads: the same draws and weights as the built-in
    geometric model with checkpoints."""
    return f"""(program
  (def flip ()
    (sample h bernoulli {_num(p)})
    (if h ((weight (log {_num(w)})) (resample) (call r flip) (let n (+ r 1)))
          ((let n 1)))
    (return n))
  (def main () (call n flip) (return n)))"""


def lgssm_program(y, a=0.9, b=0.0, q=1.0, r=0.5, m0=0.0, s0=None, tail=False) -> str:
    """Eq. (2) / Fig. 4's state-space model as a recursive program: one step
    per observation, a resample between steps. Written with the built-in
    LGSSM model's operations (x' = (a x + b) + q z; weight obs_c - d^2 / (2 r^2)),
    so at FP64 the two give the same bits. tail=True returns the recursive
    call's result directly (a self tail call), otherwise 0 after it."""
    if s0 is None:
        s0 = math.sqrt(q * q / (1.0 - a * a))
    ys = " ".join(_num(v) for v in y)
    if tail:
        rest = "(if (< (+ t 1) (len y)) ((resample) (call u step (+ t 1) x1) (return u)) ((return 0))))"
    else:
        rest = "(if (< (+ t 1) (len y)) ((resample) (call u step (+ t 1) x1)) ())\n    (return 0))"
    return f"""(program
  (data y {ys})
  (def step (t x)
    (sample x1 normal (+ (* {_num(a)} x) {_num(b)}) {_num(q)})
    (let d (- (at y t) x1))
    (let c (* -0.5 (log (* 6.283185307179586476925286766559005768394 (* {_num(r)} {_num(r)})))))
    (weight (- c (/ (* d d) (* 2.0 (* {_num(r)} {_num(r)})))))
    {rest}
  (def main ()
    (sample x0 normal {_num(m0)} {_num(s0)})
    (call u step 0 x0)
    (return 0)))"""


def hmm_program(ys, p0=0.5, flip=0.2, emit=(0.1, 0.9)) -> str:
    """Two-state hidden Markov model with binary observations: s_0 ~
    Bernoulli(p0), the state flips with probability `flip` each step, and
    y_t ~ Bernoulli(emit[s_t]); a resample between steps."""
    ys_ = " ".join(_num(v) for v in ys)
    e0, e1 = emit
    return f"""(program
  (data ys {ys_})
  (def hmm (t s)
    (sample f bernoulli {_num(flip)})
    (let s2 (+ s (* f (- 1 (* 2 s)))))
    (observe bernoulli (+ {_num(e0)} (* {_num(e1 - e0)} s2)) (at ys t))
    (if (< (+ t 1) (len ys)) ((resample) (call u hmm (+ t 1) s2)) ())
    (return 0))
  (def main ()
    (sample s0 bernoulli {_num(p0)})
    (call u hmm 0 s0)
    (return 0)))"""


def branching_program(obs) -> str:
    """A program with stochastic branching, a recursion that checkpoints at
    every level, a resample-free recursion, an inlined helper and every
    sampler: the recursive `walk` moves x by one of two kernels, then simulates
    a random-depth sum by recursion and observes obs[t]."""
    os_ = " ".join(_num(v) for v in obs)
    return f"""(program
  (data obs {os_})
  (def sq (v) (return (* v v)))
  (def depth_sum (d)
    (if (<= d 0) ((let s 0))
                 ((sample u uniform 0 1) (call r depth_sum (- d 1)) (let s (+ r u))))
    (return s))
  (def walk (t x)
    (sample b bernoulli 0.3)
    (if b ((sample x2 normal x 2.0))
          ((sample g gamma 2.0 0.5) (let x2 (- (* 0.9 x) (* 0.1 g)))))
    (sample k poisson 1.5)
    (call extra depth_sum k)
    (call e sq (- x2 (at obs t)))
    (weight (* -0.05 e))
    (observe normal (at obs t) (+ x2 (* 0.1 extra)) 1.5)
    (sample c binomial 10 0.3)
    (observe poisson 2.0 c)
    (sample bb beta 2.0 3.0)
    (sample ee exponential 2.0)
    (observe exponential 2.0 ee)
    (observe uniform 0 1 bb)
    (if (< (+ t 1) (len obs)) ((resample) (call r walk (+ t 1) x2)) ((let r x2)))
    (return r))
  (def main ()
    (sample x0 normal 0 1)
    (call r walk 0 x0)
    (return r)))"""


def hmm_observations(T: int, seed: int, p0=0.5, flip=0.2, emit=(0.1, 0.9)) -> list:
    """Binary observations simulated from hmm_program's model."""
    rng = np.random.default_rng(seed)
    s = int(rng.random() < p0)
    ys = []
    for _ in range(T):
        if rng.random() < flip:
            s = 1 - s
        ys.append(float(rng.random() < emit[s]))
    return ys


def branching_observations(T: int, seed: int) -> list:
    """Observations for branching_program: a slow random walk, rounded to 1/8."""
    rng = np.random.default_rng(seed)
    x, out = 0.0, []
    for _ in range(T):
        x = 0.9 * x + rng.normal(0.0, 0.7)
        out.append(round(x * 8.0) / 8.0)
    return out


def regime_program(obs, draws: int = 24) -> str:
    """A regime-switching program whose checkpoints sit inside the branches:
    each step draws a regime, resamples inside that regime's branch, then does
    the regime's work (`draws` Gamma draws, inlined) before observing obs[t].
    After resampling, the particles of a wavefront resume at two different
    blocks, so it exercises block bucketing."""
    os_ = " ".join(_num(v) for v in obs)

    def gammas(shape, scale):
        lines = ["(let s 0)"]
        for _ in range(draws):
            lines += [f"(sample g gamma {_num(shape)} {_num(scale)})", "(let s (+ s g))"]
        return "\n    ".join(lines) + "\n    (return s)"

    return f"""(program
  (data obs {os_})
  (def work_a (x)
    {gammas(3.0, 1.0)})
  (def work_b (x)
    {gammas(6.0, 0.5)})
  (def step (t x)
    (sample r bernoulli 0.5)
    (if r ((resample) (call s work_a x) (let x2 (+ (* 0.5 x) (* 0.02 s))))
          ((resample) (call s work_b x) (let x2 (- (* 0.5 x) (* 0.02 s)))))
    (observe normal (at obs t) x2 1.0)
    (if (< (+ t 1) (len obs)) ((call u step (+ t 1) x2)) ((let u 0)))
    (return u))
  (def main ()
    (sample x0 normal 0 1)
    (call u step 0 x0)
    (return u)))"""


def crbd_program(tree, rho=1.0, scale_lambda=1.0, scale_mu=0.5, fixed=None) -> str:
    """The CRBD model of the Appendix listing as a CorePPL-style program for
    the compiler: priors lambda ~ Gamma(1, scale_lambda), mu ~ Gamma(1, scale_mu)
    (or fixed (lambda, mu)), the correction weight (n - 1) log 2 - log n!, then a
    walk over the tree (preorder, left subtree first) that weighs every branch
    by its survival, the observed speciation or tip, and the hidden
    speciations that must go undetected, with a resample after each branch.
    The tree is data: left/right children (-1 at tips) and ages."""
    left = " ".join(str(int(v)) for v in tree["left"])
    right = " ".join(str(int(v)) for v in tree["right"])
    age = " ".join(_num(v) for v in tree["age"])
    tips = sum(1 for v in tree["left"] if v < 0)
    if fixed is None:
        prior = (f"(sample lam gamma 1.0 {_num(scale_lambda)})\n"
                 f"    (sample mu gamma 1.0 {_num(scale_mu)})")
    else:
        prior = f"(let lam {_num(fixed[0])})\n    (let mu {_num(fixed[1])})"
    return f"""(program
  (data left {left})
  (data right {right})
  (data age {age})
  (def iter (n start blen lam mu rho)
    (if (== n 0) ((return 1))
        ((sample et uniform (- start blen) start)
         (call u undetected et lam mu rho)
         (if u ((call r iter (- n 1) start blen lam mu rho) (return r)) ((return 0))))))
  (def undetected (start lam mu rho)
    (sample dur exponential mu)
    (if (> dur start) ((sample b bernoulli rho) (let c b)) ((let c 0)))
    (if c ((return 0))
        ((if (< dur start) ((let bl dur)) ((let bl start)))
         (sample n poisson (* lam bl))
         (call r iter n start bl lam mu rho)
         (return r))))
  (def simbranch (n start stop lam mu rho)
    (if (== n 0) ((return 0))
        ((sample ct uniform stop start)
         (call u undetected ct lam mu rho)
         (if u ((call v simbranch (- n 1) start stop lam mu rho) (return (+ v (log 2))))
               ((return (neg inf)))))))
  (def simtree (node parent lam mu rho)
    (let lp1 (* (neg mu) (- (at age parent) (at age node))))
    (if (>= (at left node) 0) ((let lp2 (log lam))) ((let lp2 (log rho))))
    (let st (at age parent))
    (let sp (at age node))
    (sample n poisson (* lam (- st sp)))
    (call lp3 simbranch n st sp lam mu rho)
    (weight (+ lp1 (+ lp2 lp3)))
    (resample)
    (if (>= (at left node) 0)
        ((call a simtree (at left node) node lam mu rho) (call b simtree (at right node) node lam mu rho))
        ())
    (return 0))
  (def lnfact (i k acc)
    (if (> i k) ((return acc)) ((call r lnfact (+ i 1) k (+ acc (log i))) (return r))))
  (def main ()
    {prior}
    (call lf lnfact 2 {tips} 0)
    (weight (- (* {tips - 1} (log 2)) lf))
    (resample)
    (call a simtree (at left 0) 0 lam mu {_num(rho)})
    (call b simtree (at right 0) 0 lam mu {_num(rho)})
    (return lam)))"""


def seir_program(y, n=SEIR_HUMANS) -> str:
    """The vector-borne disease model of the Appendix listing as a program for
    the compiler, with the built-in SEIR model's draw order and arithmetic
    (priors, initial counts, then one day per round: human transitions, then
    mosquito transitions, survival and births, and the reported-case
    observation), so at FP64 the two give the same bits. Each day resamples
    first, so the day's new counts pass straight into the next day's call,
    a self tail call: the stack stays at main's frame plus one day frame."""
    ys = " ".join(_num(v) for v in y)
    return f"""(program
  (data y {ys})
  (def day (t hS hE hI hR mS mE mI mR z hl hd hg ml md rho)
    (resample)
    (let hN (+ (+ (+ hS hE) hI) hR))
    (sample hTau binomial hS (- 1 (exp (neg (/ mI hN)))))
    (sample hDE binomial hTau hl)
    (sample hDI binomial hE hd)
    (sample hDR binomial hI hg)
    (sample mTau binomial mS (- 1 (exp (neg (/ hI hN)))))
    (let mN (+ (+ (+ mS mE) mI) mR))
    (sample mDE binomial mTau ml)
    (sample mDI binomial mE md)
    (sample mDR binomial mI 0)
    (sample mS2 binomial (- mS mDE) (/ 6.0 7.0))
    (sample mE2 binomial (- (+ mE mDE) mDI) (/ 6.0 7.0))
    (sample mI2 binomial (- (+ mI mDI) mDR) (/ 6.0 7.0))
    (sample mR2 binomial (+ mR mDR) (/ 6.0 7.0))
    (sample mDS binomial mN (/ 1.0 7.0))
    (let z2 (+ z hDI))
    (if (!= (at y t) -1) ((observe binomial z2 rho (at y t)) (let z2 0)) ())
    (if (< (+ t 1) (len y))
        ((call u day (+ t 1) (- hS hDE) (- (+ hE hDE) hDI) (- (+ hI hDI) hDR) (+ hR hDR)
               (+ mS2 mDS) mE2 mI2 mR2 z2 hl hd hg ml md rho)
         (return u))
        ((return 0))))
  (def main ()
    (sample hl beta 1.0 1.0)
    (sample hd beta (+ 1.0 (/ 2.0 4.4)) (- 3.0 (/ 2.0 4.4)))
    (sample hg beta (+ 1.0 (/ 2.0 4.5)) (- 3.0 (/ 2.0 4.5)))
    (sample ml beta 1.0 1.0)
    (sample md beta (+ 1.0 (/ 2.0 6.5)) (- 3.0 (/ 2.0 6.5)))
    (sample rho beta 1.0 1.0)
    (sample k poisson 5.0)
    (let hI (+ 1 k))
    (sample hE poisson 5.0)
    (sample u uniform 0.0 (+ (- (- {n} hI) hE) 1))
    (let hR (floor u))
    (sample v uniform -1.0 2.0)
    (let mS (floor (* {n} (exp (* v (log 10))))))
    (let hS (- (- (- {n} hE) hI) hR))
    (let z hI)
    (if (!= (at y 0) -1) ((observe binomial z rho (at y 0)) (let z 0)) ())
    (if (> (len y) 1) ((call w day 1 hS hE hI hR mS 0 0 0 z hl hd hg ml md rho)) ())
    (return 0)))"""
