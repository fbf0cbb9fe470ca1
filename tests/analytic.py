"""Exact targets that the SMC estimates must approach (test helpers, CPU only).

These are independent of both the oracle and the GPU path: each is a closed
form or a textbook recursion of the quantity the paper's models define.

* Weighted geometric program (Sec. 2, Fig. 2): Z = sum_n p^n w^(n-1).
* Linear-Gaussian state-space model (eq. (2), Fig. 4): the Kalman-filter
  evidence p(y_1..y_T).
* Constant-rate birth-death model (Appendix B listing): the expected product
  of the listing's weights for fixed (lambda, mu, rho). Each branch's expected
  factor is D(t_parent)/D(t_child) for the birth-death ODE
  dD/dt = -(lambda+mu) D + 2 lambda E D, whose solution is proportional to
  p1(t) below; tip factors rho cancel against p1(0) = rho, giving
  log L = corr + (n-2) log lambda + 2 log p1(t_root) + sum_{internal i != root} log p1(t_i),
  corr = (n-1) log 2 - log n!.
"""
from __future__ import annotations

import math

import numpy as np


# --- geometric ------------------------------------------------------------------

def geometric_Z(p=0.5, w=1.5):
    """sum_{n>=1} p^n w^(n-1) = (1/w) (1/(1 - p w) - 1)."""
    return (1.0 / w) * (1.0 / (1.0 - p * w) - 1.0)


def geometric_posterior(n, p=0.5, w=1.5):
    return p ** n * w ** (n - 1) / geometric_Z(p, w)


# --- linear-Gaussian state space -------------------------------------------------

def kalman_log_evidence(y, a, b, q, r, m0, s0):
    m, P = m0, s0 * s0
    ll = 0.0
    for yt in y:
        m = a * m + b
        P = a * a * P + q * q
        S = P + r * r
        ll += -0.5 * math.log(2.0 * math.pi * S) - 0.5 * (yt - m) ** 2 / S
        K = P / S
        m = m + K * (yt - m)
        P = (1.0 - K) * P
    return ll


# --- constant-rate birth-death ---------------------------------------------------

def p0(t, lam, mu, rho):
    r = lam - mu
    if abs(r) < 1e-12:
        return 1.0 - rho / (1.0 + rho * lam * t)
    e = math.exp(-r * t)
    return 1.0 - rho * r / (rho * lam + (lam * (1.0 - rho) - mu) * e)


def log_p1(t, lam, mu, rho):
    r = lam - mu
    if abs(r) < 1e-12:
        return math.log(rho) - 2.0 * math.log1p(rho * lam * t)
    # p1 = rho r^2 e^{-rt} / (rho lam + (lam (1-rho) - mu) e^{-rt})^2
    e = math.exp(-r * t)
    den = rho * lam + (lam * (1.0 - rho) - mu) * e
    return math.log(rho) + 2.0 * math.log(abs(r)) - r * t - 2.0 * math.log(abs(den))


def crbd_corr(n_tips):
    return (n_tips - 1) * math.log(2.0) - math.lgamma(n_tips + 1)


def crbd_log_lik(tree, lam, mu, rho=1.0):
    left, age = tree["left"], tree["age"]
    n_tips = int((left < 0).sum())
    ll = crbd_corr(n_tips) + (n_tips - 2) * math.log(lam) + 2.0 * log_p1(age[0], lam, mu, rho)
    for i in range(1, len(age)):
        if left[i] >= 0:
            ll += log_p1(age[i], lam, mu, rho)
    return ll


def crbd_branch_factor_rk4(t_child, t_parent, lam, mu, rho, steps=20000):
    """log D(t_parent)/D(t_child) by RK4 integration of (E, D) from the present.

    dE/dt = mu - (lam+mu) E + lam E^2, E(0) = 1 - rho
    dD/dt = -(lam+mu) D + 2 lam E D,   D(0) = rho  (D rescaled so only ratios matter)
    """
    def f(E, logD):
        return mu - (lam + mu) * E + lam * E * E, -(lam + mu) + 2.0 * lam * E

    def integrate(t_end):
        E, logD = 1.0 - rho, math.log(rho)
        h = t_end / steps
        for _ in range(steps):
            k1 = f(E, logD)
            k2 = f(E + 0.5 * h * k1[0], logD)
            k3 = f(E + 0.5 * h * k2[0], logD)
            k4 = f(E + h * k3[0], logD)
            E += h * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]) / 6.0
            logD += h * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]) / 6.0
        return logD

    return integrate(t_parent) - integrate(t_child)


def crbd_log_marginal(tree, rho=1.0, scale_lambda=1.0, scale_mu=0.5, n_grid=400):
    """log of the integral of L(lambda, mu) against the Gamma(1, scale) priors,
    by Gauss-Legendre quadrature on the prior CDF scale u = 1 - exp(-x/scale)
    (so the prior density is absorbed and the integrand is L(x(u)))."""
    nodes, weights = np.polynomial.legendre.leggauss(n_grid)
    u = 0.5 * (nodes + 1.0)
    w = 0.5 * weights
    lam = -scale_lambda * np.log1p(-u)
    mu = -scale_mu * np.log1p(-u)
    ll = np.empty((n_grid, n_grid))
    for i in range(n_grid):
        for j in range(n_grid):
            ll[i, j] = crbd_log_lik(tree, lam[i], mu[j], rho)
    mx = ll.max()
    return mx + math.log(float((w[:, None] * w[None, :] * np.exp(ll - mx)).sum()))


# --- vector-borne disease (SEIR) model: exact evidence for tiny populations -------------

def _binom_pmf(N, p):
    if N <= 0 or p <= 0.0:
        return [(0, 1.0)]
    if p >= 1.0:
        return [(N, 1.0)]
    return [(k, math.comb(N, k) * p ** k * (1.0 - p) ** (N - k)) for k in range(N + 1)]


def _expand(states, step):
    """states: {tuple: mass}; step(state) yields (new_state, probability)."""
    out = {}
    for s, w in states.items():
        for s2, q in step(s):
            if q > 0.0:
                out[s2] = out.get(s2, 0.0) + w * q
    return out


def seir_exact_log_evidence(y, n, rates, initial):
    """log P(y_0 .. y_{T-1}) of the vector-borne disease model with fixed rates
    (hLambda, hDelta, hGamma, mLambda, mDelta, rho) and fixed initial (hE, hI,
    hR, mS), by the forward algorithm over the joint counts (exact Binomial
    probabilities, one draw at a time, equal states merged). Only feasible for
    a handful of individuals."""
    hL, hD, hG, mL, mD, rho = rates
    hE0, hI0, hR0, mS0 = initial

    def condition(states, t):
        if y[t] < 0:
            return states
        out = {}
        for s, w in states.items():
            z = s[-1]
            k = int(y[t])
            if k > z:
                continue
            q = math.comb(z, k) * rho ** k * (1.0 - rho) ** (z - k)
            s2 = s[:-1] + (0,)
            out[s2] = out.get(s2, 0.0) + w * q
        return out

    # state: (hS, hE, hI, hR, mS, mE, mI, mR, z)
    states = condition({(n - hE0 - hI0 - hR0, hE0, hI0, hR0, mS0, 0, 0, 0, hI0): 1.0}, 0)
    for t in range(1, len(y)):
        # (previous state, draws so far...) as flat tuples
        st = {s + (s[0] + s[1] + s[2] + s[3], s[4] + s[5] + s[6] + s[7]): w for s, w in states.items()}
        # hTau ~ Bin(hS, 1 - exp(-mI/hN)), then dE ~ Bin(hTau, hL)
        st = _expand(st, lambda s: ((s + (k,), q) for k, q in _binom_pmf(s[0], 1.0 - math.exp(-s[6] / s[9]))))
        st = _expand(st, lambda s: ((s[:-1] + (k,), q) for k, q in _binom_pmf(s[-1], hL)))       # dE
        st = _expand(st, lambda s: ((s + (k,), q) for k, q in _binom_pmf(s[1], hD)))             # dI
        st = _expand(st, lambda s: ((s + (k,), q) for k, q in _binom_pmf(s[2], hG)))             # dR
        st = _expand(st, lambda s: ((s + (k,), q) for k, q in _binom_pmf(s[4], 1.0 - math.exp(-s[2] / s[9]))))
        st = _expand(st, lambda s: ((s[:-1] + (k,), q) for k, q in _binom_pmf(s[-1], mL)))       # mdE
        st = _expand(st, lambda s: ((s + (k,), q) for k, q in _binom_pmf(s[5], mD)))             # mdI
        # s = (hS, hE, hI, hR, mS, mE, mI, mR, z, hN, mN, dE, dI, dR, mdE, mdI)
        st = _expand(st, lambda s: [((s[0] - s[11], s[1] + s[11] - s[12], s[2] + s[12] - s[13], s[3] + s[13],
                                      s[4] - s[14], s[5] + s[14] - s[15], s[6] + s[15], s[7],
                                      s[8] + s[12], s[10]), 1.0)])
        # survival of each mosquito class, then births from the previous total
        for idx in (4, 5, 6, 7):
            st = _expand(st, lambda s, i=idx: ((s[:i] + (k,) + s[i + 1:], q)
                                               for k, q in _binom_pmf(s[i], 6.0 / 7.0)))
        st = _expand(st, lambda s: ((s[:4] + (s[4] + k,) + s[5:9], q) for k, q in _binom_pmf(s[9], 1.0 / 7.0)))
        states = condition(st, t)
    total = sum(states.values())
    return math.log(total) if total > 0 else -math.inf
