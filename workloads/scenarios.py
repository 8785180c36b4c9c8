"""Scenario parameter dictionaries for perishable-inventory value iteration.

Every dictionary has the same keys, whatever the family:

  family      "A" (lead time, FIFO), "B" (two products, one-way substitution, L = 0),
              "B1" (the paper's two-product runs: L = 1, outcome = units issued),
              "C" (weekday demand, random remaining life on arrival)
  m           maximum useful life
  L           lead time (A: >= 1; B and C: 0, the order arrives before demand)
  n_periods   demand periods (7 weekdays for C, else 1)
  a_max       [product 0, product 1] maximum order quantity (product 1 only for B)
  d_max       [product 0, product 1] demand truncation point (tail folded into d_max)
  demand      per product: {"kind": "poisson", "mean": [...]},
              {"kind": "gamma", "mean": [...], "cv": [...]} or
              {"kind": "negbin", "mean": [...], "n": [...]}; one entry per period
  rul_c0, rul_c1  C only: log(p_k(a)/p_1(a)) = c0[k] + c1[k]*a for k = 2..m
              (lists of length m, entry 0 unused and zero)
  subst_rho   B only: probability that a customer of product 0 left unserved
              accepts product 1 instead
  costs       var [2], fixed, hold, short, waste, rev [2]
  gamma       discount factor
  eps         tolerance; the span stopping threshold is eps*(1-gamma)/gamma

The only randomness is `numpy.random.default_rng([config_id, request_id])`.
"""
from __future__ import annotations

import copy

import numpy as np

__all__ = [
    "scenario_a", "scenario_b", "scenario_c", "scenario_a_paper", "PAPER_A_EXPERIMENTS",
    "scenario_c_paper", "PAPER_C_EXPERIMENTS", "PAPER_C_RUL_LARGE", "scenario_b1",
    "scenario_b_paper",
    "PAPER_B_EXPERIMENTS",
    "config0", "config1", "config2",
    "config3", "config_by_index", "serving_mix", "random_values", "sample_indices",
]


def _costs(var=(0.0, 0.0), fixed=0.0, hold=0.0, short=0.0, waste=0.0, rev=(0.0, 0.0)):
    return {"var": [float(var[0]), float(var[1])], "fixed": float(fixed),
            "hold": float(hold), "short": float(short), "waste": float(waste),
            "rev": [float(rev[0]), float(rev[1])]}


def scenario_a(m=2, L=1, a_max=10, d_max=20, demand=None, costs=None, gamma=0.99,
               eps=1e-4, issuing="fifo"):
    """Scenario A (single product, lead time L >= 1, FIFO or LIFO issuing)."""
    assert issuing in ("fifo", "lifo")
    if demand is None:
        demand = {"kind": "poisson", "mean": [4.0]}
    if costs is None:
        costs = _costs(var=(3.0, 0.0), hold=1.0, short=5.0, waste=7.0)
    return {"family": "A", "m": int(m), "L": int(L), "n_periods": 1,
            "a_max": [int(a_max), 0], "d_max": [int(d_max), 0],
            "demand": [copy.deepcopy(demand), {"kind": "none", "mean": [0.0]}],
            "rul_c0": [0.0] * int(m), "rul_c1": [0.0] * int(m), "subst_rho": 0.0,
            "costs": copy.deepcopy(costs), "gamma": float(gamma), "eps": float(eps),
            "issuing": issuing}


def scenario_b(m=3, a_max=(14, 14), d_max=(20, 20), means=(5.0, 4.0), rho=0.5,
               costs=None, gamma=0.99, eps=1e-4):
    """Scenario B (two products, L=0, product 0's unmet demand may take product 1)."""
    if costs is None:
        costs = _costs(var=(0.5, 0.5), rev=(1.0, 1.0))
    return {"family": "B", "m": int(m), "L": 0, "n_periods": 1,
            "a_max": [int(a_max[0]), int(a_max[1])],
            "d_max": [int(d_max[0]), int(d_max[1])],
            "demand": [{"kind": "poisson", "mean": [float(means[0])]},
                       {"kind": "poisson", "mean": [float(means[1])]}],
            "rul_c0": [0.0] * int(m), "rul_c1": [0.0] * int(m), "subst_rho": float(rho),
            "costs": copy.deepcopy(costs), "gamma": float(gamma), "eps": float(eps)}


def scenario_b1(m=2, a_max=(10, 10), means=(5.0, 5.0), rho=0.5, d_max=None, costs=None,
                gamma=1.0, eps=1e-4):
    """Scenario B as the paper runs it: two products, lead time 1 (yesterday's orders
    are in stock as X_m), outcome = units issued, product b's unmet customers accept
    product a with probability rho.  Poisson demand folded at d_max (default
    m * max(a_max) + 2, the paper's table bound)."""
    if costs is None:
        costs = _costs(var=(0.5, 0.5), rev=(1.0, 1.0))
    if d_max is None:
        d_max = m * max(a_max) + 2
    return {"family": "B1", "m": int(m), "L": 1, "n_periods": 1,
            "a_max": [int(a_max[0]), int(a_max[1])], "d_max": [int(d_max), int(d_max)],
            "demand": [{"kind": "poisson", "mean": [float(means[0])]},
                       {"kind": "poisson", "mean": [float(means[1])]}],
            "rul_c0": [0.0] * int(m), "rul_c1": [0.0] * int(m), "subst_rho": float(rho),
            "costs": copy.deepcopy(costs), "gamma": float(gamma), "eps": float(eps)}


# Scenario B experiments of the paper's results tables: (m, experiment) ->
# (mean demand a, b; maximum order a, b).  "P1".."P4" are the settings of the
# comparison with an earlier CUDA implementation, run for exactly 100 sweeps.
PAPER_B_EXPERIMENTS = {
    (2, "1"): ((5.0, 5.0), (10, 10)), (2, "2"): ((7.0, 3.0), (14, 6)),
    (3, "1"): ((5.0, 5.0), (15, 15)), (3, "2"): ((7.0, 3.0), (21, 9)),
    (3, "3"): ((5.0, 5.0), (13, 13)), (3, "4"): ((7.0, 3.0), (20, 4)),
    (2, "P1"): ((5.0, 5.0), (10, 10)), (2, "P2"): ((5.0, 6.0), (10, 12)),
    (2, "P3"): ((6.0, 6.0), (12, 12)), (2, "P4"): ((7.0, 7.0), (13, 13)),
}


def scenario_b_paper(m, exp):
    """Scenario B with the settings the paper fixes for all its experiments (Appendix B
    common-settings table): C_v 0.5 and C_r 1 for both products, rho 0.5, gamma 1,
    eps 1e-4, span stop (the P experiments: 100 sweeps)."""
    means, amax = PAPER_B_EXPERIMENTS[(m, str(exp))]
    return scenario_b1(m=m, a_max=amax, means=means, rho=0.5)


def scenario_c(m=3, a_max=4, d_max=8, n=None, means=None, c0=None, c1=None,
               costs=None, gamma=0.99, eps=1e-4, n_periods=7):
    """Scenario C (weekday negative-binomial demand, random remaining life, L=0)."""
    if n is None:
        n = [5.0] * n_periods
    if means is None:
        means = [4.0] * n_periods
    if c0 is None:
        c0 = [0.0] + [1.0] * (m - 1)
    if c1 is None:
        c1 = [0.0] * m
    if costs is None:
        costs = _costs(fixed=10.0, hold=1.0, short=20.0, waste=5.0)
    return {"family": "C", "m": int(m), "L": 0, "n_periods": int(n_periods),
            "a_max": [int(a_max), 0], "d_max": [int(d_max), 0],
            "demand": [{"kind": "negbin", "mean": [float(x) for x in means],
                        "n": [float(x) for x in n]}, {"kind": "none", "mean": [0.0]}],
            "rul_c0": [float(x) for x in c0], "rul_c1": [float(x) for x in c1],
            "subst_rho": 0.0, "costs": copy.deepcopy(costs), "gamma": float(gamma),
            "eps": float(eps)}


# Scenario A experiments of the paper's results table: (m, experiment, L, C_w, issuing).
# Sizes follow from m and L: (A_max + 1)^(m + L - 1) states, 11 actions, 101 outcomes.
PAPER_A_EXPERIMENTS = [
    (m, e + 1, L, cw, iss)
    for m in (2, 3, 4, 5)
    for e, (L, cw, iss) in enumerate(
        [(L, cw, iss) for L in (1, 2) for cw in (7.0, 10.0) for iss in ("lifo", "fifo")])
]


def scenario_a_paper(m, L, waste, issuing):
    """Scenario A with the settings the paper fixes for all its experiments (Appendix A,
    common-settings table): gamma demand with mean 4 and coefficient of variation 0.5,
    truncated at 100; orders up to 10; C_v 3, C_s 5, C_h 1; gamma 0.99, eps 1e-4.  The
    paper stops these solves with the sup-norm test."""
    return scenario_a(m=m, L=L, a_max=10, d_max=100,
                      demand={"kind": "gamma", "mean": [4.0], "cv": [0.5]},
                      costs=_costs(var=(3.0, 0.0), hold=1.0, short=5.0, waste=waste),
                      gamma=0.99, eps=1e-4, issuing=issuing)


# Scenario C experiments of the paper's results table that fit in memory: m in {3, 5},
# experiment 1 with remaining life on arrival independent of the order (exogenous),
# experiment 2 with it depending on the order quantity (endogenous).  Logit
# coefficients c_0^k, c_1^k for k = 2..m from the paper's useful-life table.
PAPER_C_RUL = {
    (3, 1): ([1.0, 0.5], [0.0, 0.0]),
    (3, 2): ([1.0, 0.5], [0.4, 0.8]),
    (5, 1): ([1.6, 2.6, 2.8, 1.6], [0.0, 0.0, 0.0, 0.0]),
    (5, 2): ([1.9, 3.1, 3.1, 2.5], [-0.03, -0.06, -0.03, -0.09]),
}
PAPER_C_EXPERIMENTS = sorted(PAPER_C_RUL)
# m = 8 (12,607,619,787 states): the paper fits the (s, S) heuristic only
PAPER_C_RUL_LARGE = {
    (8, 1): ([0.8, 1.4, 1.9, 2.3, 1.7, 1.2, 0.8], [0.0] * 7),
    (8, 2): ([0.8, 1.4, 1.9, 2.3, 1.7, 1.2, 0.8],
             [-0.03, -0.04, -0.05, -0.06, -0.07, -0.08, -0.09]),
}
# weekday negative-binomial demand, Monday (tau = 0) to Sunday: successes n, mean delta
PAPER_C_DEMAND_N = [3.5, 11.0, 7.2, 11.1, 5.9, 5.5, 2.2]
PAPER_C_DEMAND_MEAN = [5.7, 6.9, 6.5, 6.2, 5.8, 3.3, 3.4]


def scenario_c_paper(m, exp):
    """Scenario C with the settings the paper fixes for all its experiments (Appendix C
    common-settings, weekday-demand and useful-life tables): demand truncated at 20,
    orders and stock of each remaining life up to 20, C_f 10, C_h 1, C_s 20, C_w 5,
    gamma 0.95, eps 1e-4.  The paper stops these solves with its periodic test; at
    m = 8 (PAPER_C_RUL_LARGE) it only fits and evaluates the (s, S) heuristic."""
    c0, c1 = PAPER_C_RUL[(m, exp)] if (m, exp) in PAPER_C_RUL else PAPER_C_RUL_LARGE[(m, exp)]
    return scenario_c(m=m, a_max=20, d_max=20, n=PAPER_C_DEMAND_N,
                      means=PAPER_C_DEMAND_MEAN, c0=[0.0] + list(c0), c1=[0.0] + list(c1),
                      costs=_costs(fixed=10.0, hold=1.0, short=20.0, waste=5.0),
                      gamma=0.95, eps=1e-4)


def _jitter(rng, x, frac=0.2):
    return float(x) * float(1.0 + rng.uniform(-frac, frac))


def config0():
    """m=2, L=1, order <= 10, Poisson(4) folded at 20, costs 3/5/7/1, gamma 0.99."""
    return scenario_a(m=2, L=1, a_max=10, d_max=20,
                      demand={"kind": "poisson", "mean": [4.0]},
                      costs=_costs(var=(3.0, 0.0), hold=1.0, short=5.0, waste=7.0))


def config1(request_id=0):
    """m=4, L=2, order <= 20, gamma demand (mean 4, CV 1.5) folded at 60, costs x(1+-20%)."""
    rng = np.random.default_rng([1, request_id])
    costs = _costs(var=(_jitter(rng, 3.0), 0.0), short=_jitter(rng, 5.0),
                   waste=_jitter(rng, 7.0), hold=_jitter(rng, 1.0))
    return scenario_a(m=4, L=2, a_max=20, d_max=60,
                      demand={"kind": "gamma", "mean": [4.0], "cv": [1.5]}, costs=costs)


def config2():
    """Two products, m=3, L=0, orders <= 14 each, Poisson(5)/(4) folded at 20, rho 0.5."""
    return scenario_b(m=3, a_max=(14, 14), d_max=(20, 20), means=(5.0, 4.0), rho=0.5)


def config3(request_id=0, a_max=20):
    """Weekday NB demand (n=5, mean ~ U(5,10)) folded at 40, m=5, L=0, RUL logits ~ U(0,3)."""
    rng = np.random.default_rng([3, request_id])
    means = [float(x) for x in rng.uniform(5.0, 10.0, size=7)]
    c0 = [0.0] + [float(x) for x in rng.uniform(0.0, 3.0, size=4)]
    return scenario_c(m=5, a_max=a_max, d_max=40, n=[5.0] * 7, means=means, c0=c0,
                      c1=[0.0] * 5, gamma=0.99)


def config_by_index(i):
    return [config0, config1, config2, config3][i]()


def serving_mix(n_requests=2000, rate_per_s=100.0, seed=4, large_fraction=0.05,
                c_fraction=0.25):
    """Seeded request stream: (arrival_time_s, scenario) pairs.

    70% scenario-A instances of the small family (m in 2..3, costs x(1+-20%)),
    25% scenario-C instances with order cap in 10..20, 5% large scenario-A instances
    (the m=4, L=2, order <= 20 size).  Inter-arrival times are exponential.
    """
    rng = np.random.default_rng([4, seed])
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        u = float(rng.uniform())
        if u < large_fraction:
            sc = config1(request_id=1000 + i)
        elif u < large_fraction + c_fraction:
            sc = config3(request_id=1000 + i, a_max=int(rng.integers(10, 21)))
        else:
            m = int(rng.integers(2, 4))
            costs = _costs(var=(_jitter(rng, 3.0), 0.0), short=_jitter(rng, 5.0),
                           waste=_jitter(rng, 7.0), hold=_jitter(rng, 1.0))
            sc = scenario_a(m=m, L=1, a_max=10, d_max=20,
                            demand={"kind": "poisson", "mean": [4.0]}, costs=costs)
        out.append((t, sc))
    return out


def random_values(n, seed=0, scale=100.0, offset=-1000.0):
    """A seeded FP64 value-function guess of length n (for one-sweep parity)."""
    rng = np.random.default_rng([99, seed])
    return offset + scale * rng.standard_normal(int(n))


def sample_indices(n, k, seed=0):
    """k distinct sorted indices in [0, n), always including 0 and n-1."""
    rng = np.random.default_rng([98, seed])
    k = min(int(k), int(n))
    idx = set(rng.choice(int(n), size=max(k - 2, 0), replace=False).tolist())
    idx.update({0, int(n) - 1})
    return np.array(sorted(idx), dtype=np.int64)
