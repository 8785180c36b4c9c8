"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* PMFs: closed forms (Poisson, exponential = gamma with cv 1, geometric = negative
  binomial with n = 1, softmax ratios), unit mass, folded tails.
* Sizes: the paper's state-count columns (Scenario A and C results tables).
* Transitions: hand-worked examples (tests/golden) and exhaustive agreement with an
  independent unit-by-unit model on small instances.
* Bellman operator: agreement with a dense P(s'|s,a) model built from the unit
  model with scipy probabilities; LP optimum; policy iteration; contraction;
  MacQueen bounds; policy-evaluation fixed point.
* Special cases: the m=1 newsvendor closed form; rho=0 separability of Scenario B;
  weekday invariance of Scenario C.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import optimize, stats

import unit_model as U
import workloads as W
from oracle.oracle import Oracle, demand_pmf, life_probabilities

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_transitions.json")


# ------------------------------------------------------------------ PMFs

def test_poisson_pmf_closed_form_and_fold():
    p = demand_pmf({"kind": "poisson", "mean": [4.0]}, 20)
    for d in range(20):
        assert p[d] == pytest.approx(math.exp(-4.0) * 4.0 ** d / math.factorial(d), rel=1e-13)
    tail = 1.0 - sum(math.exp(-4.0) * 4.0 ** d / math.factorial(d) for d in range(20))
    assert p[20] == pytest.approx(tail, rel=1e-6, abs=1e-16)
    assert p.sum() == pytest.approx(1.0, abs=1e-15)
    assert p[20] == pytest.approx(1.02e-8, rel=0.01)   # tail size quoted for this case


def test_gamma_pmf_exponential_special_case():
    # cv = 1 gives shape 1: F(x) = 1 - exp(-x/mu), discretised with +-1/2
    mu, dmax = 3.0, 15
    p = demand_pmf({"kind": "gamma", "mean": [mu], "cv": [1.0]}, dmax)
    F = lambda x: 0.0 if x <= 0 else 1.0 - math.exp(-x / mu)
    for d in range(dmax):
        assert p[d] == pytest.approx(F(d + 0.5) - F(d - 0.5), rel=1e-12)
    assert p[dmax] == pytest.approx(math.exp(-(dmax - 0.5) / mu), rel=1e-12)
    assert p.sum() == pytest.approx(1.0, abs=1e-15)


def test_gamma_pmf_config1_values():
    p = demand_pmf({"kind": "gamma", "mean": [4.0], "cv": [1.5]}, 60)
    assert p.sum() == pytest.approx(1.0, abs=1e-14)
    # shape 1/1.5^2, scale 4*1.5^2: P(0) = F(1/2)
    assert p[0] == pytest.approx(stats.gamma.cdf(0.5, 1 / 2.25, scale=9.0), rel=1e-13)
    assert p[0] == pytest.approx(0.30721, abs=5e-5)
    assert p[60] == pytest.approx(2.2e-4, rel=0.01)


def test_negbin_geometric_and_integer_cases():
    # n = 1: geometric, P(k) = p (1-p)^k with p = n/(n+mean)
    mean, dmax = 6.0, 30
    p = demand_pmf({"kind": "negbin", "n": [1.0], "mean": [mean]}, dmax)
    q = 1.0 / (1.0 + mean)
    for d in range(dmax):
        assert p[d] == pytest.approx(q * (1 - q) ** d, rel=1e-12)
    assert p[dmax] == pytest.approx((1 - q) ** dmax, rel=1e-10)
    # integer n = 5: C(k+4, k) p^5 (1-p)^k
    p5 = demand_pmf({"kind": "negbin", "n": [5.0], "mean": [7.0]}, 40)
    pp = 5.0 / 12.0
    for d in range(40):
        assert p5[d] == pytest.approx(math.comb(d + 4, d) * pp ** 5 * (1 - pp) ** d, rel=1e-12)
    assert p5.sum() == pytest.approx(1.0, abs=1e-14)


def test_life_probabilities_softmax():
    sc = W.scenario_c(m=3, a_max=4, c0=[0.0, math.log(2.0), math.log(3.0)],
                      c1=[0.0, 0.0, 0.1])
    lp = life_probabilities(sc)
    for a in range(5):
        e = np.array([1.0, 2.0, 3.0 * math.exp(0.1 * a)])
        assert np.allclose(lp[a], e / e.sum(), rtol=1e-14)


def test_arrival_multinomial_against_scipy():
    sc = W.config3()
    o = Oracle(sc)
    lp = life_probabilities(sc)
    for a in (0, 1, 5, 13):
        tot = 0.0
        for y in U.compositions(a, 5):
            pr = o.arrival_prob(a, y)
            desc = [lp[a][4 - i] for i in range(5)]
            ref = stats.multinomial.pmf(list(y), n=a, p=desc) if a else 1.0
            assert pr == pytest.approx(ref, rel=1e-11, abs=1e-300)
            tot += pr
        assert tot == pytest.approx(1.0, abs=1e-13)


# ------------------------------------------------------------------ sizes

@pytest.mark.parametrize("m,L,expected", [
    (2, 1, 121), (2, 2, 1331), (3, 1, 1331), (3, 2, 14641), (4, 1, 14641),
    (4, 2, 161051), (5, 1, 161051), (5, 2, 1771561)])
def test_state_counts_scenario_a_results_table(m, L, expected):
    o = Oracle(W.scenario_a(m=m, L=L, a_max=10, d_max=20))
    assert o.n_states == expected and o.n_actions == 11


@pytest.mark.parametrize("m,expected", [(3, 3087), (5, 1361367)])
def test_state_counts_scenario_c_results_table(m, expected):
    o = Oracle(W.scenario_c(m=m, a_max=20, d_max=20))
    assert o.n_states == expected and o.n_actions == 21


def test_outcome_counts_scenario_c_results_table():
    # |Omega| = (D_max+1) * #{y : sum y <= A_max}; 37,191 for m=3 and 1,115,730 for m=5
    for m, expected in ((3, 37191), (5, 1115730)):
        n_y = sum(sum(1 for _ in U.compositions(a, m)) for a in range(21))
        assert 21 * n_y == expected


def test_config_sizes():
    assert Oracle(W.config1()).n_states == 4084101
    assert Oracle(W.config2()).n_states == 50625
    assert Oracle(W.config2()).n_actions == 225
    assert Oracle(W.config3()).n_states == 1361367


# ------------------------------------------------------------------ transitions

def _golden_scenario(case):
    s = case["scenario"]
    c = s["costs"]
    if s["family"] == "A":
        return W.scenario_a(m=s["m"], L=s["L"], a_max=s["a_max"], d_max=s["d_max"],
                            costs=W.scenarios._costs(var=(c["var"], 0), hold=c["hold"],
                                                     short=c["short"], waste=c["waste"]),
                            issuing=s.get("issuing", "fifo"))
    if s["family"] == "B":
        return W.scenario_b(m=s["m"], a_max=s["a_max"], d_max=s["d_max"],
                            costs=W.scenarios._costs(var=c["var"], rev=c["rev"]))
    return W.scenario_c(m=s["m"], a_max=s["a_max"], d_max=s["d_max"],
                        costs=W.scenarios._costs(fixed=c["fixed"], hold=c["hold"],
                                                 short=c["short"], waste=c["waste"]))


def test_golden_worked_transitions():
    cases = json.load(open(GOLD))["cases"]
    for case in cases:
        sc = _golden_scenario(case)
        o = Oracle(sc)
        s = o.encode(case["state"])
        a = case["action"]
        if isinstance(a, list):
            a = a[0] * (sc["a_max"][1] + 1) + a[1]
        sn, r = o.transition(s, a, case["omega"])
        assert list(o.decode(sn)) == case["next_state"], case["name"]
        if "next_index" in case:
            assert sn == case["next_index"]
        assert r == pytest.approx(case["reward"], abs=1e-12), case["name"]
        # the unit model agrees with the hand-worked numbers too
        sn2, r2 = U.step(sc, s, a, case["omega"])
        assert sn2 == sn and r2 == pytest.approx(r, abs=1e-12)


SMALL = [
    W.scenario_a(m=2, L=1, a_max=3, d_max=7),
    W.scenario_a(m=3, L=1, a_max=3, d_max=9),
    W.scenario_a(m=2, L=2, a_max=3, d_max=7),
    W.scenario_a(m=3, L=2, a_max=2, d_max=8),
    W.scenario_a(m=1, L=1, a_max=4, d_max=8),
    W.scenario_a(m=1, L=3, a_max=2, d_max=5),
    W.scenario_a(m=3, L=1, a_max=3, d_max=9, issuing="lifo"),
    W.scenario_a(m=3, L=2, a_max=2, d_max=8, issuing="lifo"),
    W.scenario_a(m=4, L=1, a_max=2, d_max=8, issuing="lifo"),
]


@pytest.mark.parametrize("sc", SMALL,
                         ids=lambda s: f"A-m{s['m']}-L{s['L']}-{s.get('issuing', 'fifo')}")
def test_transitions_a_match_unit_model(sc):
    o = Oracle(sc)
    for s in range(o.n_states):
        for a in range(o.n_actions):
            for om in U.all_omegas(sc):
                assert o.transition(s, a, om) == U.step(sc, s, a, om)


def test_transitions_b_match_unit_model():
    sc = W.scenario_b(m=3, a_max=(2, 3), d_max=(6, 5), means=(2.0, 1.5), rho=0.5,
                      costs=W.scenarios._costs(var=(0.5, 0.7), rev=(1.0, 1.3)))
    o = Oracle(sc)
    for s in range(o.n_states):
        for a in range(o.n_actions):
            for dA in range(7):
                for dB in range(6):
                    for k in range(dA + 1):
                        om = (dA, dB, k)
                        sn, r = o.transition(s, a, om)
                        sn2, r2 = U.step(sc, s, a, om)
                        assert sn == sn2 and r == pytest.approx(r2, abs=1e-12)


def test_transitions_c_match_unit_model():
    sc = W.scenario_c(m=3, a_max=3, d_max=5, n_periods=2)
    o = Oracle(sc)
    for s in range(o.n_states):
        for a in range(o.n_actions):
            for om in U.c_omegas(sc, a):
                sn, r = o.transition(s, a, om)
                sn2, r2 = U.step(sc, s, a, om)
                assert sn == sn2 and r == pytest.approx(r2, abs=1e-12)


@pytest.mark.parametrize("issuing", ["fifo", "lifo"])
def test_conservation_a(issuing):
    """on hand + arriving = issued + wasted + carried, for every transition (m=3, L=2).

    FIFO wastes what the demand leaves of X_1; LIFO wastes what it leaves of X_1 after
    the younger units X_2..X_m are gone."""
    sc = W.scenario_a(m=3, L=2, a_max=2, d_max=8, issuing=issuing)
    o = Oracle(sc)
    m, L = sc["m"], sc["L"]
    for s in range(o.n_states):
        dig = o.decode(s)
        stock = int(dig[L - 1:].sum())
        for a in range(o.n_actions):
            for d in range(sc["d_max"][0] + 1):
                sn, _ = o.transition(s, a, [d])
                nd = o.decode(sn)
                issued = min(d, stock)
                younger = stock - int(dig[-1]) if issuing == "lifo" else 0
                wasted = max(int(dig[-1]) - max(d - younger, 0), 0)
                carried = int(nd[L - 1:].sum()) - int(dig[L - 2])   # minus the new arrival
                assert stock == issued + wasted + carried


def test_lifo_equals_fifo_with_one_life_class():
    """m = 1: a single life class, so the issuing order cannot matter."""
    for L in (1, 2):
        fifo = Oracle(W.scenario_a(m=1, L=L, a_max=4, d_max=8))
        lifo = Oracle(W.scenario_a(m=1, L=L, a_max=4, d_max=8, issuing="lifo"))
        V = np.random.default_rng(3).normal(0.0, 20.0, fifo.n_states)
        for x, y in zip(fifo.sweep(V), lifo.sweep(V)):
            assert np.array_equal(x, y)


def test_lifo_differs_from_fifo_when_ages_mix():
    """m = 2 with both ages on hand and demand below the total: FIFO keeps the young
    units, LIFO keeps the old ones (which then expire)."""
    fifo = Oracle(W.scenario_a(m=2, L=1, a_max=5, d_max=9))
    lifo = Oracle(W.scenario_a(m=2, L=1, a_max=5, d_max=9, issuing="lifo"))
    s = fifo.encode([2, 3])                     # X_2 = 2 young, X_1 = 3 old
    assert fifo.transition(s, 0, [2]) == (fifo.encode([0, 2]), -2.0 * 1.0 - 7.0 * 1.0)
    assert lifo.transition(s, 0, [2]) == (lifo.encode([0, 0]), -7.0 * 3.0)


# ------------------------------------------------------------------ Bellman operator

def _dense(sc):
    o = Oracle(sc)
    pmf1 = o.pmf1 if sc["family"] == "B" else None
    lp = life_probabilities(sc) if sc["family"] == "C" else None
    P, r = U.dense_model(sc, o.pmf0, pmf1, lp)
    return o, P, r


DENSE = [
    W.scenario_a(m=2, L=2, a_max=3, d_max=7),
    W.scenario_a(m=3, L=1, a_max=3, d_max=8, issuing="lifo"),
    W.scenario_a(m=3, L=1, a_max=3, d_max=9, demand={"kind": "gamma", "mean": [2.0],
                                                      "cv": [0.8]}),
    W.scenario_b(m=3, a_max=(2, 2), d_max=(4, 3), means=(1.5, 1.2), rho=0.5),
    W.scenario_c(m=3, a_max=3, d_max=5, n_periods=3, n=[2.0, 5.0, 3.0],
                 means=[1.5, 2.5, 2.0], c0=[0.0, 0.5, 1.0], c1=[0.0, 0.1, -0.2]),
]
DENSE_IDS = ["A-m2L2", "A-m3L1-lifo", "A-m3L1-gamma", "B-m3", "C-m3-endogenous"]


@pytest.fixture(scope="module", params=list(range(len(DENSE))), ids=DENSE_IDS)
def dense(request):
    return (DENSE[request.param],) + _dense(DENSE[request.param])


def test_sweep_matches_dense_model(dense):
    sc, o, P, r = dense
    rng = np.random.default_rng(5)
    for _ in range(3):
        V = rng.normal(-50.0, 20.0, o.n_states)
        Vn, pi, gap = o.sweep(V)
        Vd, pid, Q = U.bellman(P, r, sc["gamma"], V)
        assert np.allclose(Vn, Vd, rtol=1e-12, atol=1e-10)
        Qs = np.sort(Q, axis=0)
        clear = (Qs[-1] - Qs[-2]) > 1e-9
        assert np.array_equal(pi[clear], pid[clear])
        assert np.allclose(gap[clear], (Qs[-1] - Qs[-2])[clear], atol=1e-9)
        q = o.q_states(V, np.arange(o.n_states))
        assert np.allclose(q, Q.T, rtol=1e-12, atol=1e-10)


def _lp_optimum(P, r, gamma):
    A, S, _ = P.shape
    Aub = np.concatenate([gamma * P[a] - np.eye(S) for a in range(A)])
    bub = np.concatenate([-r[a] for a in range(A)])
    res = optimize.linprog(np.ones(S), A_ub=Aub, b_ub=bub, bounds=[(None, None)] * S,
                           method="highs", options={"primal_feasibility_tolerance": 1e-10,
                                                    "dual_feasibility_tolerance": 1e-10})
    assert res.status == 0
    return res.x


def _policy_iteration(P, r, gamma):
    A, S, _ = P.shape
    pi = np.zeros(S, dtype=int)
    for _ in range(200):
        Pp = P[pi, np.arange(S)]
        rp = r[pi, np.arange(S)]
        V = np.linalg.solve(np.eye(S) - gamma * Pp, rp)
        Q = r + gamma * P @ V
        new = Q.argmax(axis=0)
        keep = Q[pi, np.arange(S)] >= Q.max(axis=0) - 1e-12
        new[keep] = pi[keep]
        if np.array_equal(new, pi):
            return V, pi, Q
        pi = new
    raise AssertionError("policy iteration did not settle")


def test_vi_against_lp_and_policy_iteration(dense):
    sc, o, P, r = dense
    g = sc["gamma"]
    res = o.solve(thr=1e-11)
    assert res["converged"]
    V_lp = _lp_optimum(P, r, g)
    V_pi, pi_star, Q = _policy_iteration(P, r, g)
    assert np.allclose(V_lp, V_pi, rtol=1e-7, atol=1e-6)
    k = g / (1.0 - g)
    lo = res["V"] + k * res["dmin"]
    hi = res["V"] + k * res["dmax"]
    # MacQueen bounds bracket the optimum
    assert np.all(lo <= V_pi + 1e-7) and np.all(V_pi <= hi + 1e-7)
    vhat = res["V"] + k * 0.5 * (res["dmax"] + res["dmin"])
    assert np.allclose(vhat, V_pi, rtol=1e-8, atol=1e-6)
    Qs = np.sort(Q, axis=0)
    clear = (Qs[-1] - Qs[-2]) > 1e-6
    assert np.array_equal(res["pi"][clear], pi_star[clear])


def test_supnorm_stop_bound(dense):
    """The sup-norm rule (Appendix A): once max|V_i - V_{i-1}| < eps the iterate is
    within gamma eps / (1 - gamma) of the optimum (LP), and it never stops earlier
    than the first sweep meeting the rule."""
    sc, o, P, r = dense
    g = sc["gamma"]
    V_lp = _lp_optimum(P, r, g)
    for eps in (1e-2, 1e-5):
        res = o.solve(thr=eps, stop_rule="supnorm")
        assert res["converged"] and max(abs(res["dmax"]), abs(res["dmin"])) < eps
        assert np.abs(res["V"] - V_lp).max() <= g * eps / (1.0 - g) + 1e-6
        if res["sweeps"] > 1:
            prev = o.solve(thr=eps, fixed_sweeps=res["sweeps"] - 1)
            assert max(abs(prev["dmax"]), abs(prev["dmin"])) >= eps


def _no_order_c(P):
    """Scenario C with ordering priced out (fixed cost 1e6) and one-day stock: from
    the second day on every state holds nothing and earns the weekday's shortage
    reward, so after the first sweep every state's increments are the same cycle of
    rewards."""
    return W.scenario_c(m=2, a_max=2, d_max=6, n_periods=P, gamma=0.9,
                        means=[1.0 + 0.5 * t for t in range(P)], n=[3.0] * P,
                        costs=W.scenarios._costs(fixed=1e6, hold=1.0, short=20.0, waste=5.0))


@pytest.mark.parametrize("P", [2, 3, 7])
def test_periodic_rule_stops_after_one_full_cycle(P):
    """Appendix C's periodic test on the instance above: the window of the last P
    increments holds one whole weekly cycle for every state once it no longer
    contains the first sweep (whose reward depends on the stock held), so the test
    is met exactly at sweep P + 1 and not before."""
    o = Oracle(_no_order_c(P))
    res = o.solve(thr=1e-4, stop_rule="periodic")
    assert res["converged"] and res["sweeps"] == P + 1
    assert np.all(res["pi"] == 0)


def test_periodic_rule_keeps_the_converged_policy():
    """The point of the periodic test (Appendix C): once every state gains the same
    amount per cycle the greedy policy no longer changes.  It stops far earlier than
    the span rule and its policy equals the tightly converged one."""
    sc = W.scenario_c(m=3, a_max=6, d_max=12, n_periods=3, means=[2.0, 3.5, 2.5],
                      n=[5.0] * 3, c0=[0.0, 1.0, 2.0])
    o = Oracle(sc)
    per = o.solve(thr=1e-4, stop_rule="periodic")
    tight = o.solve(thr=1e-11)
    assert per["converged"] and per["sweeps"] < tight["sweeps"] // 2
    clear = tight["gap"] > 1e-3
    assert np.array_equal(per["pi"][clear], tight["pi"][clear])


def test_policy_evaluation_fixed_point(dense):
    sc, o, P, r = dense
    g = sc["gamma"]
    res = o.solve(thr=1e-11)
    S = o.n_states
    pi = res["pi"]
    Vp = np.linalg.solve(np.eye(S) - g * P[pi, np.arange(S)], r[pi, np.arange(S)])
    Vn, pi2, gap = o.sweep(Vp)
    assert np.allclose(Vn, Vp, rtol=1e-10, atol=1e-8)     # greedy w.r.t. its own value


def test_contraction(dense):
    sc, o, P, r = dense
    g = sc["gamma"]
    rng = np.random.default_rng(11)
    for _ in range(4):
        V = rng.normal(0.0, 30.0, o.n_states)
        Uu = rng.normal(0.0, 30.0, o.n_states)
        TV, _, _ = o.sweep(V)
        TU, _, _ = o.sweep(Uu)
        assert np.abs(TV - TU).max() <= g * np.abs(V - Uu).max() + 1e-9
        sp = lambda x: x.max() - x.min()
        assert sp(TV - TU) <= g * sp(V - Uu) + 1e-9


# ------------------------------------------------------------------ special cases

def test_newsvendor_m1_closed_form():
    """m=1, L=1: every leftover expires, so the order is state-independent.

    a* is the critical fractile min{a : F(a) >= (g*Cs - Cv)/(g*(Cs+Cw))} and
    V*(x) = G(x) + h(a*)/(1-g), with G(x) = -Cs E[D-x]+ - Cw E[x-D]+ and
    h(a) = -Cv a + g G(a).
    """
    sc = W.scenario_a(m=1, L=1, a_max=10, d_max=20)
    g, c = sc["gamma"], sc["costs"]
    pmf = np.array([stats.poisson.pmf(d, 4.0) for d in range(20)] + [stats.poisson.sf(19, 4.0)])
    F = np.cumsum(pmf)
    ratio = (g * c["short"] - c["var"][0]) / (g * (c["short"] + c["waste"]))
    assert ratio == pytest.approx(0.16414, abs=1e-5)
    a_star = int(np.argmax(F >= ratio))
    assert a_star == 2
    d = np.arange(21)
    G = np.array([-(c["short"] * np.maximum(d - x, 0) + c["waste"] * np.maximum(x - d, 0)) @ pmf
                  for x in range(11)])
    h = -c["var"][0] * np.arange(11) + g * G
    V_star = G + h.max() / (1.0 - g)
    o = Oracle(sc)
    res = o.solve()
    k = g / (1 - g)
    vhat = res["V"] + k * 0.5 * (res["dmax"] + res["dmin"])
    assert np.allclose(vhat, V_star, rtol=1e-12, atol=1e-9)
    assert np.all(res["pi"] == a_star)
    long = o.solve(fixed_sweeps=4000)
    assert np.allclose(long["V"], V_star, rtol=1e-12, atol=1e-9)


def test_b_rho_zero_separability():
    base = dict(m=3, d_max=(5, 4), means=(2.0, 1.5), rho=0.0,
                costs=W.scenarios._costs(var=(0.5, 0.6), rev=(1.0, 1.2)))
    full = Oracle(W.scenario_b(a_max=(2, 3), **base)).solve(thr=1e-12)
    oa = Oracle(W.scenario_b(a_max=(2, 0), **base))
    ob = Oracle(W.scenario_b(a_max=(0, 3), **base))
    ra, rb = oa.solve(thr=1e-12), ob.solve(thr=1e-12)
    g = 0.99
    k = g / (1 - g)
    vh = lambda res: res["V"] + k * 0.5 * (res["dmax"] + res["dmin"])
    Vf, Va, Vb = vh(full), vh(ra), vh(rb)
    nA, nB = oa.n_states, ob.n_states
    assert nA * nB == len(Vf)
    sep = Va[:, None] + Vb[None, :]
    assert np.allclose(Vf.reshape(nA, nB), sep, rtol=1e-9, atol=1e-7)
    # policy separates too: joint index aA*(4)+aB
    pf = full["pi"].reshape(nA, nB)
    assert np.array_equal(pf // 4, np.repeat(ra["pi"][:, None] // 1, nB, axis=1))
    assert np.array_equal(pf % 4, np.repeat(rb["pi"][None, :], nA, axis=0))


def test_c_weekday_invariance():
    sc = W.scenario_c(m=3, a_max=4, d_max=8, n=[3.0] * 7, means=[3.0] * 7)
    o = Oracle(sc)
    res = o.solve(thr=1e-10)
    V = res["V"].reshape(7, -1)
    assert np.allclose(V, V[0][None, :], rtol=0, atol=1e-9)
    assert np.array_equal(res["pi"].reshape(7, -1), np.repeat(res["pi"].reshape(7, -1)[:1], 7, 0))


def test_fixed_sweeps_counts():
    o = Oracle(W.config0())
    r = o.solve(fixed_sweeps=7)
    assert r["sweeps"] == 7
    r2 = o.solve(fixed_sweeps=3)
    r3 = o.solve(fixed_sweeps=4, v0=None)
    Vn, _, _ = o.sweep(r2["V"])
    assert np.allclose(Vn, o.solve(fixed_sweeps=4)["V"], rtol=0, atol=0)
    assert r3["sweeps"] == 4


def test_ties_go_to_lowest_action():
    """With no ordering cost and V = 0 every action has the same Q: pi must be 0."""
    for sc in (W.scenario_a(m=2, L=1, a_max=4, d_max=6,
                            costs=W.scenarios._costs(hold=1.0, short=5.0, waste=7.0)),
               W.scenario_c(m=3, a_max=3, d_max=5,
                            costs=W.scenarios._costs(hold=1.0, short=5.0, waste=2.0))):
        if sc["family"] == "C":
            continue  # arrivals change the stock, so actions differ even at V = 0
        o = Oracle(sc)
        Vn, pi, gap = o.sweep(np.zeros(o.n_states))
        assert np.all(pi == 0) and np.all(gap == 0.0)
    sc = W.scenario_b(m=3, a_max=(2, 2), d_max=(3, 3), means=(1.0, 1.0),
                      costs=W.scenarios._costs(rev=(0.0, 0.0)))
    o = Oracle(sc)
    Vn, pi, gap = o.sweep(np.zeros(o.n_states))
    assert np.all(pi == 0) and np.all(gap == 0.0)
