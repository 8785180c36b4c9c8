"""Pins of the oracle's rollout simulator (Simulation section: rollouts, return and
KPIs; Philox counter-based random numbers).

* Its Philox4x64-10 equals numpy's implementation of the same published generator.
* Each rollout equals a replay in the unit-by-unit model of tests/unit_model.py,
  with draws taken from numpy's Philox and sampled by the stated rules.
* At the paper's settings, the means and standard deviations over 10,000 rollouts
  of the value-iteration policy, and the best base-stock level with its return,
  match what the paper prints for scenarios A and C (tests/golden/paper_rollouts.json)
  within the sampling error of two 10,000-rollout means plus the printed rounding.
"""
import json
import os

import numpy as np
import pytest

import unit_model as U
import workloads as W
from oracle.oracle import Oracle, demand_pmf, life_probabilities, philox4x64_10

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_rollouts.json")))


def _numpy_philox(counter, key):
    # numpy's Philox advances its counter before producing each block of 4 words
    cint = sum(int(v) << (64 * i) for i, v in enumerate(counter))
    kint = sum(int(v) << (64 * i) for i, v in enumerate(key))
    return np.random.Philox(counter=(cint - 1) % 2 ** 256, key=kint).random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((7, 3, 1, 0), (12345, 0)),
    ((2 ** 64 - 1, 2 ** 63, 5, 9), (2 ** 40 + 17, 2 ** 64 - 2)),
    ((999, 464, 6, 0), (2023, 0)),
])
def test_philox_matches_numpy(counter, key):
    assert np.array_equal(philox4x64_10(counter, key), _numpy_philox(counter, key))


def _u(seed, r, t, b, w):
    x = int(_numpy_philox((r, t, b, 0), (seed, 0))[w])
    return (x >> 11) * 2.0 ** -53


def _inverse_cdf(pmf, u):
    c = 0.0
    for d in range(len(pmf) - 1):
        c += pmf[d]
        if u < c:
            return d
    return len(pmf) - 1


def _replay(sc, table, n_roll, warmup, horizon, seed):
    """Rollouts in the unit model; returns (ret, kpi) like Oracle.simulate."""
    fam, m = sc["family"], sc["m"]
    pmfs = [demand_pmf(sc["demand"][0], sc["d_max"][0], t) for t in range(sc["n_periods"])]
    pmf1 = demand_pmf(sc["demand"][1], sc["d_max"][1]) if fam in ("B", "B1") else None
    life = life_probabilities(sc) if fam == "C" else None
    ret = np.zeros(n_roll)
    kpi = np.zeros((n_roll, 3))
    pkpi = np.zeros((n_roll, 2, 3))
    for r in range(n_roll):
        s, g, acc = 0, 1.0, 0.0
        tot = {"demand": 0, "met": 0, "expired": 0, "received": 0, "held": 0}
        per = [dict(tot), dict(tot)]
        for t in range(warmup + horizon):
            a = int(table[s])
            dig = U.decode(sc, s)
            if fam == "A":
                om = (_inverse_cdf(pmfs[0], _u(seed, r, t, 0, 0)),)
            elif fam == "B":
                nb = sc["a_max"][1] + 1
                dA = _inverse_cdf(pmfs[0], _u(seed, r, t, 0, 0))
                dB = _inverse_cdf(pmf1, _u(seed, r, t, 0, 1))
                stockA = a // nb + sum(dig[:m - 1])
                unmet = max(dA - stockA, 0)
                k = sum(1 for i in range(unmet) if _u(seed, r, t, 1 + i // 4, i % 4)
                        < sc["subst_rho"])
                om = (dA, dB, k)
            elif fam == "B1":
                dA = _inverse_cdf(pmfs[0], _u(seed, r, t, 0, 0))
                dB = _inverse_cdf(pmf1, _u(seed, r, t, 0, 1))
                excess = max(dB - sum(dig[m:]), 0)
                du = sum(1 for i in range(excess) if _u(seed, r, t, 1 + i // 4, i % 4)
                         < sc["subst_rho"])
                om = (dA, dB, du)
            else:
                d = _inverse_cdf(pmfs[dig[0]], _u(seed, r, t, 0, 0))
                y = [0] * (m + 1)                       # y[life]
                for i in range(a):
                    u, c, lf = _u(seed, r, t, 1 + i // 4, i % 4), 0.0, m
                    for k in range(1, m):
                        c += life[a][k - 1]
                        if u < c:
                            lf = k
                            break
                    y[lf] += 1
                om = (d,) + tuple(y[m - i] for i in range(m))
            s, rw, cnt = U.day(sc, s, a, om)
            if t >= warmup:
                acc += g * rw
                g *= sc["gamma"]
                for key in tot:
                    tot[key] += cnt[key]
                    for k in range(2 if "product" in cnt else 0):
                        per[k][key] += cnt["product"][k][key]
        ret[r] = acc
        kpi[r] = _kpis(tot, horizon)
        for k in range(2):
            pkpi[r, k] = _kpis(per[k], horizon)
    return ret, kpi, pkpi


def _kpis(tot, horizon):
    return (100.0 * tot["met"] / tot["demand"] if tot["demand"] else 100.0,
            100.0 * tot["expired"] / tot["received"] if tot["received"] else 0.0,
            tot["held"] / horizon)


REPLAY = [
    W.scenario_a(m=3, L=2, a_max=5, d_max=9),
    W.scenario_a(m=3, L=1, a_max=6, d_max=10, issuing="lifo",
                 demand={"kind": "gamma", "mean": [3.0], "cv": [0.8]}),
    W.scenario_b(m=3, a_max=(3, 4), d_max=(6, 5), means=(3.0, 2.0), rho=0.6),
    W.scenario_c(m=3, a_max=5, d_max=8, c0=[0.0, 1.0, 0.5], c1=[0.0, 0.2, -0.1]),
    W.scenario_b1(m=2, a_max=(4, 3), means=(3.0, 2.5), rho=0.5, d_max=10),
]


@pytest.mark.parametrize("sc", REPLAY, ids=["A-fifo", "A-lifo", "B", "C-endogenous", "B1"])
def test_rollouts_match_unit_model_replay(sc):
    o = Oracle(sc)
    rng = np.random.default_rng(5)
    table = rng.integers(0, o.n_actions, size=o.n_states).astype(np.int32)
    ret, kpi = o.simulate("table", table=table, n_rollouts=6, warmup=4, horizon=25, seed=77)
    r2, k2, p2 = _replay(sc, table, 6, 4, 25, 77)
    assert np.allclose(ret[0], r2, rtol=1e-13, atol=1e-9)
    assert np.array_equal(kpi[0], k2)
    if sc["family"] in ("B", "B1"):
        _, kpi3, pkpi = o.simulate("table", table=table, n_rollouts=6, warmup=4, horizon=25,
                                   seed=77, by_product=True)
        assert np.array_equal(kpi3, kpi)
        assert np.array_equal(pkpi[0], p2)


def test_heuristics_follow_their_definitions():
    """Base stock orders up to S from stock on hand and in transit; the modified
    base stock adds the expected excess of the oldest units; (s, S) orders only at
    or below s and only when s < S."""
    sc = W.scenario_a(m=2, L=2, a_max=6, d_max=8)
    o = Oracle(sc)
    for S in (0, 4, 6):                   # orders <= S <= a_max: the state space holds them
        table = np.array([max(S - int(np.sum(U.decode(sc, s))), 0)
                          for s in range(o.n_states)], dtype=np.int32)
        a, ka = o.simulate("base_stock", params=[[S]], n_rollouts=5, warmup=3, horizon=20)
        b, kb = o.simulate("table", table=table, n_rollouts=5, warmup=3, horizon=20)
        assert np.array_equal(a, b) and np.array_equal(ka, kb)
    sc = W.scenario_b(m=3, a_max=(4, 3), d_max=(6, 5), means=(3.0, 2.0), rho=0.5)
    o = Oracle(sc)
    SA, SB = 4, 3
    rows = []
    for s in range(o.n_states):
        dig = U.decode(sc, s)
        qa = int(np.floor(max(SA - sum(dig[:2]) + max(dig[1] - 3.0, 0.0), 0.0)))
        qb = int(np.floor(max(SB - sum(dig[2:]) + max(dig[3] - 2.0, 0.0), 0.0)))
        assert qa <= SA and qb <= SB
        rows.append(qa * 4 + qb)
    a, _ = o.simulate("mod_base_stock", params=[[SA, SB]], n_rollouts=5, warmup=2, horizon=15)
    b, _ = o.simulate("table", table=np.array(rows, np.int32), n_rollouts=5, warmup=2,
                      horizon=15)
    assert np.array_equal(a, b)
    sc = W.scenario_c(m=3, a_max=6, d_max=8)
    o = Oracle(sc)
    prm = [1, 5, 3, 3, 0, 6, 2, 4, 6, 2, 0, 0, 4, 6]
    rows = []
    for s in range(o.n_states):
        dig = U.decode(sc, s)
        lo, hi = prm[2 * dig[0]], prm[2 * dig[0] + 1]
        I = sum(dig[1:])
        rows.append(min(max(hi - I, 0), 6) if (lo < hi and I <= lo) else 0)
    a, _ = o.simulate("s_S", params=[prm], n_rollouts=5, warmup=2, horizon=15)
    b, _ = o.simulate("table", table=np.array(rows, np.int32), n_rollouts=5, warmup=2,
                      horizon=15)
    assert np.array_equal(a, b)


def test_heuristic_orders_are_not_capped():
    """With nothing on hand or in transit a heuristic orders S units, S being its
    largest order (Heuristic policies passage), also above the maximum order
    quantity of value iteration: one day from the empty state shows the order in
    the reward and, for scenario B, in the units received."""
    sc = W.scenario_a(m=2, L=2, a_max=6, d_max=8)
    o = Oracle(sc)
    pmf = demand_pmf(sc["demand"][0], sc["d_max"][0])
    c = sc["costs"]
    for S in (3, 9, 40):
        ret, _ = o.simulate("base_stock", params=[[S]], n_rollouts=4, warmup=0, horizon=1,
                            seed=6)
        for r in range(4):
            d = _inverse_cdf(pmf, _u(6, r, 0, 0, 0))
            want = -c["var"][0] * S - c["short"] * d     # empty shelf: all demand unmet
            assert abs(ret[0, r] - want) < 1e-12
    sc = W.scenario_b1(m=2, a_max=(4, 3), means=(3.0, 2.5), rho=0.5, d_max=10)
    o = Oracle(sc)
    c = sc["costs"]
    for SA, SB in ((2, 1), (9, 7), (30, 0)):
        ret, kpi, pk = o.simulate("mod_base_stock", params=[[SA, SB]], n_rollouts=3, warmup=0,
                                  horizon=1, seed=2, by_product=True)
        assert np.all(ret == -(c["var"][0] * SA + c["var"][1] * SB))  # nothing to sell yet
        assert np.all(pk[0, :, :, 1] == 0.0)                          # received, none expired
        assert np.all(kpi[0, :, 2] == 0.0) and np.all(pk[0, :, :, 2] == 0.0)


def test_policies_share_random_numbers():
    """Rollout r of every candidate sees the same demand, so a candidate repeated in
    the grid gives identical rollouts."""
    sc = W.scenario_a(m=2, L=1, a_max=8, d_max=12)
    o = Oracle(sc)
    ret, kpi = o.simulate("base_stock", params=[[5], [7], [5]], n_rollouts=50, seed=3)
    assert np.array_equal(ret[0], ret[2]) and np.array_equal(kpi[0], kpi[2])
    assert not np.array_equal(ret[0], ret[1])


def _close(ours, printed, sd, n=10000, digits=0):
    """Two independent n-rollout means of a quantity with standard deviation sd
    differ by at most 4 standard errors of their difference, plus half a unit of
    the printed rounding."""
    return abs(ours - printed) <= 4.0 * sd * np.sqrt(2.0 / n) + 0.5 * 10.0 ** -digits


@pytest.mark.parametrize("row", GOLD["scenario_a"], ids=lambda r: f"m{r['m']}e{r['exp']}")
def test_scenario_a_rollouts_match_the_paper(row):
    sc = W.scenario_a_paper(row["m"], row["L"], float(row["c_waste"]), row["issuing"])
    o = Oracle(sc)
    vi = o.solve(thr=1e-4, stop_rule="supnorm")
    ret, kpi = o.simulate("table", table=vi["pi"], n_rollouts=10000, seed=1)
    mean, sd = ret[0].mean(), ret[0].std(ddof=1)
    assert _close(mean, row["vi_return"][0], sd)
    assert abs(sd - row["vi_return"][1]) <= 2.0
    k = kpi[0]
    assert _close(k[:, 0].mean(), row["vi_service"], k[:, 0].std(), digits=1)
    assert _close(k[:, 1].mean(), row["vi_wastage"], k[:, 1].std(), digits=1)
    assert _close(k[:, 2].mean(), row["vi_holding"], k[:, 2].std(), digits=1)
    grid, _ = o.simulate("base_stock", params=[[S] for S in range(11)], n_rollouts=10000,
                         seed=1)
    best = int(np.argmax(grid.mean(axis=1)))
    assert best == row["s_best"]
    assert _close(grid[best].mean(), row["so_return"][0], grid[best].std(ddof=1))


@pytest.mark.parametrize("row", GOLD["scenario_c"], ids=lambda r: f"m{r['m']}e{r['exp']}")
def test_scenario_c_rollouts_match_the_paper(row):
    sc = W.scenario_c_paper(row["m"], row["exp"])
    o = Oracle(sc)
    vi = o.solve(thr=1e-4, stop_rule="periodic")
    ret, kpi = o.simulate("table", table=vi["pi"], n_rollouts=10000, seed=1)
    mean, sd = ret[0].mean(), ret[0].std(ddof=1)
    assert _close(mean, row["vi_return"][0], sd)
    assert abs(sd - row["vi_return"][1]) <= 2.0
    k = kpi[0]
    assert _close(k[:, 0].mean(), row["vi_service"], k[:, 0].std(), digits=1)
    assert _close(k[:, 1].mean(), row["vi_wastage"], k[:, 1].std(), digits=1)
    assert _close(k[:, 2].mean(), row["vi_holding"], k[:, 2].std(), digits=1)


@pytest.mark.parametrize("row", GOLD["scenario_c_heuristic"],
                         ids=lambda r: f"m{r['m']}e{r['exp']}")
def test_scenario_c_heuristic_matches_the_paper(row):
    """The paper's best weekday (s, S) parameters, rolled out 10,000 times, give its
    simulation-optimization return and KPIs."""
    sc = W.scenario_c_paper(row["m"], row["exp"])
    o = Oracle(sc)
    prm = [v for pair in zip(row["s"], row["S"]) for v in pair]
    ret, kpi = o.simulate("s_S", params=[prm], n_rollouts=10000, seed=1)
    mean, sd = ret[0].mean(), ret[0].std(ddof=1)
    assert _close(mean, row["so_return"][0], sd)
    assert abs(sd - row["so_return"][1]) <= 2.0
    k = kpi[0]
    assert _close(k[:, 0].mean(), row["so_service"], k[:, 0].std(), digits=1)
    assert _close(k[:, 1].mean(), row["so_wastage"], k[:, 1].std(), digits=1)
    assert _close(k[:, 2].mean(), row["so_holding"], k[:, 2].std(), digits=1)
