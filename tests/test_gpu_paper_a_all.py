"""Every experiment of Appendix A, solved and rolled out on the GPU: the results table
(value-iteration return and the best base-stock policy's return) and the KPI table
(best base-stock level, service level, wastage and holding of both policies), each over
10,000 rollouts of 100 warm-up and 365 counted days.

Two independent 10,000-rollout means differ by at most four standard errors of their
difference, plus half a unit of the printed rounding; standard deviations agree to
the printed precision plus a margin.  The best base-stock level of a grid S = 0..A_max
under common random numbers must be the paper's level or within sampling error of it.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_rollouts.json")))
ROWS = GOLD["scenario_a_all"]
N = 10000


def _close(ours, printed, sd, digits=0):
    return abs(ours - printed) <= 4.0 * sd * np.sqrt(2.0 / N) + 0.5 * 10.0 ** -digits


def _kpis_match(st, printed):
    """st: the 8 statistics of one policy (return, service, wastage, holding)."""
    for q, name in enumerate(("service", "wastage", "holding")):
        mean, sd = st[2 + 2 * q], st[3 + 2 * q]
        assert _close(mean, printed[name][0], sd, digits=1), (name, mean, printed[name])
        assert abs(sd - printed[name][1]) <= 0.15, (name, sd, printed[name])


@pytest.mark.parametrize("row", ROWS, ids=lambda r: f"m{r['m']}e{r['exp']}")
def test_paper_a_experiment(row):
    sc = W.scenario_a_paper(row["m"], row["L"], float(row["c_waste"]), row["issuing"])
    m = pvi.mdp_create(sc)
    assert m.n_states == row["states"]
    pvi.vi_solve(m, precision="fp64", eps=1e-4, stop_rule="supnorm")
    st = pvi.policy_rollouts(m, n_rollouts=N, seed=1, per_rollout=False)["stats"][0]
    assert _close(st[0], row["vi_return"][0], st[1]), (st[0], row["vi_return"])
    assert abs(st[1] - row["vi_return"][1]) <= 2.0
    _kpis_match(st, row["vi_kpi"])
    grid = [[S] for S in range(sc["a_max"][0] + 1)]
    best, stats = pvi.heuristic_search(m, "base_stock", grid, n_rollouts=N, seed=1)
    at = row["s_best"]
    assert stats[best, 0] - stats[at, 0] <= 4.0 * stats[at, 1] * np.sqrt(2.0 / N)
    assert _close(stats[at, 0], row["so_return"][0], stats[at, 1])
    assert abs(stats[at, 1] - row["so_return"][1]) <= 2.0
    _kpis_match(stats[at], row["so_kpi"])
