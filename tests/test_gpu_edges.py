"""Degenerate instances of every family through the C ABI against the oracle: one
action (scenario A then has a single state), demand that is always zero or at most
one unit, two order sizes, the shortest lives, and substitution that always or never
happens.  Tolerances as for the other parity tests: one FP64 backup 1e-12 normwise,
FP32 storage 1e-6; converged FP64 solves match the oracle's sweep count and V to
1e-12 and its policy wherever the oracle's best-minus-second gap exceeds 1e-6;
rollouts of a seeded table match draw for draw.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu

EDGES = {
    "A-one-action": W.scenario_a(m=3, L=2, a_max=0, d_max=6),
    "A-zero-demand": W.scenario_a(m=2, L=1, a_max=4, d_max=0),
    "A-demand-0-or-1": W.scenario_a(m=3, L=1, a_max=3, d_max=1),
    "A-two-orders-L3": W.scenario_a(m=4, L=3, a_max=1, d_max=3),
    "A-lifo-two-orders": W.scenario_a(m=3, L=2, a_max=1, d_max=4, issuing="lifo"),
    "B-product0-fixed": W.scenario_b(m=3, a_max=(0, 4), d_max=(5, 5), means=(2.0, 2.0),
                                     rho=0.5),
    "B-always-substitute": W.scenario_b(m=2, a_max=(3, 3), d_max=(6, 6), means=(2.0, 2.0),
                                        rho=1.0),
    "C-m2": W.scenario_c(m=2, a_max=6, d_max=9),
    "C-two-orders": W.scenario_c(m=4, a_max=1, d_max=3),
    "B1-product-b-fixed": W.scenario_b1(m=2, a_max=(3, 0), means=(2.0, 1.0), rho=0.5,
                                        d_max=8, gamma=0.95),
    "B1-m1": W.scenario_b1(m=1, a_max=(1, 1), means=(1.0, 1.0), rho=1.0, d_max=3,
                           gamma=0.9),
}


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(EDGES))
def test_one_backup(name):
    sc = EDGES[name]
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    assert (m.n_states, m.n_actions) == (o.n_states, o.n_actions)
    V = W.random_values(o.n_states, seed=3, scale=5.0, offset=-20.0)
    Vo, pio, gapo = o.sweep(V)
    Vg, pig, gapg = pvi.vi_backup(m, V, "fp64")
    assert relerr(Vg, Vo) < 1e-12
    clear = gapo > 1e-9
    assert np.array_equal(pig[clear], pio[clear])
    V32, _, _ = pvi.vi_backup(m, V, "fp32")
    assert relerr(V32, Vo) < 1e-6


@pytest.mark.parametrize("name", list(EDGES))
def test_converged(name):
    sc = EDGES[name]
    o = Oracle(sc)
    ref = o.solve()
    m = pvi.mdp_create(sc)
    res = pvi.vi_solve(m, precision="fp64")
    assert res["status"] == pvi.PVI_OK
    assert res["sweeps_fp64"] == ref["sweeps"]
    assert relerr(pvi.value_get(m), ref["V"]) < 1e-12
    pol, _ = pvi.policy_get(m)
    clear = ref["gap"] > 1e-6
    assert np.array_equal(pol[clear], ref["pi"][clear])
    res = pvi.vi_solve(m, precision="fp32")
    assert res["status"] == pvi.PVI_OK
    pol, _ = pvi.policy_get(m)
    clear = ref["gap"] > 1e-3
    assert np.array_equal(pol[clear], ref["pi"][clear])


@pytest.mark.parametrize("name", list(EDGES))
def test_rollouts(name):
    sc = EDGES[name]
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    rng = np.random.default_rng([23, len(name)])
    table = rng.integers(0, o.n_actions, size=o.n_states).astype(np.int32)
    g = pvi.policy_rollouts(m, table=table, n_rollouts=200, warmup=5, horizon=60, seed=11)
    ret, kpi = o.simulate("table", table=table, n_rollouts=200, warmup=5, horizon=60, seed=11)
    assert np.allclose(g["ret"], ret, rtol=1e-12, atol=1e-9)
    assert np.array_equal(g["kpi"], kpi)
