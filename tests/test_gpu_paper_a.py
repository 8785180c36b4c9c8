"""GPU parity at the paper's own scenario-A settings (Appendix A common-settings table:
gamma demand, mean 4, coefficient of variation 0.5, truncated at 100; orders up to
10; C_v 3, C_s 5, C_h 1; C_w 7 or 10; gamma 0.99; FIFO or LIFO issuing; the
sup-norm stop with eps 1e-4), at every size of the results table: 121, 1,331,
14,641, 161,051 and 1,771,561 states, 11 actions, 101 demand outcomes.

Small sizes: the converged FP64 solve equals the oracle's (same sweep count, V within
1e-12 normwise, policies equal wherever the oracle's gap exceeds 1e-6).  Large sizes:
one FP64 backup of a seeded V checked on sampled states that the oracle backs up one
by one, and the converged solve checked by what the sup-norm stop guarantees: with
|V_n - V_{n-1}| < eps, every Q of V_n lies within gamma*eps of the same Q of V_{n-1},
so the oracle's backup of the returned V is within gamma*eps of it, and the returned
policy (the argmax over Q of V_{n-1}) is the oracle's argmax over Q of V_n wherever
that gap exceeds 2*gamma*eps.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _case(m, L, cw, iss):
    return W.scenario_a_paper(m, L, cw, iss)


def _id(m, L, cw, iss):
    return f"m{m}L{L}Cw{int(cw)}{iss}"


# the four settings at 121 states and the eight at 1,331 (m=2 L=2 and m=3 L=1)
SMALL = [(m, L, cw, iss) for (m, _, L, cw, iss) in W.PAPER_A_EXPERIMENTS
         if m + L - 1 <= 3]
# one FIFO and one LIFO per larger shape, alternating the waste cost
LARGE = [(3, 2, 7.0, "lifo"), (4, 1, 10.0, "fifo"), (4, 2, 10.0, "lifo"),
         (5, 1, 7.0, "fifo"), (5, 2, 7.0, "fifo"), (5, 2, 10.0, "lifo")]


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_preset_table_matches_the_paper():
    """32 experiments: m 2..5, each over L in {1, 2}, C_w in {7, 10} and both issuing
    rules, in the results table's order (LIFO before FIFO, C_w 7 before 10)."""
    ex = W.PAPER_A_EXPERIMENTS
    assert len(ex) == 32
    assert [e[1] for e in ex[:8]] == list(range(1, 9))
    assert ex[0] == (2, 1, 1, 7.0, "lifo") and ex[7] == (2, 8, 2, 10.0, "fifo")
    sc = W.scenario_a_paper(5, 2, 10.0, "lifo")
    m = pvi.mdp_create(sc)
    assert (m.n_states, m.n_actions) == (1771561, 11)
    r = pvi.vi_solve(m, precision="fp64", fixed_sweeps=1)
    # the sweeps and the policy extraction
    assert r["logical_backups"] == 1771561 * 11 * 101 * (r["sweeps_fp64"] + 1)


@pytest.mark.parametrize("case", SMALL, ids=[_id(*c) for c in SMALL])
def test_paper_a_small_converged_fp64(case):
    sc = _case(*case)
    o = Oracle(sc)
    ref = o.solve(thr=EPS, stop_rule="supnorm")
    m = pvi.mdp_create(sc)
    res = pvi.vi_solve(m, precision="fp64", eps=EPS, stop_rule="supnorm")
    assert res["status"] == pvi.PVI_OK
    assert res["sweeps_fp64"] == ref["sweeps"]
    assert relerr(pvi.value_get(m), ref["V"]) < 1e-12
    pol, _ = pvi.policy_get(m)
    clear = ref["gap"] > 1e-6
    assert clear.mean() > 0.9
    assert np.array_equal(pol[clear], ref["pi"][clear])


@pytest.mark.parametrize("case", SMALL[::3], ids=[_id(*c) for c in SMALL[::3]])
def test_paper_a_small_fp32_schedule(case):
    """FP32 sweeps then the FP64 polish: within the sup-norm rule's own bound of the
    oracle's converged V, and the same policy wherever the oracle's gap is clear."""
    sc = _case(*case)
    o = Oracle(sc)
    ref = o.solve(thr=EPS, stop_rule="supnorm")
    m = pvi.mdp_create(sc)
    res = pvi.vi_solve(m, precision="fp32_wide", eps=EPS, stop_rule="supnorm")
    assert res["status"] == pvi.PVI_OK
    g = sc["gamma"]
    assert np.abs(pvi.value_get(m) - ref["V"]).max() <= 2 * g * EPS / (1 - g)
    pol, _ = pvi.policy_get(m)
    clear = ref["gap"] > 1e-3
    assert np.array_equal(pol[clear], ref["pi"][clear])


@pytest.mark.parametrize("case", LARGE, ids=[_id(*c) for c in LARGE])
def test_paper_a_large_one_backup_sampled(case):
    sc = _case(*case)
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    V = W.random_values(o.n_states, seed=11)
    Vg, pig, _ = pvi.vi_backup(m, V, "fp64")
    idx = W.sample_indices(o.n_states, 1500, seed=11)
    Q = o.q_states(V, idx)
    assert relerr(Vg[idx], Q.max(axis=1)) < 1e-12
    Qs = np.sort(Q, axis=1)
    clear = (Qs[:, -1] - Qs[:, -2]) > 1e-9
    assert np.array_equal(pig[idx][clear], Q.argmax(axis=1)[clear])


@pytest.mark.parametrize("prec", ["fp64", "fp32_wide"])
@pytest.mark.parametrize("case", LARGE, ids=[_id(*c) for c in LARGE])
def test_paper_a_large_converged_sampled(case, prec):
    sc = _case(*case)
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    res = pvi.vi_solve(m, precision=prec, eps=EPS, stop_rule="supnorm")
    assert res["status"] == pvi.PVI_OK
    assert max(abs(res["dmax"]), abs(res["dmin"])) < EPS
    V = pvi.value_get(m)
    pol, _ = pvi.policy_get(m)
    idx = W.sample_indices(o.n_states, 1500, seed=12)
    Q = o.q_states(V, idx)
    g = sc["gamma"]
    # rounding of the FP64 sweeps (about 1e-13 of |V| ~ 2e3) is far below gamma*eps
    assert np.abs(Q.max(axis=1) - V[idx]).max() < g * EPS * (1 + 1e-6)
    Qs = np.sort(Q, axis=1)
    clear = (Qs[:, -1] - Qs[:, -2]) > 2 * g * EPS * (1 + 1e-6)
    assert clear.mean() > 0.9
    assert np.array_equal(pol[idx][clear], Q.argmax(axis=1)[clear])
