"""Parity at the full sizes of configs 1-3, against the FP64 oracle.

* One backup of a seeded V over every state of config 1 (4,084,101 states) and
  config 2 (50,625 states; the oracle enumerates every (d_A, d_B, k) outcome, so the
  states are checked in chunks) in FP64 (1e-12), compensated FP32 and FP32 storage
  with FP64 sums (1e-6), normwise; the argmax wherever the oracle's best-minus-second
  Q exceeds 1e-9.  Config 3 (1,361,367 states; about 2.2 million outcome terms per
  state in the oracle) at 2,000 sampled states.
* Converged solves, certified by one oracle backup of the returned V (all states
  for configs 1 and 2, 1,000 sampled states for config 3): the returned V is
  T applied to the previous iterate, so T V - V must lie in [gamma dmin, gamma
  dmax] with dmin, dmax the solve's last increments; then V* lies within
  gamma / (1 - gamma) (dmax - dmin) / 2 of the bound midpoint V + gamma / (1 -
  gamma) (dmax + dmin) / 2 (MacQueen's bounds), which must be below 1e-5 of max|V|.
  The policy must equal the oracle's argmax of Q(V) wherever its gap exceeds 1e-6,
  and the Q gaps must agree.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu


def normwise(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def elementwise(a, b):
    return float((np.abs(a - b) / np.maximum(np.abs(b), 1e-300)).max())


def check_backup(Vg, pig, q_or_best, pi_or, gap_or, tol):
    assert normwise(Vg, q_or_best) < tol
    clear = gap_or > 1e-9
    assert np.array_equal(pig[clear], pi_or[clear])


def certify(res, V, pol, gap, TV, pi_or, gap_or, g):
    """The checks of the module docstring, on the states the oracle backed up."""
    dv = TV - V
    assert res["final_span"] < res["threshold"]
    assert dv.max() <= g * res["dmax"] + 1e-9 and dv.min() >= g * res["dmin"] - 1e-9
    half_width = g / (1.0 - g) * 0.5 * (res["dmax"] - res["dmin"])
    assert half_width / np.abs(V).max() < 1e-5
    clear = gap_or > 1e-6
    assert np.array_equal(pol[clear], pi_or[clear])
    assert np.allclose(gap[clear], gap_or[clear], rtol=1e-6, atol=1e-8)


def q_best(q):
    qs = np.sort(q, axis=1)
    return q.max(axis=1), q.argmax(axis=1).astype(np.int32), qs[:, -1] - qs[:, -2]


# ------------------------------------------------------------------ config 1

@pytest.fixture(scope="module")
def cfg1():
    sc = W.config1()
    return sc, Oracle(sc), pvi.mdp_create(sc)


@pytest.fixture(scope="module")
def cfg1_backup(cfg1):
    sc, o, m = cfg1
    V = W.random_values(o.n_states, seed=7, scale=50.0, offset=-800.0)
    return V, o.sweep(V)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("fp32_wide", 1e-6)])
def test_config1_one_backup_all_states(cfg1, cfg1_backup, prec, tol):
    sc, o, m = cfg1
    V, (Vo, pio, gapo) = cfg1_backup
    Vg, pig, gapg = pvi.vi_backup(m, V, prec)
    check_backup(Vg, pig, Vo, pio, gapo, tol)
    if prec == "fp64":
        assert elementwise(Vg, Vo) < 1e-12
        clear = gapo > 1e-9
        assert np.allclose(gapg[clear], gapo[clear], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_solve_certified_all_states(cfg1, prec):
    sc, o, m = cfg1
    res = pvi.vi_solve(m, precision=prec)
    V = pvi.value_get(m)
    pol, gap = pvi.policy_get(m)
    TV, pio, gapo = o.sweep(V)
    certify(res, V, pol, gap, TV, pio, gapo, sc["gamma"])


# ------------------------------------------------------------------ config 2

CHUNKS = 10


@pytest.fixture(scope="module")
def cfg2():
    sc = W.config2()
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    V = W.random_values(o.n_states, seed=12, scale=3.0, offset=120.0)
    backups = {p: pvi.vi_backup(m, V, p) for p in ("fp64", "fp32", "fp32_wide")}
    res = pvi.vi_solve(m, precision="fp32")
    sol = (res, pvi.value_get(m), *pvi.policy_get(m))
    return sc, o, V, backups, sol


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_config2_one_backup_all_states(cfg2, chunk):
    sc, o, V, backups, _ = cfg2
    idx = np.array_split(np.arange(o.n_states), CHUNKS)[chunk]
    best, arg, gp = q_best(o.q_states(V, idx))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("fp32_wide", 1e-6)):
        Vg, pig, _ = backups[prec]
        check_backup(Vg[idx], pig[idx], best, arg, gp, tol)


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_config2_solve_certified_all_states(cfg2, chunk):
    sc, o, _, _, (res, V, pol, gap) = cfg2
    idx = np.array_split(np.arange(o.n_states), CHUNKS)[chunk]
    best, arg, gp = q_best(o.q_states(V, idx))
    certify(res, V[idx], pol[idx], gap[idx], best, arg, gp, sc["gamma"])


# ------------------------------------------------------------------ config 3

@pytest.fixture(scope="module")
def cfg3():
    sc = W.config3()
    return sc, Oracle(sc), pvi.mdp_create(sc)


def test_config3_one_backup_sampled(cfg3):
    sc, o, m = cfg3
    V = W.random_values(o.n_states, seed=13, scale=30.0, offset=-900.0)
    idx = W.sample_indices(o.n_states, 2000, seed=5)
    best, arg, gp = q_best(o.q_states(V, idx))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("fp32_wide", 1e-6)):
        Vg, pig, _ = pvi.vi_backup(m, V, prec)
        check_backup(Vg[idx], pig[idx], best, arg, gp, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config3_solve_certified_sampled(cfg3, prec):
    sc, o, m = cfg3
    res = pvi.vi_solve(m, precision=prec)
    V = pvi.value_get(m)
    pol, gap = pvi.policy_get(m)
    idx = W.sample_indices(o.n_states, 1000, seed=6 if prec == "fp64" else 8)
    best, arg, gp = q_best(o.q_states(V, idx))
    certify(res, V[idx], pol[idx], gap[idx], best, arg, gp, sc["gamma"])
