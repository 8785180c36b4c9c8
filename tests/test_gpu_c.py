"""GPU parity of scenario C (weekday demand, random remaining life) through the C ABI.

Tolerances as for scenarios A and B.  The oracle enumerates every (demand,
arrival split) outcome; the GPU sums the same outcomes in two exact stages.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu

SMALL = [
    W.scenario_c(m=3, a_max=4, d_max=8, means=[3.0, 4.0, 3.5, 5.0, 4.5, 2.0, 2.5],
                 n=[5.0, 3.0, 4.0, 6.0, 5.0, 2.0, 3.0], c0=[0.0, 0.8, 1.5]),
    W.scenario_c(m=4, a_max=3, d_max=6, n_periods=3, means=[2.0, 3.0, 2.5], n=[4.0, 5.0, 3.0],
                 c0=[0.0, 0.5, 1.0, 2.0]),
    W.scenario_c(m=2, a_max=5, d_max=7, n_periods=2, means=[3.0, 4.0], n=[5.0, 5.0],
                 c0=[0.0, 1.0]),
    W.scenario_c(m=5, a_max=3, d_max=5, n_periods=2, means=[2.0, 2.5], n=[5.0, 4.0],
                 c0=[0.0, 1.6, 2.6, 2.8, 1.6]),
    W.scenario_c(m=3, a_max=9, d_max=12, n_periods=7, c0=[0.0, 2.0, 0.5]),
]
IDS = ["m3-P7", "m4-P3", "m2-P2", "m5-P2", "m3-R10"]


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def vhat(V, res, g):
    return V + g / (1.0 - g) * 0.5 * (res["dmax"] + res["dmin"])


@pytest.mark.parametrize("sc", SMALL, ids=IDS)
def test_one_backup(sc):
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    V = W.random_values(o.n_states, seed=21, scale=20.0, offset=-300.0)
    Vo, pio, gapo = o.sweep(V)
    Vg, pig, gapg = pvi.vi_backup(m, V, "fp64")
    assert relerr(Vg, Vo) < 1e-12
    clear = gapo > 1e-9
    assert np.array_equal(pig[clear], pio[clear])
    assert np.allclose(gapg[clear], gapo[clear], rtol=1e-8, atol=1e-9)
    V32, _, _ = pvi.vi_backup(m, V, "fp32")
    assert relerr(V32, Vo) < 1e-6


@pytest.mark.parametrize("sc", SMALL, ids=IDS)
def test_converged(sc):
    o = Oracle(sc)
    ref = o.solve()
    tight = o.solve(thr=1e-11)
    m = pvi.mdp_create(sc)
    res = pvi.vi_solve(m, precision="fp64")
    assert res["sweeps_fp64"] == ref["sweeps"]
    assert relerr(pvi.value_get(m), ref["V"]) < 1e-12
    pol, _ = pvi.policy_get(m)
    clear = tight["gap"] > 1e-6
    assert np.array_equal(pol[clear], tight["pi"][clear])
    g = sc["gamma"]
    res = pvi.vi_solve(m, precision="fp32")
    assert res["final_span"] < res["threshold"]
    assert relerr(vhat(pvi.value_get(m), res, g), vhat(ref["V"], ref, g)) < 1e-5
    pol, _ = pvi.policy_get(m)
    assert np.array_equal(pol[clear], tight["pi"][clear])


# remaining life on arrival that depends on the order size (c_1 != 0): one merge
# chain per order size on the GPU
ENDO = [
    W.scenario_c(m=3, a_max=4, d_max=8, c1=[0.0, 0.1, -0.1]),
    W.scenario_c(m=2, a_max=5, d_max=7, n_periods=2, means=[3.0, 4.0], n=[5.0, 5.0],
                 c0=[0.0, 1.0], c1=[0.0, -0.3]),
    W.scenario_c(m=4, a_max=3, d_max=6, n_periods=3, means=[2.0, 3.0, 2.5], n=[4.0, 5.0, 3.0],
                 c0=[0.0, 0.5, 1.0, 2.0], c1=[0.0, 0.4, -0.2, 0.3]),
    W.scenario_c(m=5, a_max=3, d_max=5, n_periods=2, means=[2.0, 2.5], n=[5.0, 4.0],
                 c0=[0.0, 1.9, 3.1, 3.1, 2.5], c1=[0.0, -0.03, -0.06, -0.03, -0.09]),
    W.scenario_c(m=3, a_max=9, d_max=12, n_periods=7, c0=[0.0, 1.0, 0.5], c1=[0.0, 0.4, 0.8]),
]
ENDO_IDS = ["m3", "m2-P2", "m4-P3", "m5-P2", "m3-R10"]


@pytest.mark.parametrize("sc", ENDO, ids=ENDO_IDS)
def test_endogenous_one_backup(sc):
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    for seed in (31, 32):
        V = W.random_values(o.n_states, seed=seed, scale=20.0, offset=-300.0)
        Vo, pio, gapo = o.sweep(V)
        Vg, pig, gapg = pvi.vi_backup(m, V, "fp64")
        assert relerr(Vg, Vo) < 1e-12
        clear = gapo > 1e-9
        assert np.array_equal(pig[clear], pio[clear])
        assert np.allclose(gapg[clear], gapo[clear], rtol=1e-8, atol=1e-9)
        V32, _, _ = pvi.vi_backup(m, V, "fp32")
        assert relerr(V32, Vo) < 1e-6


@pytest.mark.parametrize("sc", ENDO, ids=ENDO_IDS)
def test_endogenous_converged(sc):
    o = Oracle(sc)
    ref = o.solve()
    tight = o.solve(thr=1e-11)
    m = pvi.mdp_create(sc)
    res = pvi.vi_solve(m, precision="fp64")
    assert res["sweeps_fp64"] == ref["sweeps"]
    assert relerr(pvi.value_get(m), ref["V"]) < 1e-12
    pol, _ = pvi.policy_get(m)
    clear = tight["gap"] > 1e-6
    assert np.array_equal(pol[clear], tight["pi"][clear])
    g = sc["gamma"]
    res = pvi.vi_solve(m, precision="fp32")
    assert res["final_span"] < res["threshold"]
    assert relerr(vhat(pvi.value_get(m), res, g), vhat(ref["V"], ref, g)) < 1e-5
