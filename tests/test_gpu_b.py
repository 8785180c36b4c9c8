"""GPU parity of scenario B (two products, substitution) through the C ABI.

Same tolerances as scenario A: FP64 backup 1e-12, FP32 storage 1e-6 per sweep,
converged V (bound midpoint) 1e-5, normwise relative to max |V|; policies equal
wherever the oracle's Q gap exceeds 1e-6 (1e-9 for single backups).
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu

C = W.scenarios._costs
SMALL = [
    W.scenario_b(m=3, a_max=(3, 4), d_max=(6, 5), means=(2.0, 1.5), rho=0.5),
    W.scenario_b(m=2, a_max=(5, 6), d_max=(8, 7), means=(3.0, 2.5), rho=0.3,
                 costs=C(var=(0.4, 0.6), rev=(1.0, 1.3))),
    W.scenario_b(m=4, a_max=(2, 2), d_max=(4, 4), means=(1.5, 1.0), rho=1.0),
    W.scenario_b(m=3, a_max=(4, 3), d_max=(7, 6), means=(2.5, 2.0), rho=0.0),
]
IDS = ["m3-rho.5", "m2-rho.3", "m4-rho1", "m3-rho0"]


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def vhat(V, res, g):
    return V + g / (1.0 - g) * 0.5 * (res["dmax"] + res["dmin"])


@pytest.mark.parametrize("sc", SMALL, ids=IDS)
def test_one_backup(sc):
    o = Oracle(sc)
    m = pvi.mdp_create(sc)
    V = W.random_values(o.n_states, seed=11, scale=5.0, offset=40.0)
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
    for prec in ("fp32", "fp32_wide"):
        res = pvi.vi_solve(m, precision=prec)
        assert res["final_span"] < res["threshold"]
        assert relerr(vhat(pvi.value_get(m), res, g), vhat(ref["V"], ref, g)) < 1e-5
        pol, _ = pvi.policy_get(m)
        assert np.array_equal(pol[clear], tight["pi"][clear])
