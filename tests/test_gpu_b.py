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


WIDE = SMALL + [
    W.scenario_b(m=3, a_max=(14, 14), d_max=(20, 20), means=(5.0, 4.0), rho=0.5),
    W.scenario_b(m=2, a_max=(15, 9), d_max=(26, 11), means=(9.0, 3.0), rho=0.8),
]


@pytest.mark.parametrize("sc", WIDE, ids=IDS + ["R15-d20", "R16-d26"])
def test_tiled_kernels_match_per_cell_kernels(sc, monkeypatch):
    """The tiled stage kernels (one pass over each FIFO path for every oldest digit)
    and the per-cell kernels (PVI_B_TILED=0) take the same terms in the same order:
    one FP64 and one FP32 backup, three fixed sweeps and a converged solve give
    bit-identical values and policies."""
    o = Oracle(sc)
    V = W.random_values(o.n_states, seed=12, scale=5.0, offset=40.0)
    runs = []
    for tiled in ("0", None):
        if tiled is None:
            monkeypatch.delenv("PVI_B_TILED", raising=False)
        else:
            monkeypatch.setenv("PVI_B_TILED", tiled)
        m = pvi.mdp_create(sc)
        monkeypatch.delenv("PVI_B_TILED", raising=False)
        out = [pvi.vi_backup(m, V, "fp64"), pvi.vi_backup(m, V, "fp32")]
        pvi.vi_solve(m, precision="fp64", fixed_sweeps=3)
        out.append(pvi.value_get(m))
        res = pvi.vi_solve(m, precision="fp64")
        out.append((res["sweeps_fp64"], pvi.value_get(m), pvi.policy_get(m)))
        res = pvi.vi_solve(m, precision="fp32")
        out.append((res["sweeps_fp32"], res["sweeps_fp64"], pvi.value_get(m)))
        runs.append(out)
    (a64, a32, a3, (an, aV, ap), (af, ad, aW)), (b64, b32, b3, (bn, bV, bp), (bf, bd, bW)) = runs
    for x, y in zip(a64 + a32, b64 + b32):
        assert np.array_equal(x, y)
    assert np.array_equal(a3, b3)
    assert an == bn and np.array_equal(aV, bV)
    assert np.array_equal(ap[0], bp[0]) and np.array_equal(ap[1], bp[1])
    assert (af, ad) == (bf, bd) and np.array_equal(aW, bW)
    assert relerr(a64[0], o.sweep(V)[0]) < 1e-12
