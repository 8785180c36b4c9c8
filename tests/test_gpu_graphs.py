"""Captured sweep graphs against direct launches.

vi_solve replays an instantiated graph of eight sweeps (backup and span launches)
between host checks of the device stop flag; timed solves (time_kernels) launch
every kernel directly.  Both run the same kernels on the same tables in the same
order, so V, the policy and the sweep counts must be identical.  Each handle's graph
is replayed by several solves in a row, with other eager work and synchronisation
between them, and every replay is checked.
"""
import numpy as np
import pytest

import workloads as W
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu

CASES = {
    "A-fifo": W.config0(),
    "A-lifo": W.scenario_a(m=3, L=2, a_max=8, d_max=20, issuing="lifo"),
    "A-config1": W.config1(),
    "B": W.scenario_b(m=3, a_max=(6, 5), d_max=(12, 10), means=(4.0, 3.0), rho=0.5),
    "B1": W.scenario_b_paper(2, 1),
    "C": W.scenario_c(m=3, a_max=6, d_max=10, c0=[0.0, 1.0, 0.5]),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_wide"])
def test_graph_replays_equal_direct_launches(name, prec):
    sc = CASES[name]
    m = pvi.mdp_create(sc)
    ref = pvi.vi_solve(m, precision=prec, time_kernels=True)       # direct launches
    V0, (P0, G0) = pvi.value_get(m), pvi.policy_get(m)
    rng = np.random.default_rng([31, len(name)])
    for rep in range(3):
        res = pvi.vi_solve(m, precision=prec)                      # graph replays
        assert (res["sweeps_fp32"], res["sweeps_fp64"]) == (ref["sweeps_fp32"],
                                                            ref["sweeps_fp64"])
        assert np.array_equal(pvi.value_get(m), V0)
        P, G = pvi.policy_get(m)
        assert np.array_equal(P, P0) and np.array_equal(G, G0)
        # eager work on the same handle between replays
        Vr = rng.standard_normal(m.n_states)
        pvi.vi_backup(m, Vr, "fp64")


def test_fixed_sweeps_through_graphs():
    """fixed_sweeps that are not a multiple of the graph length still run exactly."""
    sc = W.config0()
    m = pvi.mdp_create(sc)
    for n in (1, 7, 8, 9, 23, 64):
        a = pvi.vi_solve(m, precision="fp64", fixed_sweeps=n)
        Va = pvi.value_get(m)
        b = pvi.vi_solve(m, precision="fp64", fixed_sweeps=n, time_kernels=True)
        assert a["sweeps_fp64"] == b["sweeps_fp64"] == n
        assert np.array_equal(Va, pvi.value_get(m))
