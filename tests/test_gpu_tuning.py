"""Choices the autotuner times at a shape's first solve, against the fixed rules
(PVI_TUNE=0): scenario C's merge block width, and scenario A's tiles per wavefront G
and path points per staged chunk CH.  They only change how the work is cut into
workgroups and staged, not any sum, so every choice must give bit-identical solves."""
import os

import numpy as np
import pytest

import workloads as W
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tuned_merge_equals_rule(prec):
    sc = W.config3(a_max=10)                     # m = 5: merge levels 3 and 4 are tuned
    os.environ["PVI_TUNE"] = "0"
    try:
        plain = pvi.mdp_create(sc)
        a = pvi.vi_solve(plain, precision=prec, stop_rule="periodic")
    finally:
        del os.environ["PVI_TUNE"]
    tuned = pvi.mdp_create(sc)
    b = pvi.vi_solve(tuned, precision=prec, stop_rule="periodic")
    assert (a["sweeps_fp32"], a["sweeps_fp64"]) == (b["sweeps_fp32"], b["sweeps_fp64"])
    assert np.array_equal(pvi.value_get(plain), pvi.value_get(tuned))
    assert np.array_equal(pvi.policy_get(plain)[0], pvi.policy_get(tuned)[0])


@pytest.mark.parametrize("width", [4, 8, 12, 16, 32])
def test_every_block_width_equals_rule(width):
    """Each block width the tuner may pick (forced with PVI_C_BLOCK) gives the same
    FP64 and FP32-storage solves as the LDS rule."""
    sc = W.config3(a_max=10)
    ref = {}
    os.environ["PVI_TUNE"] = "0"
    try:
        plain = pvi.mdp_create(sc)
        for prec in ("fp64", "fp32"):
            pvi.vi_solve(plain, precision=prec, stop_rule="periodic")
            ref[prec] = (pvi.value_get(plain), pvi.policy_get(plain)[0])
    finally:
        del os.environ["PVI_TUNE"]
    os.environ["PVI_C_BLOCK"] = str(width)
    try:
        forced = pvi.mdp_create(sc)
        for prec in ("fp64", "fp32"):
            pvi.vi_solve(forced, precision=prec, stop_rule="periodic")
            assert np.array_equal(pvi.value_get(forced), ref[prec][0])
            assert np.array_equal(pvi.policy_get(forced)[0], ref[prec][1])
    finally:
        del os.environ["PVI_C_BLOCK"]


A_SHAPES = {
    "config1": W.config1(),
    "paper-m5L2": W.scenario_a_paper(5, 2, 1.0, "fifo"),
    "paper-m3L2": W.scenario_a_paper(3, 2, 1.0, "fifo"),
    "m3L1-R13": W.scenario_a(m=3, L=1, a_max=12, d_max=30),
}


def _solve_a(sc, env, monkeypatch):
    for k in ("PVI_TUNE", "PVI_A_GROUP", "PVI_A_CHUNK"):
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    m = pvi.mdp_create(sc)
    out = {}
    for prec in ("fp64", "fp32"):
        r = pvi.vi_solve(m, precision=prec)
        out[prec] = (r["sweeps_fp32"], r["sweeps_fp64"], pvi.value_get(m), pvi.policy_get(m))
    return out


def _same(a, b):
    for prec in a:
        assert a[prec][:2] == b[prec][:2]
        assert np.array_equal(a[prec][2], b[prec][2])
        assert np.array_equal(a[prec][3][0], b[prec][3][0])
        assert np.array_equal(a[prec][3][1], b[prec][3][1])


@pytest.mark.parametrize("name", list(A_SHAPES))
def test_scenario_a_choices_equal_rule(name, monkeypatch):
    sc = A_SHAPES[name]
    rule = _solve_a(sc, {"PVI_TUNE": "0"}, monkeypatch)
    _same(_solve_a(sc, {}, monkeypatch), rule)          # the tuned choice
    R = sc["a_max"][0] + 1
    gmax = min(16, 64 // R)
    rmax = 8 if R <= 8 else 16 if R <= 16 else 24 if R <= 24 else 32
    for G in sorted({1, 2, gmax} & set(range(1, gmax + 1))):
        chmax = max(1, 64 // ((rmax // 8) * G))
        for CH in sorted({1, max(1, chmax // 2), chmax}):
            _same(_solve_a(sc, {"PVI_A_GROUP": str(G), "PVI_A_CHUNK": str(CH)}, monkeypatch),
                  rule)
