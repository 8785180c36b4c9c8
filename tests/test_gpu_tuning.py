"""The scenario-C merge block width chosen by timing at a handle's first solve
against the LDS rule (PVI_TUNE=0): the block width only changes how the work is cut
into workgroups, not any sum, so the solves must be bit-identical."""
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
