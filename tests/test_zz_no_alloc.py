"""vi_solve_noalloc (the solve whose working memory is a fixed device array of the
library) against vi_solve's FP64 solve, through the C ABI.

Same kernels in the same order, so V, policy, Q gap and sweep counts are compared
bit for bit.  Two calls in a row, the second on a smaller instance, show that the
array's leftovers from one call never reach the next.  Sizes beyond the array's
limits and unsupported options are refused.
"""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2303_10672_amd import pvi

pytestmark = pytest.mark.gpu


def outputs(n):
    return (torch.full((n,), np.nan, dtype=torch.float64, device="cuda"),
            torch.full((n,), -1, dtype=torch.int32, device="cuda"),
            torch.full((n,), np.nan, dtype=torch.float64, device="cuda"))


def solve_noalloc(sc, **kw):
    m = pvi.mdp_create(sc)
    v, pi, gap = outputs(m.n_states)
    torch.cuda.synchronize()
    r = pvi.vi_solve_noalloc(m, v.data_ptr(), pi.data_ptr(), gap.data_ptr(), **kw)
    return r, v.cpu().numpy(), pi.cpu().numpy(), gap.cpu().numpy()


def solve_alloc(sc, **kw):
    m = pvi.mdp_create(sc)
    r = pvi.vi_solve(m, precision="fp64", **kw)
    pol, gap = pvi.policy_get(m)
    return r, pvi.value_get(m), pol, gap


def same(a, b):
    ra, Va, pa, ga = a
    rb, Vb, pb, gb = b
    assert ra["sweeps_fp64"] == rb["sweeps_fp64"]
    assert ra["final_span"] == rb["final_span"]
    assert np.array_equal(Va, Vb)
    assert np.array_equal(pa, pb)
    assert np.array_equal(ga, gb)


def test_two_calls_second_smaller():
    # 4,084,101 states (the config-1 instance), then 121 states
    for sc in (W.config1(), W.config0()):
        same(solve_noalloc(sc), solve_alloc(sc))


def test_lifo_supnorm_v0_and_fixed_sweeps():
    sc = W.scenario_a_paper(3, 2, 1.0, "lifo")
    same(solve_noalloc(sc, stop_rule="supnorm"), solve_alloc(sc, stop_rule="supnorm"))
    sc = W.config1(request_id=7)
    v0 = W.random_values(4084101, seed=3)
    same(solve_noalloc(sc, v0=v0, fixed_sweeps=7), solve_alloc(sc, v0=v0, fixed_sweeps=7))


def test_no_device_memory_taken():
    sc = W.config1(request_id=3)
    solve_noalloc(sc)                     # first call: code objects and runtime staging
    m = pvi.mdp_create(sc)
    v, pi, gap = outputs(m.n_states)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    pvi.vi_solve_noalloc(m, v.data_ptr(), pi.data_ptr(), gap.data_ptr())
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0


def test_refused():
    big = W.scenario_a(m=5, L=2, a_max=20, d_max=60,
                       demand={"kind": "poisson", "mean": [4.0]})  # 85,766,121 states
    m = pvi.mdp_create(big)
    with pytest.raises(pvi.PviError) as e:
        pvi.vi_solve_noalloc(m, 1 << 20, 1 << 20, 1 << 20)
    assert e.value.status == pvi.PVI_E_INVALID and "limit" in str(e.value)
    mc = pvi.mdp_create(W.config3())
    v, pi, gap = outputs(16)
    with pytest.raises(pvi.PviError) as e:
        pvi.vi_solve_noalloc(mc, v.data_ptr(), pi.data_ptr(), gap.data_ptr())
    assert e.value.status == pvi.PVI_E_INVALID
    m0 = pvi.mdp_create(W.config0())
    with pytest.raises(pvi.PviError) as e:
        pvi.vi_solve_noalloc(m0, 0, pi.data_ptr(), gap.data_ptr())
    assert e.value.status == pvi.PVI_E_INVALID
