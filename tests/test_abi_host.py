"""Host-side checks of the C ABI (no GPU): exports, validation, encoding, tables."""
import ctypes
import os
import re
import struct

import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle, life_probabilities
from paper_2303_10672_amd import pvi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pvi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(pvi.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_sizes_match_header_layout():
    # pvi_mdp_desc: 5 int32 + 3x2 int32 + 2x7x2 doubles + 2 ptrs + 16 doubles + ...
    assert ctypes.sizeof(pvi.Desc) % 8 == 0
    assert ctypes.sizeof(pvi.Opts) == 72
    assert pvi.Opts.checkpoint_path.offset == 56
    assert ctypes.sizeof(pvi.Result) == 112
    assert pvi.Result.vhat_shift.offset == 96 and pvi.Result.device_ms.offset == 104
    assert ctypes.sizeof(pvi.RolloutOpts) == 80
    assert pvi.RolloutOpts.product_kpis.offset == 64


def test_binding_layouts_match_the_header_as_compiled(tmp_path):
    """Sizes and field offsets of the result and option structs as a C compiler lays
    them out from include/pvi.h, against the Python binding's ctypes structures."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = {"pvi_result": (pvi.Result, [k for k, _ in pvi.Result._fields_]),
              "pvi_solve_opts": (pvi.Opts, [k for k, _ in pvi.Opts._fields_])}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pvi.h"', "int main(void) {"]
    for st, (_, names) in fields.items():
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for n in names:
            lines.append(f'printf("{st} {n} %zu\\n", offsetof({st}, {n}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        st, key, val = line.split()
        got[(st, key)] = int(val)
    for st, (cls, names) in fields.items():
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for n in names:
            assert got[(st, n)] == getattr(cls, n).offset, (st, n)


def test_rollout_options_are_validated_before_the_device():
    lib = ctypes.CDLL(pvi.LIB_PATH)
    P = ctypes.POINTER
    lib.policy_rollouts.argtypes = [ctypes.c_void_p, P(pvi.RolloutOpts), P(ctypes.c_double),
                                    P(ctypes.c_double), P(ctypes.c_double)]
    lib.heuristic_search.argtypes = [ctypes.c_void_p, P(pvi.RolloutOpts), P(ctypes.c_double),
                                     P(ctypes.c_int32)]
    m = pvi.mdp_create(W.config0())
    st = np.zeros(8 * 11)
    null = P(ctypes.c_double)()

    def run(policy="base_stock", table=None, params=[[5]], **kw):
        o, keep = pvi._rollout_opts(m, policy, table, params, kw.get("n", 10), kw.get("w", 5),
                                    kw.get("h", 20), 0, kw.get("start", 0), None)
        for k, v in kw.get("set", {}).items():
            setattr(o, k, v)
        return lib.policy_rollouts(m.handle, ctypes.byref(o), pvi._dptr(st), null, null)

    assert run(policy="mod_base_stock", params=[[3, 3]]) == pvi.PVI_E_INVALID  # A has no B rule
    assert run(policy="s_S", params=[[1, 2] * 7]) == pvi.PVI_E_INVALID
    assert run(n=0) == pvi.PVI_E_INVALID
    assert run(h=0) == pvi.PVI_E_INVALID
    assert run(w=-1) == pvi.PVI_E_INVALID
    assert run(start=121) == pvi.PVI_E_INVALID
    assert run(set={"struct_size": 60}) == pvi.PVI_E_INVALID
    msg = pvi._lib.pvi_last_error().decode()
    assert "struct_size" in msg
    # per-product outputs need two products ...
    out = np.zeros(12)
    assert run(set={"product_stats": pvi._dptr(out)}) == pvi.PVI_E_INVALID
    assert "two-product" in pvi._lib.pvi_last_error().decode()
    assert run(set={"product_kpis": pvi._dptr(out)}) == pvi.PVI_E_INVALID
    # ... and are not read when struct_size stops before them, so a caller built
    # before they existed (64 bytes) is served: these requests reach the device
    assert run(set={"product_stats": pvi._dptr(out), "struct_size": 72}) == pvi.PVI_E_DEVICE
    assert run(set={"product_kpis": pvi._dptr(out), "struct_size": 64}) == pvi.PVI_E_DEVICE
    assert run(set={"kind": 9}) == pvi.PVI_E_INVALID
    # heuristic orders are uncapped, so parameters and the 32-bit counts are bounded
    assert run(params=[[1 << 21]]) == pvi.PVI_E_INVALID
    assert "2^20" in pvi._lib.pvi_last_error().decode()
    assert run(params=[[5], [-(1 << 21)]]) == pvi.PVI_E_INVALID
    assert run(params=[[1 << 16]], h=1 << 14) == pvi.PVI_E_INVALID
    assert "32-bit" in pvi._lib.pvi_last_error().decode()
    assert run(params=[[1 << 20]], h=1 << 10) == pvi.PVI_E_INVALID   # 2 (m + L) 2^20 2^10
    assert run(params=[[1 << 20]], h=1 << 8) == pvi.PVI_E_DEVICE
    bad = np.zeros(121, np.int32)
    bad[7] = 11                                       # 11 actions: 0..10
    assert run(policy="table", table=bad) == pvi.PVI_E_INVALID
    assert run(policy="table", table=None) == pvi.PVI_E_NOT_READY   # nothing solved yet
    assert run(set={"n_rollouts": 1 << 30, "n_policies": 4}) == pvi.PVI_E_INVALID
    # a valid request reaches the device, which this machine lacks
    assert run(params=[[S] for S in range(11)]) == pvi.PVI_E_DEVICE
    o, keep = pvi._rollout_opts(m, "table", np.zeros(121, np.int32), None, 5, 1, 5, 0, 0, None)
    best = ctypes.c_int32()
    assert lib.heuristic_search(m.handle, ctypes.byref(o), pvi._dptr(st),
                                ctypes.byref(best)) == pvi.PVI_E_INVALID


def test_older_struct_sizes_are_accepted_and_new_fields_checked():
    """A descriptor or options struct that ends before the newest field (issuing,
    stop_rule) is accepted with that field read as 0; a full-size struct with a bad
    value is rejected; anything shorter than the first layout is rejected."""
    lib = ctypes.CDLL(pvi.LIB_PATH)
    lib.mdp_create.argtypes = [ctypes.POINTER(pvi.Desc), ctypes.POINTER(ctypes.c_void_p)]
    lib.mdp_destroy.argtypes = [ctypes.c_void_p]
    d, keep = pvi.make_desc(W.config0())
    h = ctypes.c_void_p()
    d.issuing = 7
    assert lib.mdp_create(ctypes.byref(d), ctypes.byref(h)) == pvi.PVI_E_INVALID
    d.struct_size = pvi.Desc.issuing.offset        # the layout before `issuing`
    assert lib.mdp_create(ctypes.byref(d), ctypes.byref(h)) == pvi.PVI_OK
    lib.mdp_destroy(h)
    d.struct_size = pvi.Desc.issuing.offset - 8
    assert lib.mdp_create(ctypes.byref(d), ctypes.byref(h)) == pvi.PVI_E_INVALID
    sc = W.scenario_b(m=2, a_max=(2, 2), d_max=(4, 4), means=(1.0, 1.0), rho=0.5)
    d2, keep2 = pvi.make_desc(sc)
    d2.issuing = pvi.ISSUING["lifo"]                  # LIFO is defined for scenario A only
    assert lib.mdp_create(ctypes.byref(d2), ctypes.byref(h)) == pvi.PVI_E_INVALID

    m = pvi.mdp_create(W.config0())
    lib.vi_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(pvi.Opts), ctypes.c_void_p]
    o = pvi.make_opts("fp64", sc=W.config0())
    o.stop_rule = 5
    assert lib.vi_solve(m.handle, ctypes.byref(o), None) == pvi.PVI_E_INVALID
    o.struct_size = pvi.Opts.stop_rule.offset          # older callers: rule reads as span
    assert lib.vi_solve(m.handle, ctypes.byref(o), None) == pvi.PVI_E_DEVICE
    o.struct_size = pvi.Opts.stop_rule.offset - 4
    assert lib.vi_solve(m.handle, ctypes.byref(o), None) == pvi.PVI_E_INVALID


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_counts_encoding_and_pmfs_match_oracle(cfg):
    sc = W.config_by_index(cfg)
    m = pvi.mdp_create(sc)
    o = Oracle(sc)
    assert m.n_states == o.n_states and m.n_actions == o.n_actions
    for s in W.sample_indices(o.n_states, 200, seed=cfg):
        dg = pvi.mdp_decode(m, s)
        assert np.array_equal(dg, o.decode(s))
        assert pvi.mdp_encode(m, dg) == s
    for t in range(sc["n_periods"]):
        assert np.allclose(pvi.mdp_demand_pmf(m, 0, t), o.pmf0[t], rtol=1e-12, atol=1e-15)
    if sc["family"] == "B":
        assert np.allclose(pvi.mdp_demand_pmf(m, 1, 0), o.pmf1, rtol=1e-12, atol=1e-15)
    if sc["family"] == "C":
        assert np.allclose(pvi.mdp_life_probs(m), life_probabilities(sc), rtol=1e-13)


def test_gamma_pmf_small_shape_matches_oracle():
    for cv in (0.3, 0.5, 1.0, 1.5, 3.0):
        sc = W.scenario_a(m=2, L=1, a_max=5, d_max=100,
                          demand={"kind": "gamma", "mean": [4.0], "cv": [cv]})
        m = pvi.mdp_create(sc)
        assert np.allclose(pvi.mdp_demand_pmf(m), Oracle(sc).pmf0[0], rtol=1e-11, atol=1e-15)


def _bad(**kw):
    sc = W.config0()
    sc.update(kw)
    return sc


@pytest.mark.parametrize("sc,msg", [
    (_bad(gamma=1.0), "gamma"),
    (_bad(gamma=0.0), "gamma"),
    (_bad(m=0), "m out of range"),
    (_bad(m=9), "m out of range"),
    (_bad(L=0), "L >= 1"),
    (_bad(a_max=[32, 0]), "a_max"),
    (_bad(d_max=[-1, 0]), "d_max"),
    (_bad(n_periods=3), "n_periods"),
    (W.scenario_c(m=1), "m >= 2"),
    (dict(W.scenario_b(), L=1), "L = 0"),
    (dict(W.scenario_b(), subst_rho=1.5), "subst_rho"),
])
def test_invalid_descriptors_are_rejected(sc, msg):
    with pytest.raises(pvi.PviError) as e:
        pvi.mdp_create(sc)
    assert e.value.status == pvi.PVI_E_INVALID
    assert msg in str(e.value)


def test_bad_demand_table_rejected():
    sc = W.config0()
    sc["demand"][0] = {"kind": "table", "table": [0.5] * 21}
    with pytest.raises(pvi.PviError):
        pvi.mdp_create(sc)
    sc["demand"][0] = {"kind": "table", "table": [1.0] + [0.0] * 20}
    m = pvi.mdp_create(sc)
    assert pvi.mdp_demand_pmf(m)[0] == 1.0


def test_encode_rejects_out_of_range_digits():
    m = pvi.mdp_create(W.config0())
    with pytest.raises(pvi.PviError):
        pvi.mdp_encode(m, [11, 0])
    with pytest.raises(pvi.PviError):
        pvi.mdp_decode(m, 121)


def test_results_not_ready_before_a_solve():
    m = pvi.mdp_create(W.config0())
    with pytest.raises(pvi.PviError) as e:
        pvi.policy_get(m)
    assert e.value.status == pvi.PVI_E_NOT_READY


def test_no_device_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    m = pvi.mdp_create(W.config0())
    with pytest.raises(pvi.PviError) as e:
        pvi.vi_solve(m)
    assert e.value.status == pvi.PVI_E_DEVICE


def test_lead_time_one_two_product_family_validation():
    """The paper's scenario B: gamma = 1 only for this family, L = 1, and a clear
    INVALID (before any device work) when one product's stock vectors exceed what the
    GPU stages in LDS."""
    lib = ctypes.CDLL(pvi.LIB_PATH)
    lib.mdp_create.argtypes = [ctypes.POINTER(pvi.Desc), ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    d, keep = pvi.make_desc(W.scenario_b_paper(2, 1))
    assert lib.mdp_create(ctypes.byref(d), ctypes.byref(h)) == pvi.PVI_OK
    d.lead_time = 0
    assert lib.mdp_create(ctypes.byref(d), ctypes.byref(h)) == pvi.PVI_E_INVALID
    a, keep2 = pvi.make_desc(W.config0())
    a.gamma = 1.0
    assert lib.mdp_create(ctypes.byref(a), ctypes.byref(h)) == pvi.PVI_E_INVALID
    big = pvi.mdp_create(W.scenario_b1(m=4, a_max=(1, 16), means=(1.0, 5.0)))
    with pytest.raises(pvi.PviError) as e:
        pvi.vi_solve(big, precision="fp64")
    assert e.value.status == pvi.PVI_E_INVALID and "on the GPU" in str(e.value)
    m = pvi.mdp_create(W.scenario_b_paper(3, 1))
    assert (m.n_states, m.n_actions) == (16777216, 256)


def test_checkpoint_options_are_checked_before_the_device(tmp_path):
    """Checkpoint options and files are validated on the host: a bad interval, a
    missing path, a missing file (PVI_E_IO), a file that is not a checkpoint or is of
    another version (PVI_E_INVALID); checkpoint_read reports the same."""
    m = pvi.mdp_create(W.config0())

    def solve(**kw):
        o = pvi.make_opts("fp64", 1e-4, 1000, 0, None, None, 0, False, m.sc, "span",
                          kw.get("checkpoint"), kw.get("every", 0), kw.get("resume", False))
        return pvi._lib.vi_solve(m.handle, ctypes.byref(o), None)

    err = lambda: pvi._lib.pvi_last_error().decode()
    assert solve(every=-1, checkpoint="x") == pvi.PVI_E_INVALID
    assert solve(every=5) == pvi.PVI_E_INVALID and "checkpoint_path" in err()
    assert solve(resume=True) == pvi.PVI_E_INVALID
    missing = str(tmp_path / "none.ckpt")
    assert solve(checkpoint=missing, resume=True) == pvi.PVI_E_IO
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint at all, just some bytes of text" * 2)
    assert solve(checkpoint=str(junk), resume=True) == pvi.PVI_E_INVALID
    assert "not a checkpoint" in err()
    short = tmp_path / "short.ckpt"
    short.write_bytes(b"PVICKPT1")
    assert solve(checkpoint=str(short), resume=True) == pvi.PVI_E_IO
    # right magic, another descriptor's fingerprint
    hdr = struct.pack("<8sIIQqiiiiii", b"PVICKPT1", 1, 0, 12345, 121, 11, 0, 3, 0, 1, 0)
    other = tmp_path / "other.ckpt"
    other.write_bytes(hdr + np.zeros(121).tobytes())
    assert solve(checkpoint=str(other), resume=True) == pvi.PVI_E_INVALID
    assert "another MDP" in err()
    newer = tmp_path / "newer.ckpt"
    newer.write_bytes(struct.pack("<8sIIQqiiiiii", b"PVICKPT1", 3, 0, 0, 121, 11, 0, 3, 0, 1, 0))
    assert solve(checkpoint=str(newer), resume=True) == pvi.PVI_E_INVALID
    assert "version" in err()
    with pytest.raises(pvi.PviError):
        pvi.checkpoint_read(m, missing)
    with pytest.raises(pvi.PviError):
        pvi.checkpoint_read(m, str(other))


def test_scenario_c_beyond_2_31_states_serves_heuristic_rollouts_only():
    """Scenario C at m = 8 (12,607,619,787 states) is created for rollouts of
    heuristics; a solve, a single backup or a table policy on it is refused before the
    device, a heuristic rollout reaches the device (absent here).  Other families stay
    limited to 2^31 states."""
    m = pvi.mdp_create(W.scenario_c_paper(8, 1))
    assert m.n_states == 7 * 21 ** 7
    o = pvi.make_opts("fp64", 1e-4, 1000, 0, None, None, 0, False, m.sc, "periodic")
    assert pvi._lib.vi_solve(m.handle, ctypes.byref(o), None) == pvi.PVI_E_INVALID
    assert "heuristic rollouts only" in pvi._lib.pvi_last_error().decode()
    st = np.zeros(8)
    null = ctypes.POINTER(ctypes.c_double)()
    prm = [[8, 19, 8, 15, 8, 18, 7, 18, 8, 14, 3, 13, 4, 16]]
    ro, keep = pvi._rollout_opts(m, "s_S", None, prm, 10, 5, 20, 0, 0, None)
    assert pvi._lib.policy_rollouts(m.handle, ctypes.byref(ro), pvi._dptr(st), null, null) == \
        pvi.PVI_E_DEVICE
    ro, keep = pvi._rollout_opts(m, "table", None, None, 10, 5, 20, 0, 0, None)
    assert pvi._lib.policy_rollouts(m.handle, ctypes.byref(ro), pvi._dptr(st), null, null) == \
        pvi.PVI_E_INVALID
    assert "2^31" in pvi._lib.pvi_last_error().decode()
    with pytest.raises(pvi.PviError, match="2\\^31"):
        pvi.mdp_create(W.scenario_a(m=5, L=4, a_max=20, d_max=30))   # 21^8 states
