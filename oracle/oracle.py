"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` may
import this module.  The library under `paper_2303_10672_amd/` never does.

The demand and remaining-life tables are built here with scipy.stats, an
implementation independent of the GPU library's own table code:

* Scenario A gamma demand (Appendix A, demand equation): P(d) = F(d+1/2) - F(d-1/2)
  for d < d_max with F(x <= 0) = 0, and P(d_max) = 1 - F(d_max - 1/2).  The paper's
  "coefficient of variation" is read as sigma/mu, so shape = 1/cv^2, scale = mu*cv^2.
* Poisson demand (Scenario B description; folded the same way as Scenario C):
  P(d) = pmf(d) for d < d_max, P(d_max) = 1 - F(d_max - 1).
* Negative binomial demand (Appendix C, demand equation): n target successes and
  mean delta, p = n/(n+delta); P(d) = pmf(d) for d < d_max, P(d_max) = 1 - F(d_max-1).
* Remaining life on arrival (Appendix C, age-on-arrival equations):
  log(p_k(a)/p_1(a)) = c0_k + c1_k * a for k = 2..m, normalised to sum to one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
from scipy import stats

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pvi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_FAMILY = {"A": 0, "B": 1, "C": 2, "B1": 3}


def build(force=True):
    """Compile the oracle's C library in place (gcc, OpenMP, plain -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", _LIB, "-lm"])
    return _LIB


class _OrMdp(ctypes.Structure):
    _fields_ = [
        ("family", ctypes.c_int32), ("m", ctypes.c_int32), ("L", ctypes.c_int32),
        ("n_periods", ctypes.c_int32), ("a_max", ctypes.c_int32 * 2),
        ("d_max", ctypes.c_int32 * 2), ("pmf0", ctypes.POINTER(ctypes.c_double)),
        ("pmf1", ctypes.POINTER(ctypes.c_double)), ("rul_p", ctypes.POINTER(ctypes.c_double)),
        ("rho", ctypes.c_double), ("c_var", ctypes.c_double * 2), ("c_fixed", ctypes.c_double),
        ("c_hold", ctypes.c_double), ("c_short", ctypes.c_double), ("c_waste", ctypes.c_double),
        ("c_rev", ctypes.c_double * 2), ("gamma", ctypes.c_double), ("issuing", ctypes.c_int32),
        ("issue_p", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.or_num_states.restype = ctypes.c_int64
        lib.or_num_states.argtypes = [P(_OrMdp)]
        lib.or_num_actions.restype = ctypes.c_int32
        lib.or_num_actions.argtypes = [P(_OrMdp)]
        lib.or_decode.argtypes = [P(_OrMdp), ctypes.c_int64, P(ctypes.c_int32)]
        lib.or_encode.restype = ctypes.c_int64
        lib.or_encode.argtypes = [P(_OrMdp), P(ctypes.c_int32)]
        lib.or_q_states.argtypes = [P(_OrMdp), P(ctypes.c_double), P(ctypes.c_int64),
                                    ctypes.c_int64, P(ctypes.c_double)]
        lib.or_sweep.argtypes = [P(_OrMdp), P(ctypes.c_double), P(ctypes.c_double),
                                 P(ctypes.c_int32), P(ctypes.c_double)]
        lib.or_solve.argtypes = [P(_OrMdp), ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int32),
                                 P(ctypes.c_double), P(ctypes.c_double)]
        lib.or_transition.argtypes = [P(_OrMdp), ctypes.c_int64, ctypes.c_int32,
                                      P(ctypes.c_int32), P(ctypes.c_int64), P(ctypes.c_double)]
        lib.or_philox4x64_10.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64),
                                         P(ctypes.c_uint64)]
        lib.or_simulate.argtypes = [P(_OrMdp), ctypes.c_int32, P(ctypes.c_int32),
                                    P(ctypes.c_int32), P(ctypes.c_double), ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_uint64, ctypes.c_int64, P(ctypes.c_double),
                                    P(ctypes.c_double), P(ctypes.c_double)]
        lib.or_arrival_prob.restype = ctypes.c_double
        lib.or_arrival_prob.argtypes = [P(_OrMdp), ctypes.c_int32, P(ctypes.c_int32)]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


# ---------------------------------------------------------------- tables

def demand_pmf(spec, d_max, period=0):
    """Truncated demand PMF over 0..d_max with the tail folded into d_max."""
    kind = spec["kind"]
    d = np.arange(d_max + 1, dtype=np.float64)
    out = np.zeros(d_max + 1)
    if kind == "poisson":
        mu = spec["mean"][period]
        out[:d_max] = stats.poisson.pmf(d[:d_max], mu)
        out[d_max] = stats.poisson.sf(d_max - 1, mu)
    elif kind == "gamma":
        mu, cv = spec["mean"][period], spec["cv"][period]
        shape, scale = 1.0 / cv ** 2, mu * cv ** 2

        def F(x):
            return np.where(x <= 0.0, 0.0, stats.gamma.cdf(np.maximum(x, 0.0), shape,
                                                            scale=scale))
        out[:d_max] = F(d[:d_max] + 0.5) - F(d[:d_max] - 0.5)
        out[d_max] = stats.gamma.sf(d_max - 0.5, shape, scale=scale)
    elif kind == "negbin":
        n, mean = spec["n"][period], spec["mean"][period]
        p = n / (n + mean)
        out[:d_max] = stats.nbinom.pmf(d[:d_max], n, p)
        out[d_max] = stats.nbinom.sf(d_max - 1, n, p)
    elif kind == "none":
        out[:] = 0.0
        out[0] = 1.0
    else:
        raise ValueError(f"unknown demand kind {kind!r}")
    return out


def life_probabilities(sc):
    """p_k(a) for a in 0..a_max, k = 1..m (column k-1)."""
    m, a_max = sc["m"], sc["a_max"][0]
    c0 = np.asarray(sc["rul_c0"], dtype=np.float64)
    c1 = np.asarray(sc["rul_c1"], dtype=np.float64)
    out = np.zeros((a_max + 1, m))
    for a in range(a_max + 1):
        logits = np.zeros(m)
        logits[1:] = c0[1:m] + c1[1:m] * a
        w = np.exp(logits - logits.max())
        out[a] = w / w.sum()
    return out


def issue_probabilities(sc, pmf_a, pmf_b):
    """Scenario B as the paper runs it (Scenario B description, Appendix B outcome
    probabilities): P(h_a, h_b | I_a, I_b) for the units issued of each product.

    Product b issues h_b = min(D_b, I_b); its c = D_b - h_b unmet customers each
    accept product a with probability rho, so D_u ~ Bin(c, rho); product a issues
    h_a = min(D_a + D_u, I_a).  Summed here over D_a, D_b and D_u from their PMFs.
    (The paper's conditional P(D_u | I_b, D_b >= I_b) is read as the joint with
    {D_b >= I_b}, so that the five cases sum to one.)  Returns [I_a][I_b][h_a][h_b]."""
    m, rho = sc["m"], float(sc["subst_rho"])
    HA, HB = m * sc["a_max"][0] + 1, m * sc["a_max"][1] + 1
    da, db = len(pmf_a) - 1, len(pmf_b) - 1
    # distribution of D_a + Bin(c, rho) for every excess c
    tot = []
    for c in range(db + 1):
        bn = stats.binom.pmf(np.arange(c + 1), c, rho) if c > 0 else np.ones(1)
        tot.append(np.convolve(pmf_a, bn))
    P = np.zeros((HA, HB, HA, HB))
    for Ia in range(HA):
        for Ib in range(HB):
            for d in range(db + 1):
                if d < Ib:
                    dist, hb = pmf_a, d
                else:
                    dist, hb = tot[d - Ib], Ib
                capped = np.zeros(Ia + 1)
                capped[:min(Ia, len(dist))] = dist[:Ia]
                capped[Ia] += dist[Ia:].sum()
                P[Ia, Ib, :Ia + 1, hb] += pmf_b[d] * capped
    return P


class Oracle:
    """One scenario, ready for oracle sweeps and solves."""

    def __init__(self, sc):
        self.sc = sc
        self.lib = _load()
        fam = sc["family"]
        P = int(sc["n_periods"])
        self.pmf0 = np.ascontiguousarray(np.stack(
            [demand_pmf(sc["demand"][0], sc["d_max"][0], t) for t in range(P)]))
        if fam in ("B", "B1"):
            self.pmf1 = np.ascontiguousarray(demand_pmf(sc["demand"][1], sc["d_max"][1]))
        else:
            self.pmf1 = np.zeros(1)
        if fam == "B1":
            self.issue_p = np.ascontiguousarray(issue_probabilities(sc, self.pmf0[0], self.pmf1))
        else:
            self.issue_p = np.zeros(1)
        if fam == "C":
            self.rul = np.ascontiguousarray(life_probabilities(sc))
        else:
            self.rul = np.zeros(1)
        c = sc["costs"]
        self.s = _OrMdp()
        self.s.family = _FAMILY[fam]
        self.s.m, self.s.L, self.s.n_periods = sc["m"], sc["L"], P
        self.s.a_max[0], self.s.a_max[1] = sc["a_max"]
        self.s.d_max[0], self.s.d_max[1] = sc["d_max"]
        self.s.pmf0, self.s.pmf1, self.s.rul_p = _dp(self.pmf0), _dp(self.pmf1), _dp(self.rul)
        self.s.rho = sc["subst_rho"]
        self.s.c_var[0], self.s.c_var[1] = c["var"]
        self.s.c_fixed, self.s.c_hold = c["fixed"], c["hold"]
        self.s.c_short, self.s.c_waste = c["short"], c["waste"]
        self.s.c_rev[0], self.s.c_rev[1] = c["rev"]
        self.s.gamma = sc["gamma"]
        self.s.issuing = {"fifo": 0, "lifo": 1}[sc.get("issuing", "fifo")]
        self.s.issue_p = _dp(self.issue_p)
        self.ref = ctypes.byref(self.s)
        self.n_states = int(self.lib.or_num_states(self.ref))
        self.n_actions = int(self.lib.or_num_actions(self.ref))
        # span rule: eps (1 - gamma)/gamma; with gamma = 1 (Scenario B) the test of
        # Appendix B as written, span < eps
        g = sc["gamma"]
        self.threshold = sc["eps"] if g == 1.0 else sc["eps"] * (1.0 - g) / g

    # encoding --------------------------------------------------------------
    def n_digits(self):
        fam, m, L = self.sc["family"], self.sc["m"], self.sc["L"]
        return {"A": m + L - 1, "B": 2 * (m - 1), "C": m, "B1": 2 * m}[fam]

    def decode(self, idx):
        out = np.zeros(self.n_digits(), dtype=np.int32)
        self.lib.or_decode(self.ref, int(idx), _ip(out))
        return out

    def encode(self, digits):
        d = np.ascontiguousarray(digits, dtype=np.int32)
        return int(self.lib.or_encode(self.ref, _ip(d)))

    # transitions -----------------------------------------------------------
    def transition(self, s, a, omega):
        om = np.ascontiguousarray(omega, dtype=np.int32)
        sn = ctypes.c_int64()
        r = ctypes.c_double()
        self.lib.or_transition(self.ref, int(s), int(a), _ip(om), ctypes.byref(sn),
                               ctypes.byref(r))
        return int(sn.value), float(r.value)

    def arrival_prob(self, a, y_desc):
        y = np.ascontiguousarray(y_desc, dtype=np.int32)
        return float(self.lib.or_arrival_prob(self.ref, int(a), _ip(y)))

    # backups ---------------------------------------------------------------
    def q_states(self, V, states):
        V = np.ascontiguousarray(V, dtype=np.float64)
        st = np.ascontiguousarray(states, dtype=np.int64)
        q = np.zeros((len(st), self.n_actions))
        self.lib.or_q_states(self.ref, _dp(V), _lp(st), len(st), _dp(q))
        return q

    def initial_values(self):
        """V0: zero, except for the paper's Scenario B, whose V0(s) is the expected
        one-day sales revenue (Appendix B, initial value equation)."""
        if self.sc["family"] != "B1":
            return np.zeros(self.n_states)
        m = self.sc["m"]
        HA, HB = self.issue_p.shape[0], self.issue_p.shape[1]
        ra, rb = self.sc["costs"]["rev"]
        rev = np.zeros((HA, HB))
        for Ia in range(HA):
            for Ib in range(HB):
                P = self.issue_p[Ia, Ib]
                rev[Ia, Ib] = sum(P[ha, hb] * (ra * ha + rb * hb)
                                  for ha in range(Ia + 1) for hb in range(Ib + 1))
        V = np.zeros(self.n_states)
        for s in range(self.n_states):
            d = self.decode(s)
            V[s] = rev[int(d[:m].sum()), int(d[m:].sum())]
        return V

    def sweep(self, V):
        V = np.ascontiguousarray(V, dtype=np.float64)
        Vn = np.zeros(self.n_states)
        pi = np.zeros(self.n_states, dtype=np.int32)
        gap = np.zeros(self.n_states)
        self.lib.or_sweep(self.ref, _dp(V), _dp(Vn), _ip(pi), _dp(gap))
        return Vn, pi, gap

    def solve(self, thr=None, max_sweeps=100000, fixed_sweeps=0, v0=None, stop_rule="span"):
        """Value iteration.  Returns dict(V, pi, gap, sweeps, span, dmax, dmin, converged).

        stop_rule "span": max(V'-V) - min(V'-V) < thr (Appendix B); "supnorm":
        max |V' - V| < thr (Appendix A); "periodic": Appendix C's test over the last
        n_periods increments, with thr the relative tolerance.
        """
        thr = self.threshold if thr is None else float(thr)
        if v0 is None:
            V = self.initial_values()
        else:
            V = np.array(v0, dtype=np.float64)
        pi = np.zeros(self.n_states, dtype=np.int32)
        gap = np.zeros(self.n_states)
        st = np.zeros(4)
        rule = {"span": 0, "supnorm": 1, "periodic": 2}[stop_rule]
        rc = self.lib.or_solve(self.ref, thr, int(max_sweeps), int(fixed_sweeps), rule, _dp(V),
                               _ip(pi), _dp(gap), _dp(st))
        return {"V": V, "pi": pi, "gap": gap, "sweeps": int(st[0]), "span": st[1],
                "dmax": st[2], "dmin": st[3], "converged": rc == 0}

    # rollouts --------------------------------------------------------------
    def simulate(self, policy="table", table=None, params=None, n_rollouts=1000, warmup=100,
                 horizon=365, seed=0, start=0, by_product=False):
        """Rollouts of one tabulated policy or of several heuristic parameter vectors.

        policy: "table" (table = action per state), "base_stock" (params rows [S]),
        "mod_base_stock" ([S_0, S_1]) or "s_S" ([s_0, S_0, ..., s_6, S_6]).
        Returns (ret [n_pol, n_rollouts], kpi [n_pol, n_rollouts, 3]) with the KPIs
        service level %, wastage % and mean holding; with by_product (two-product
        families) also pkpi [n_pol, n_rollouts, 2, 3], the same KPIs per product
        (Appendix B, KPI tables)."""
        kind = {"table": 0, "base_stock": 1, "mod_base_stock": 2, "s_S": 3}[policy]
        if kind == 0:
            tab = np.ascontiguousarray(table, dtype=np.int32)
            assert tab.shape == (self.n_states,)
            prm = None
            n_pol = 1
        else:
            tab = None
            rows = np.atleast_2d(np.asarray(params, dtype=np.int32))
            prm = np.zeros((rows.shape[0], 16), dtype=np.int32)
            prm[:, :rows.shape[1]] = rows
            n_pol = rows.shape[0]
        mu = np.array([float(self.sc["demand"][k]["mean"][0]) for k in range(2)])
        ret = np.zeros((n_pol, n_rollouts))
        kpi = np.zeros((n_pol, n_rollouts, 3))
        if by_product:
            assert self.sc["family"] in ("B", "B1"), "per-product KPIs need two products"
            pkpi = np.zeros((n_pol, n_rollouts, 2, 3))
        null_i = ctypes.POINTER(ctypes.c_int32)()
        self.lib.or_simulate(self.ref, kind, _ip(tab) if tab is not None else null_i,
                             _ip(prm) if prm is not None else null_i, _dp(mu), n_pol,
                             int(n_rollouts), int(warmup), int(horizon),
                             ctypes.c_uint64(int(seed)), int(start), _dp(ret), _dp(kpi),
                             _dp(pkpi) if by_product else ctypes.POINTER(ctypes.c_double)())
        return (ret, kpi, pkpi) if by_product else (ret, kpi)


def philox4x64_10(counter, key):
    """Philox4x64-10 of one counter block (the oracle's generator, for its pins)."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    P = ctypes.POINTER(ctypes.c_uint64)
    _load().or_philox4x64_10(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out
