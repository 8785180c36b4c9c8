"""ctypes binding of libpvi.so (include/pvi.h), with the C ABI's names.

The binding only marshals arguments: scenario dictionaries become pvi_mdp_desc
structs and numpy arrays become pointers.  Every step of value iteration runs in
the library's HIP kernels.  There is no fallback: if libpvi.so is missing,
`load()` raises, and on a machine without a gfx950 device the solves return
PVI_E_DEVICE, which is raised here as PviError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpvi.so")

PVI_OK, PVI_E_INVALID, PVI_E_NOMEM, PVI_E_DEVICE = 0, 1, 2, 3
PVI_E_NOT_CONVERGED, PVI_E_NOT_READY, PVI_E_CANCELLED, PVI_E_BUSY = 4, 5, 6, 7
PVI_E_IO = 8
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "NOT_CONVERGED",
                5: "NOT_READY", 6: "CANCELLED", 7: "BUSY"}
FAMILY = {"A": 0, "B": 1, "C": 2, "B1": 3}
DEMAND = {"none": 0, "poisson": 1, "gamma": 2, "negbin": 3, "table": 4}
ISSUING = {"fifo": 0, "lifo": 1}
STOP_RULE = {"span": 0, "supnorm": 1, "periodic": 2}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_wide": 2}
MAX_PERIODS, MAX_LIFE = 7, 8


class PviError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("family", ctypes.c_int32), ("m", ctypes.c_int32),
        ("lead_time", ctypes.c_int32), ("n_periods", ctypes.c_int32),
        ("a_max", ctypes.c_int32 * 2), ("d_max", ctypes.c_int32 * 2),
        ("demand_kind", ctypes.c_int32 * 2),
        ("demand_mean", (ctypes.c_double * MAX_PERIODS) * 2),
        ("demand_shape", (ctypes.c_double * MAX_PERIODS) * 2),
        ("demand_table", ctypes.POINTER(ctypes.c_double) * 2),
        ("rul_c0", ctypes.c_double * MAX_LIFE), ("rul_c1", ctypes.c_double * MAX_LIFE),
        ("subst_rho", ctypes.c_double), ("c_var", ctypes.c_double * 2),
        ("c_fixed", ctypes.c_double), ("c_hold", ctypes.c_double),
        ("c_short", ctypes.c_double), ("c_waste", ctypes.c_double),
        ("c_rev", ctypes.c_double * 2), ("gamma", ctypes.c_double),
        ("issuing", ctypes.c_int32),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
        ("eps", ctypes.c_double), ("max_sweeps", ctypes.c_int32),
        ("fixed_sweeps", ctypes.c_int32), ("v0", ctypes.POINTER(ctypes.c_double)),
        ("stream", ctypes.c_void_p), ("check_every", ctypes.c_int32),
        ("time_kernels", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
        ("checkpoint_path", ctypes.c_char_p), ("checkpoint_every", ctypes.c_int32),
        ("resume", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("sweeps_fp32", ctypes.c_int32),
        ("sweeps_fp64", ctypes.c_int32), ("backup_launches", ctypes.c_int32 * 2),
        ("final_span", ctypes.c_double), ("threshold", ctypes.c_double),
        ("dmax", ctypes.c_double), ("dmin", ctypes.c_double), ("wall_ms", ctypes.c_double),
        ("backup_ms", ctypes.c_double * 2), ("logical_backups", ctypes.c_int64),
        ("executed_terms", ctypes.c_int64), ("vhat_shift", ctypes.c_double),
        ("device_ms", ctypes.c_double),
    ]

    def to_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


POLICY_KIND = {"table": 0, "base_stock": 1, "mod_base_stock": 2, "s_S": 3}
POLICY_PARAMS = 16


class TicketInfo(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32), ("small", ctypes.c_int32), ("worker", ctypes.c_int32),
        ("sweeps", ctypes.c_int32), ("status", ctypes.c_int32), ("launch", ctypes.c_int32),
        ("bytes", ctypes.c_int64), ("t_submit_ms", ctypes.c_double),
        ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
    ]


class RolloutOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("kind", ctypes.c_int32),
        ("table", ctypes.POINTER(ctypes.c_int32)), ("params", ctypes.POINTER(ctypes.c_int32)),
        ("n_policies", ctypes.c_int32), ("n_rollouts", ctypes.c_int32),
        ("warmup_days", ctypes.c_int32), ("horizon_days", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("start_state", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("product_kpis", ctypes.POINTER(ctypes.c_double)),
        ("product_stats", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None
_P = ctypes.POINTER


def load():
    """Load libpvi.so (built by paper_2303_10672_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2303_10672_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, _P(ctypes.c_double)
    sig = {
        "mdp_create": (i32, [_P(Desc), _P(vp)]),
        "mdp_destroy": (i32, [vp]),
        "mdp_num_states": (i64, [vp]),
        "mdp_num_actions": (i32, [vp]),
        "mdp_num_digits": (i32, [vp]),
        "mdp_encode": (i32, [vp, _P(i32), _P(i64)]),
        "mdp_decode": (i32, [vp, i64, _P(i32)]),
        "mdp_demand_pmf": (i32, [vp, i32, i32, dp]),
        "mdp_life_probs": (i32, [vp, dp]),
        "vi_solve": (i32, [vp, _P(Opts), _P(Result)]),
        "vi_backup": (i32, [vp, i32, dp, dp, _P(i32), dp]),
        "vi_solve_noalloc": (i32, [vp, _P(Opts), vp, vp, vp, _P(Result)]),
        "policy_get": (i32, [vp, _P(i32), dp]),
        "value_get": (i32, [vp, dp]),
        "checkpoint_read": (i32, [vp, ctypes.c_char_p, dp, _P(i32), _P(i32)]),
        "policy_get_device": (i32, [vp, vp, vp]),
        "pvi_server_create": (i32, [i64, i32, _P(vp)]),
        "pvi_server_destroy": (i32, [vp]),
        "vi_batch_submit": (i32, [vp, _P(vp), _P(Opts), i32, _P(ctypes.c_uint64)]),
        "vi_poll": (i32, [vp, ctypes.c_uint64, _P(Result)]),
        "vi_wait": (i32, [vp, ctypes.c_uint64, i64, _P(Result)]),
        "pvi_server_stats": (i32, [vp, dp, dp, _P(i64)]),
        "vi_ticket_info": (i32, [vp, ctypes.c_uint64, _P(TicketInfo)]),
        "policy_rollouts": (i32, [vp, _P(RolloutOpts), dp, dp, dp]),
        "heuristic_search": (i32, [vp, _P(RolloutOpts), dp, _P(i32)]),
        "pvi_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        if not hasattr(lib, name):
            continue
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st, what):
    if st != PVI_OK:
        msg = _lib.pvi_last_error().decode(errors="replace")
        raise PviError(st, f"{what}: {msg}")


def _dptr(a):
    return a.ctypes.data_as(_P(ctypes.c_double)) if a is not None else None


def _iptr(a):
    return a.ctypes.data_as(_P(ctypes.c_int32)) if a is not None else None


def make_desc(sc):
    """Marshal a scenario dictionary (see workloads.scenarios) into pvi_mdp_desc."""
    d = Desc()
    d.struct_size = ctypes.sizeof(Desc)
    d.family = FAMILY[sc["family"]]
    d.m, d.lead_time = sc["m"], sc["L"]
    d.n_periods = sc["n_periods"]
    d.a_max[0], d.a_max[1] = sc["a_max"]
    d.d_max[0], d.d_max[1] = sc["d_max"]
    keep = []
    for k in range(2):
        spec = sc["demand"][k]
        d.demand_kind[k] = DEMAND[spec["kind"]]
        means = spec.get("mean", [0.0])
        shape = spec.get("cv", spec.get("n", [0.0]))
        for t in range(MAX_PERIODS):
            d.demand_mean[k][t] = means[t] if t < len(means) else means[0]
            d.demand_shape[k][t] = shape[t] if t < len(shape) else shape[0]
        if spec["kind"] == "table":
            tab = np.ascontiguousarray(spec["table"], dtype=np.float64)
            keep.append(tab)
            d.demand_table[k] = _dptr(tab)
    for i in range(min(len(sc["rul_c0"]), MAX_LIFE)):
        d.rul_c0[i] = sc["rul_c0"][i]
        d.rul_c1[i] = sc["rul_c1"][i]
    d.subst_rho = sc["subst_rho"]
    c = sc["costs"]
    d.c_var[0], d.c_var[1] = c["var"]
    d.c_fixed, d.c_hold, d.c_short, d.c_waste = c["fixed"], c["hold"], c["short"], c["waste"]
    d.c_rev[0], d.c_rev[1] = c["rev"]
    d.gamma = sc["gamma"]
    d.issuing = ISSUING[sc.get("issuing", "fifo")]
    return d, keep


class Mdp:
    """Owning wrapper of a pvi_mdp handle."""

    def __init__(self, handle, sc):
        self.handle = handle
        self.sc = sc

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.mdp_destroy(h)

    @property
    def n_states(self):
        return int(_lib.mdp_num_states(self.handle))

    @property
    def n_actions(self):
        return int(_lib.mdp_num_actions(self.handle))


def mdp_create(sc):
    lib = load()
    d, keep = make_desc(sc)
    h = ctypes.c_void_p()
    _check(lib.mdp_create(ctypes.byref(d), ctypes.byref(h)), "mdp_create")
    del keep
    return Mdp(h, sc)


def mdp_destroy(m):
    h, m.handle = m.handle, None
    if h:
        _check(_lib.mdp_destroy(h), "mdp_destroy")


def mdp_num_states(m):
    return m.n_states


def mdp_num_actions(m):
    return m.n_actions


def mdp_num_digits(m):
    return int(_lib.mdp_num_digits(m.handle))


def mdp_encode(m, digits):
    dg = np.ascontiguousarray(digits, dtype=np.int32)
    out = ctypes.c_int64()
    _check(_lib.mdp_encode(m.handle, _iptr(dg), ctypes.byref(out)), "mdp_encode")
    return int(out.value)


def mdp_decode(m, idx):
    out = np.zeros(mdp_num_digits(m), dtype=np.int32)
    _check(_lib.mdp_decode(m.handle, int(idx), _iptr(out)), "mdp_decode")
    return out


def mdp_demand_pmf(m, product=0, period=0):
    out = np.zeros(m.sc["d_max"][product] + 1)
    _check(_lib.mdp_demand_pmf(m.handle, product, period, _dptr(out)), "mdp_demand_pmf")
    return out


def mdp_life_probs(m):
    out = np.zeros((m.sc["a_max"][0] + 1) * m.sc["m"])
    _check(_lib.mdp_life_probs(m.handle, _dptr(out)), "mdp_life_probs")
    return out.reshape(m.sc["a_max"][0] + 1, m.sc["m"])


def make_opts(precision="fp32", eps=None, max_sweeps=100000, fixed_sweeps=0, v0=None,
              stream=None, check_every=0, time_kernels=False, sc=None, stop_rule="span",
              checkpoint=None, checkpoint_every=0, resume=False):
    o = Opts()
    if checkpoint is not None:
        o.checkpoint_path = os.fsencode(checkpoint)
    o.checkpoint_every = int(checkpoint_every)
    o.resume = 1 if resume else 0
    o.stop_rule = STOP_RULE[stop_rule]
    o.struct_size = ctypes.sizeof(Opts)
    o.precision = PRECISION[precision]
    o.eps = float(eps if eps is not None else (sc["eps"] if sc else 1e-4))
    o.max_sweeps = int(max_sweeps)
    o.fixed_sweeps = int(fixed_sweeps)
    o.v0 = _dptr(v0)
    o.stream = stream
    o.check_every = int(check_every)
    o.time_kernels = 1 if time_kernels else 0
    return o


def vi_solve(m, precision="fp32", eps=None, max_sweeps=100000, fixed_sweeps=0, v0=None,
             stream=None, check_every=0, time_kernels=False, allow_not_converged=False,
             stop_rule="span", checkpoint=None, checkpoint_every=0, resume=False):
    """Blocking solve; returns the pvi_result fields as a dict.  checkpoint: file
    written every checkpoint_every FP64 sweeps and at the end, or read when resume."""
    v0a = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
    o = make_opts(precision, eps, max_sweeps, fixed_sweeps, v0a, stream, check_every,
                  time_kernels, m.sc, stop_rule, checkpoint, checkpoint_every, resume)
    r = Result()
    st = _lib.vi_solve(m.handle, ctypes.byref(o), ctypes.byref(r))
    if not (allow_not_converged and st == PVI_E_NOT_CONVERGED):
        _check(st, "vi_solve")
    return r.to_dict()


def vi_solve_noalloc(m, d_v, d_policy, d_gap, eps=None, max_sweeps=100000, fixed_sweeps=0,
                     v0=None, stream=None, stop_rule="span", allow_not_converged=False):
    """FP64 scenario-A solve with no device allocation (vi_solve_noalloc).  d_v,
    d_policy, d_gap: device addresses (e.g. tensor.data_ptr()) of float64[N_S],
    int32[N_S] and float64[N_S] outputs.  Returns the pvi_result fields as a dict."""
    v0a = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
    o = make_opts("fp64", eps, max_sweeps, fixed_sweeps, v0a, stream, 0, False, m.sc,
                  stop_rule)
    r = Result()
    st = _lib.vi_solve_noalloc(m.handle, ctypes.byref(o), ctypes.c_void_p(d_v),
                               ctypes.c_void_p(d_policy), ctypes.c_void_p(d_gap),
                               ctypes.byref(r))
    if not (allow_not_converged and st == PVI_E_NOT_CONVERGED):
        _check(st, "vi_solve_noalloc")
    return r.to_dict()


def vi_backup(m, v_in, precision="fp64"):
    """One backup of V: returns (T(V), argmax policy, FP64 Q gap)."""
    v = np.ascontiguousarray(v_in, dtype=np.float64)
    n = m.n_states
    out = np.zeros(n)
    pol = np.zeros(n, dtype=np.int32)
    gap = np.zeros(n)
    _check(_lib.vi_backup(m.handle, PRECISION[precision], _dptr(v), _dptr(out), _iptr(pol),
                          _dptr(gap)), "vi_backup")
    return out, pol, gap


def policy_get(m):
    n = m.n_states
    pol = np.zeros(n, dtype=np.int32)
    gap = np.zeros(n)
    _check(_lib.policy_get(m.handle, _iptr(pol), _dptr(gap)), "policy_get")
    return pol, gap


def value_get(m):
    v = np.zeros(m.n_states)
    _check(_lib.value_get(m.handle, _dptr(v)), "value_get")
    return v


def checkpoint_read(m, path):
    """(last V [N_S], FP64 sweeps, stopped) of a checkpoint file of this handle's MDP."""
    v = np.zeros(m.n_states)
    sweeps, stopped = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.checkpoint_read(m.handle, os.fsencode(path), _dptr(v), ctypes.byref(sweeps),
                                ctypes.byref(stopped)), "checkpoint_read")
    return v, int(sweeps.value), bool(stopped.value)


def policy_get_device(m, d_policy_ptr, stream=None):
    _check(_lib.policy_get_device(m.handle, ctypes.c_void_p(d_policy_ptr), stream),
           "policy_get_device")


def last_error():
    return load().pvi_last_error().decode(errors="replace")


class Server:
    """Request server (pvi_server_*): continuous batching of solves on one GPU."""

    def __init__(self, hbm_budget_bytes=0, small_batch=256):
        load()
        h = ctypes.c_void_p()
        _check(_lib.pvi_server_create(int(hbm_budget_bytes), int(small_batch), ctypes.byref(h)),
               "pvi_server_create")
        self.handle = h
        self._keep = {}

    def close(self):
        h, self.handle = self.handle, None
        if h:
            _check(_lib.pvi_server_destroy(h), "pvi_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, mdps, precision="fp32", eps=None, max_sweeps=100000, fixed_sweeps=0,
               stop_rule="span"):
        """vi_batch_submit: returns one ticket per MDP (same options for all)."""
        n = len(mdps)
        arr = (ctypes.c_void_p * n)(*[m.handle for m in mdps])
        o = make_opts(precision, eps, max_sweeps, fixed_sweeps, None, None, 0, False,
                      mdps[0].sc if n else None, stop_rule)
        t = (ctypes.c_uint64 * n)()
        _check(_lib.vi_batch_submit(self.handle, arr, ctypes.byref(o), n, t), "vi_batch_submit")
        tickets = list(t)
        for tk, m in zip(tickets, mdps):
            self._keep[tk] = m
        return tickets

    def poll(self, ticket):
        r = Result()
        st = _lib.vi_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(r))
        return st, (r.to_dict() if st != PVI_E_NOT_READY else None)

    def wait(self, ticket, timeout_us=-1):
        r = Result()
        st = _lib.vi_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(r))
        return st, r.to_dict()

    def ticket_info(self, ticket):
        """vi_ticket_info: state (queued/running/done), path, worker, sweeps so far, times."""
        i = TicketInfo()
        _check(_lib.vi_ticket_info(self.handle, ctypes.c_uint64(ticket), ctypes.byref(i)),
               "vi_ticket_info")
        return {"state": ("queued", "running", "done")[i.state], "small": bool(i.small),
                "worker": i.worker, "sweeps": i.sweeps, "status": i.status, "launch": i.launch,
                "bytes": i.bytes,
                "t_submit_ms": i.t_submit_ms, "t_start_ms": i.t_start_ms,
                "t_done_ms": i.t_done_ms}

    def stats(self):
        p50, p99 = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        _check(_lib.pvi_server_stats(self.handle, ctypes.byref(p50), ctypes.byref(p99),
                                     ctypes.byref(n)), "pvi_server_stats")
        return {"p50_ms": p50.value, "p99_ms": p99.value, "completed": n.value}


def pvi_server_create(hbm_budget_bytes=0, small_batch=256):
    return Server(hbm_budget_bytes, small_batch)


def pvi_server_destroy(server):
    server.close()


def vi_batch_submit(server, mdps, **kw):
    return server.submit(mdps, **kw)


def vi_poll(server, ticket):
    return server.poll(ticket)


def vi_wait(server, ticket, timeout_us=-1):
    return server.wait(ticket, timeout_us)


def pvi_server_stats(server):
    return server.stats()


def _rollout_opts(m, policy, table, params, n_rollouts, warmup, horizon, seed, start, stream):
    o = RolloutOpts()
    o.struct_size = ctypes.sizeof(RolloutOpts)
    o.kind = POLICY_KIND[policy]
    keep = []
    if policy == "table":
        o.n_policies = 1
        if table is not None:
            tab = np.ascontiguousarray(table, dtype=np.int32)
            if tab.shape != (m.n_states,):
                raise ValueError("table needs one action per state")
            keep.append(tab)
            o.table = _iptr(tab)
    else:
        rows = np.atleast_2d(np.asarray(params, dtype=np.int32))
        prm = np.zeros((rows.shape[0], POLICY_PARAMS), dtype=np.int32)
        prm[:, :rows.shape[1]] = rows
        keep.append(prm)
        o.params = _iptr(prm)
        o.n_policies = rows.shape[0]
    o.n_rollouts, o.warmup_days, o.horizon_days = int(n_rollouts), int(warmup), int(horizon)
    o.seed, o.start_state = int(seed), int(start)
    o.stream = stream
    return o, keep


def _product_outputs(o, n_rollouts, by_product, per_rollout):
    """Host arrays for the per-product KPIs (pkpi [n_pol, n_rollouts, 2, 3] when
    per_rollout, pstats [n_pol, 2, 6]) pointed to by the options."""
    if not by_product:
        return None, None
    pstats = np.zeros((o.n_policies, 2, 6))
    pkpi = np.zeros((o.n_policies, int(n_rollouts), 2, 3)) if per_rollout else None
    o.product_stats = _dptr(pstats)
    if per_rollout:
        o.product_kpis = _dptr(pkpi)
    return pkpi, pstats


def policy_rollouts(m, policy="table", table=None, params=None, n_rollouts=10000, warmup=100,
                    horizon=365, seed=0, start=0, stream=None, per_rollout=True,
                    by_product=False):
    """Rollouts of a policy (table: the given one, or the handle's solved policy when
    table is None) or of heuristic parameter rows.  Returns dict(stats [n_pol, 8],
    ret [n_pol, n_rollouts], kpi [n_pol, n_rollouts, 3]) (ret, kpi None unless
    per_rollout); with by_product (two-product families) also pstats [n_pol, 2, 6]
    (mean, sd of service, wastage, holding per product) and pkpi [n_pol, n_rollouts,
    2, 3]."""
    o, keep = _rollout_opts(m, policy, table, params, n_rollouts, warmup, horizon, seed, start,
                            stream)
    n = o.n_policies
    stats = np.zeros((n, 8))
    ret = np.zeros((n, int(n_rollouts))) if per_rollout else None
    kpi = np.zeros((n, int(n_rollouts), 3)) if per_rollout else None
    pkpi, pstats = _product_outputs(o, n_rollouts, by_product, per_rollout)
    null = _P(ctypes.c_double)()
    _check(_lib.policy_rollouts(m.handle, ctypes.byref(o), _dptr(stats),
                                _dptr(ret) if per_rollout else null,
                                _dptr(kpi) if per_rollout else null), "policy_rollouts")
    del keep
    out = {"stats": stats, "ret": ret, "kpi": kpi}
    if by_product:
        out.update(pstats=pstats, pkpi=pkpi)
    return out


def heuristic_search(m, policy, params, n_rollouts=10000, warmup=100, horizon=365, seed=0,
                     start=0, stream=None, by_product=False):
    """Simulation optimization over heuristic parameter rows: (best row index, stats),
    and with by_product the per-product statistics [n_pol, 2, 6] as a third item."""
    o, keep = _rollout_opts(m, policy, None, params, n_rollouts, warmup, horizon, seed, start,
                            stream)
    stats = np.zeros((o.n_policies, 8))
    _, pstats = _product_outputs(o, n_rollouts, by_product, False)
    best = ctypes.c_int32()
    _check(_lib.heuristic_search(m.handle, ctypes.byref(o), _dptr(stats), ctypes.byref(best)),
           "heuristic_search")
    del keep
    if by_product:
        return int(best.value), stats, pstats
    return int(best.value), stats
