"""An independent unit-by-unit model of the three scenarios, used only by tests.

The oracle writes each transition as the paper's digit formulas.  This module
instead keeps an explicit list of units, each with its days of life left, issues
the oldest first (youngest first for LIFO scenario A), throws away what reaches the
end of its life, and counts the
costs by looking at the units.  Building dense P(s'|s,a) and r(s,a) from it gives
a second, structurally different model of the same MDP, so the oracle's Bellman
operator can be checked against it on tiny instances.

State layouts (most significant digit first):
  A: [O_{L-1}, ..., O_1, X_m, ..., X_1]   (in-transit orders, then stock by life)
  B: [A_{m-1}, ..., A_1, B_{m-1}, ..., B_1]
  C: [tau, X_{m-1}, ..., X_1]
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import stats


def radices(sc):
    fam, m, L = sc["family"], sc["m"], sc["L"]
    if fam == "A":
        return [sc["a_max"][0] + 1] * (m + L - 1)
    if fam == "B":
        return [sc["a_max"][0] + 1] * (m - 1) + [sc["a_max"][1] + 1] * (m - 1)
    if fam == "B1":
        return [sc["a_max"][0] + 1] * m + [sc["a_max"][1] + 1] * m
    return [sc["n_periods"]] + [sc["a_max"][0] + 1] * (m - 1)


def encode(sc, digits):
    idx = 0
    for d, r in zip(digits, radices(sc)):
        assert 0 <= d < r
        idx = idx * r + int(d)
    return idx


def decode(sc, idx):
    rad = radices(sc)
    out = [0] * len(rad)
    for i in range(len(rad) - 1, -1, -1):
        out[i] = idx % rad[i]
        idx //= rad[i]
    return out


def n_states(sc):
    return int(np.prod(radices(sc)))


def n_actions(sc):
    if sc["family"] in ("B", "B1"):
        return (sc["a_max"][0] + 1) * (sc["a_max"][1] + 1)
    return sc["a_max"][0] + 1


def _units(counts_by_life):
    """Expand {life: count} into a list of lives, oldest (fewest days left) first."""
    out = []
    for life in sorted(counts_by_life):
        out += [life] * counts_by_life[life]
    return out


def _serve(units, demand):
    """Issue `demand` units, oldest first.  Returns (issued, leftover list)."""
    n = min(demand, len(units))
    return n, units[n:]


def _serve_youngest(units, demand):
    """Issue `demand` units, youngest (most days left) first."""
    n = min(demand, len(units))
    return n, units[:len(units) - n]


def step(sc, s, a, omega):
    """One day of the unit model.  Returns (next state index, reward)."""
    sn, rw, _ = day(sc, s, a, omega)
    return sn, rw


def day(sc, s, a, omega):
    """One day of the unit model: (next state index, reward, counts), where counts
    holds the day's demand, demand met, units expired, units received into stock and
    units held at the end of the day (scenario C: including tonight's expiries); for
    two products also "product", the same counts per product."""
    fam, m, L = sc["family"], sc["m"], sc["L"]
    c = sc["costs"]
    dig = decode(sc, s)
    if fam == "A":
        pipeline = dig[:L - 1]              # most recent order first
        stock = {life: dig[(L - 1) + (m - life)] for life in range(1, m + 1)}
        units = _units(stock)
        d = omega[0]
        serve = _serve_youngest if sc.get("issuing", "fifo") == "lifo" else _serve
        issued, left = serve(units, d)
        short = d - issued
        expired = sum(1 for u in left if u == 1)
        kept = [u - 1 for u in left if u > 1]
        reward = (-c["var"][0] * a - c["hold"] * len(kept) - c["short"] * short
                  - c["waste"] * expired)
        if L == 1:
            arriving, new_pipeline = a, []
        else:
            arriving, new_pipeline = pipeline[-1], [a] + pipeline[:-1]
        held = len(kept)
        kept += [m] * arriving
        counts = [sum(1 for u in kept if u == life) for life in range(m, 0, -1)]
        tally = {"demand": d, "met": issued, "expired": expired, "received": arriving,
                 "held": held}
        return encode(sc, new_pipeline + counts), float(reward), tally
    if fam == "B1":
        # lead time 1: stock of life m is yesterday's order; product b's unmet
        # customers (omega[2] of them accept) take product a's leftovers
        nb = sc["a_max"][1] + 1
        aA, aB = a // nb, a % nb
        stA = {life: dig[m - life] for life in range(1, m + 1)}
        stB = {life: dig[m + (m - life)] for life in range(1, m + 1)}
        dA, dB, du = omega
        hA, leftA = _serve(_units(stA), dA)
        hB, leftB = _serve(_units(stB), dB)
        assert du <= dB - hB
        hS, leftA = _serve(leftA, du)
        reward = (-(c["var"][0] * aA + c["var"][1] * aB) + c["rev"][0] * (hA + hS)
                  + c["rev"][1] * hB)
        nA = [u - 1 for u in leftA if u > 1]
        nB = [u - 1 for u in leftB if u > 1]
        dA_ = [aA] + [sum(1 for u in nA if u == life) for life in range(m - 1, 0, -1)]
        dB_ = [aB] + [sum(1 for u in nB if u == life) for life in range(m - 1, 0, -1)]
        tally = {"demand": dA + dB, "met": hA + hS + hB, "received": aA + aB,
                 "expired": sum(1 for u in leftA + leftB if u == 1), "held": len(nA) + len(nB)}
        # per product: product b's customers served by product a count for b
        tally["product"] = [
            {"demand": dA, "met": hA, "received": aA,
             "expired": sum(1 for u in leftA if u == 1), "held": len(nA)},
            {"demand": dB, "met": hB + hS, "received": aB,
             "expired": sum(1 for u in leftB if u == 1), "held": len(nB)}]
        return encode(sc, dA_ + dB_), float(reward), tally
    if fam == "B":
        nb = sc["a_max"][1] + 1
        aA, aB = a // nb, a % nb
        stA = {life: dig[(m - 1) - life] for life in range(1, m)}
        stB = {life: dig[(m - 1) + (m - 1) - life] for life in range(1, m)}
        stA[m], stB[m] = aA, aB             # L = 0: today's order is on hand
        dA, dB, k = omega
        hA, leftA = _serve(_units(stA), dA)
        hB, leftB = _serve(_units(stB), dB)
        hS, leftB = _serve(leftB, k)        # substitutes take product 1 leftovers
        reward = (-(c["var"][0] * aA + c["var"][1] * aB) + c["rev"][0] * hA
                  + c["rev"][1] * (hB + hS))
        nA = [u - 1 for u in leftA if u > 1]
        nB = [u - 1 for u in leftB if u > 1]
        dA_ = [sum(1 for u in nA if u == life) for life in range(m - 1, 0, -1)]
        dB_ = [sum(1 for u in nB if u == life) for life in range(m - 1, 0, -1)]
        tally = {"demand": dA + dB, "met": hA + hB + hS, "received": aA + aB,
                 "expired": sum(1 for u in leftA + leftB if u == 1), "held": len(nA) + len(nB)}
        # per product: product 0's customers served by product 1 count for product 0
        tally["product"] = [
            {"demand": dA, "met": hA + hS, "received": aA,
             "expired": sum(1 for u in leftA if u == 1), "held": len(nA)},
            {"demand": dB, "met": hB, "received": aB,
             "expired": sum(1 for u in leftB if u == 1), "held": len(nB)}]
        return encode(sc, dA_ + dB_), float(reward), tally
    # C
    cap = sc["a_max"][0]
    tau = dig[0]
    d, y_desc = omega[0], list(omega[1:])
    y = {m - i: y_desc[i] for i in range(m)}          # y[life]
    stock = {life: dig[m - life] for life in range(1, m)}
    held = {}
    for life in range(1, m):
        held[life] = min(stock[life] + y[life], cap)    # excess refused at delivery
    held[m] = y[m]
    units = _units(held)
    issued, left = _serve(units, d)
    short = d - issued
    expired = sum(1 for u in left if u == 1)
    reward = (-(c["fixed"] if a > 0 else 0.0) - c["hold"] * len(left)
              - c["short"] * short - c["waste"] * expired)
    kept = [u - 1 for u in left if u > 1]
    counts = [sum(1 for u in kept if u == life) for life in range(m - 1, 0, -1)]
    tally = {"demand": d, "met": issued, "expired": expired, "held": len(left),
             "received": sum(held.values()) - sum(stock.values())}
    return encode(sc, [(tau + 1) % sc["n_periods"]] + counts), float(reward), tally


def compositions(total, parts):
    """All (y_m, ..., y_1) of non-negative integers summing to total."""
    if parts == 1:
        yield (total,)
        return
    for first in range(total, -1, -1):
        for rest in compositions(total - first, parts - 1):
            yield (first,) + rest


def outcomes(sc, s, a, pmf0, pmf1, life_p):
    """(omega, probability) pairs for state s and action a; probabilities from scipy."""
    fam, m = sc["family"], sc["m"]
    if fam == "A":
        return [((d,), float(pmf0[0][d])) for d in range(len(pmf0[0]))]
    if fam == "B":
        nb = sc["a_max"][1] + 1
        aA = a // nb
        dig = decode(sc, s)
        stockA = aA + sum(dig[:m - 1])
        out = []
        for dA in range(len(pmf0[0])):
            u = max(dA - stockA, 0)
            for dB in range(len(pmf1)):
                for k in range(u + 1):
                    pk = stats.binom.pmf(k, u, sc["subst_rho"]) if u > 0 else 1.0
                    out.append(((dA, dB, k), float(pmf0[0][dA] * pmf1[dB] * pk)))
        return out
    if fam == "B1":
        dig = decode(sc, s)
        stockB = sum(dig[m:])
        out = []
        for dA in range(len(pmf0[0])):
            for dB in range(len(pmf1)):
                c = max(dB - stockB, 0)
                for du in range(c + 1):
                    pu = stats.binom.pmf(du, c, sc["subst_rho"]) if c > 0 else 1.0
                    out.append(((dA, dB, du), float(pmf0[0][dA] * pmf1[dB] * pu)))
        return out
    tau = decode(sc, s)[0]
    out = []
    p = life_p[a]                             # p[k-1] = P(life k)
    probs_desc = [p[m - 1 - i] for i in range(m)]
    for y in compositions(a, m):
        py = stats.multinomial.pmf(list(y), n=a, p=probs_desc) if a > 0 else 1.0
        for d in range(len(pmf0[tau])):
            out.append(((d,) + tuple(y), float(py * pmf0[tau][d])))
    return out


def dense_model(sc, pmf0, pmf1=None, life_p=None):
    """P[a, s, s'] and expected reward r[a, s] of the unit model."""
    S, A = n_states(sc), n_actions(sc)
    P = np.zeros((A, S, S))
    r = np.zeros((A, S))
    for s in range(S):
        for a in range(A):
            for om, pr in outcomes(sc, s, a, pmf0, pmf1, life_p):
                if pr == 0.0:
                    continue
                sn, rw = step(sc, s, a, om)
                P[a, s, sn] += pr
                r[a, s] += pr * rw
    return P, r


def bellman(P, r, gamma, V):
    Q = r + gamma * np.einsum("ast,t->as", P, V)
    return Q.max(axis=0), Q.argmax(axis=0), Q


def all_omegas(sc):
    fam, m = sc["family"], sc["m"]
    if fam == "A":
        return [(d,) for d in range(sc["d_max"][0] + 1)]
    if fam == "B":
        umax = sc["d_max"][0]
        return [(dA, dB, k) for dA in range(sc["d_max"][0] + 1)
                for dB in range(sc["d_max"][1] + 1) for k in range(umax + 1)]
    return None


def c_omegas(sc, a):
    return [(d,) + y for d in range(sc["d_max"][0] + 1)
            for y in compositions(a, sc["m"])]


__all__ = ["radices", "encode", "decode", "n_states", "n_actions", "step", "day", "outcomes",
           "dense_model", "bellman", "compositions", "all_omegas", "c_omegas",
           "itertools"]
