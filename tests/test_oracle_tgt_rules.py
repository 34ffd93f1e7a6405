"""Pins for the three counting rules inside the oracle's reading of Alg. 1, each checked
against the mathematics that fixes it rather than against a retyped copy of the oracle's
formula:

  * NWalks: the smallest pair count that Hoeffding's inequality certifies, with the bound
    evaluated here in its exponential form and the union over the 2m directed estimates;
  * CalculateTau: the smallest truncation whose spectral tail bound is within eps/2,
    checked with 60-digit powers of lambda on both sides of the returned value;
  * the push stop rule (the Alg. 1 while loop): per source, the level at which the
    support volume first reaches the walk pairs still needed, with the walk vectors
    h_l = P^l e_s taken from exact rational matrix powers and the supports from boolean
    reachability, and the walk pairs per directed edge that follow from it.
"""
import decimal
import math
from fractions import Fraction

import numpy as np
import pytest

import graphgen


# ------------------------------------------------------------------ NWalks
def _hoeffding_fail(n, L, hmax, ds, eps):
    """Two-sided Hoeffding bound on P(|mean of n pair statistics - expectation| >= eps/4)
    for statistics confined to a range of width R = 2 L hmax / d_s (a walk sums at most L
    values in [0, hmax] on each side, and the pair statistic is divided by d_s)."""
    R = 2.0 * L * hmax / ds
    t = eps / 4.0
    return 2.0 * math.exp(-2.0 * n * t * t / (R * R))


def _hoeffding_min_n(L, hmax, ds, eps, delta, m):
    """Smallest n >= 1 with the failure bound at most delta / (2m): solved in log form,
    n* = ln(2 / target) R^2 / (2 t^2).  Returns (n, n*)."""
    R = 2.0 * L * hmax / ds
    t = eps / 4.0
    target = delta / (2.0 * m)
    nstar = math.log(2.0 / target) * R * R / (2.0 * t * t)
    return max(1, math.ceil(nstar)), nstar


def test_nwalks_is_the_smallest_hoeffding_count(orc):
    """Rules out: a wrong union bound (ln(2m/delta) instead of ln(4m/delta)), a range of
    width L*hmax/d_s instead of 2 L hmax/d_s, a deviation of eps/2 instead of eps/4, floor in
    place of ceiling, and a count without the max(1, .) floor."""
    checked = 0
    differs_with_half_union = 0
    for L in (1, 2, 3, 7, 20, 61):
        for hmax in (1.0, 0.5, 1.0 / 3.0, 0.137, 0.0123, 3.1e-4):
            for ds in (1, 2, 5, 17, 1000):
                for m in (10, 8000, 4984862):
                    for delta in (0.01, 0.1):
                        for eps in (0.05, 0.1, 0.3):
                            c = orc.cconst(eps, delta, m)
                            n = orc.nwalks(L, hmax, ds, c)
                            want, nstar = _hoeffding_min_n(L, hmax, ds, eps, delta, m)
                            if nstar > 1e17 or abs(nstar - round(nstar)) <= 1e-9 * max(nstar, 1.0):
                                continue  # too close to an integer to decide in FP64
                            assert n == want, (L, hmax, ds, m, delta, eps, n, want)
                            # the count meets the bound and one pair fewer would not
                            target = delta / (2.0 * m)
                            assert _hoeffding_fail(n, L, hmax, ds, eps) <= target * (1 + 1e-12)
                            if n > 1:
                                assert _hoeffding_fail(n - 1, L, hmax, ds, eps) > target
                            half = max(1, math.ceil(math.log(2.0 * m / delta) * nstar /
                                                    math.log(4.0 * m / delta)))
                            differs_with_half_union += half != n
                            checked += 1
    assert checked > 3000
    # the grid can tell the two union bounds apart
    assert differs_with_half_union > 100


# ------------------------------------------------------------------ CalculateTau
def _tau_exact(ds, dt, lam, eps):
    """Smallest tau >= 0 with (1/d_s + 1/d_t) lam^(tau+1) <= (eps/2)(1 - lam), from the log
    form; returns (tau, margin) where margin measures how far the decision at tau and tau-1
    is from the threshold (relative), so near-ties can be skipped."""
    w = 1.0 / ds + 1.0 / dt
    rhs = (eps / 2.0) * (1.0 - lam)
    x = math.log(rhs / w) / math.log(lam) - 1.0
    tau = max(0, math.ceil(x))
    return tau, abs(x - round(x))


@pytest.mark.parametrize("lam", [0.3, 0.6606, 0.9115, 0.99, 0.9999])
def test_tau_is_minimal(orc, lam):
    """Rules out: the exponent tau instead of tau + 1, eps in place of eps/2, a missing
    (1 - lambda) factor, a weight of 1/d_s alone, and any tau larger than needed."""
    D = decimal.Decimal
    decimal.getcontext().prec = 60
    lamD = D(lam)
    checked = 0
    for ds in (1, 2, 3, 10, 97, 30106):
        for dt in (1, 4, 10, 5000):
            for eps in (0.005, 0.05, 0.1, 0.3, 1.0):
                tau = orc.tau(ds, dt, lam, eps)
                want, margin = _tau_exact(ds, dt, lam, eps)
                if margin < 1e-9:
                    continue
                assert tau == want, (ds, dt, lam, eps, tau, want)
                # both sides of the returned tau at 60 significant digits
                w = D(1) / D(ds) + D(1) / D(dt)
                rhs = D(eps) / D(2) * (D(1) - lamD)
                assert w * lamD ** (tau + 1) <= rhs
                if tau > 0:
                    assert w * lamD ** tau > rhs
                assert orc.tau(dt, ds, lam, eps) == tau  # symmetric in (s, t)
                checked += 1
    assert checked > 100


def test_tau_cap(orc):
    assert orc.tau(2, 2, 0.9999, 0.01, tau_cap=50) == 50
    assert orc.tau(2, 2, 0.9999, 0.01) > 50


# ------------------------------------------------------------------ push stop rule
def _cycle_with_star():
    """An odd cycle C_9 (vertices 0..8) with a hub 9 joined to vertex 0 and to six leaves
    10..15: non-bipartite, with a hub row next to degree-2 and degree-1 rows."""
    e = [(i, (i + 1) % 9) for i in range(9)] + [(9, 0)] + [(9, 10 + k) for k in range(6)]
    return graphgen.from_edges(e, 16, name="c9_star6")


def _graphs():
    return [
        ("toy", graphgen.toy_graph()),
        ("er40", graphgen.largest_component(graphgen.er_gnm(40, 110, 3))),
        ("c9star", _cycle_with_star()),
    ]


def _reference_schedule(g, lam, eps, delta):
    """For every source s: the stop level ttau_s of the Alg. 1 while loop read as
    'push while vol(supp h_l) < sum over t with tau_st > l of NWalks(tau_st - l, hmax_l)',
    bounded by max_t tau_st, and the walk pairs of every directed edge.  h_l = P^l e_s in
    exact rationals (P = D^-1 A), supports by boolean reachability, tau from the log form,
    NWalks as max(1, ceil(c q^2)) with c from ln(4m/delta).  Returns (ttau[n], nreq[nnz],
    ambiguous[n]): a source is ambiguous when some count it needs lies within 1e-9 of an
    integer, where FP64 rounding may decide either way."""
    n, rp, ci = g.n, g.row_ptr, g.col_idx
    deg = np.diff(rp)
    m = g.nnz // 2
    c = 32.0 * math.log(4.0 * m / delta) / (eps * eps)
    nbrs = [list(map(int, ci[rp[x]:rp[x + 1]])) for x in range(n)]
    ttau = np.zeros(n, dtype=np.int64)
    nreq = np.zeros(g.nnz, dtype=np.int64)
    amb = np.zeros(n, dtype=bool)

    def nw(L, hmax, ds):
        x = c * float(Fraction(L) * hmax / ds) ** 2
        if abs(x - round(x)) < 1e-9 * max(1.0, x):
            return max(1, math.ceil(x)), True
        return max(1, math.ceil(x)), False

    for s in range(n):
        taus = []
        for t in nbrs[s]:
            tv, margin = _tau_exact(int(deg[s]), int(deg[t]), lam, eps)
            amb[s] |= margin < 1e-9
            taus.append(tv)
        maxtau = max(taus)
        h = [Fraction(0)] * n
        h[s] = Fraction(1)
        supp = {s}
        level = 0
        while True:
            vol = sum(int(deg[x]) for x in supp)
            hmax = max(h[x] for x in supp)
            need = 0
            for tv in taus:
                if tv > level:
                    k, a = nw(tv - level, hmax, int(deg[s]))
                    need += k
                    amb[s] |= a
            if vol >= need or level >= maxtau:
                break
            h = [sum((h[y] for y in nbrs[x]), Fraction(0)) / int(deg[x]) for x in range(n)]
            supp = {y for x in supp for y in nbrs[x]}
            level += 1
        ttau[s] = level
        hmax = max(h[x] for x in supp)
        for i, tv in enumerate(taus):
            if tv > level:
                k, a = nw(tv - level, hmax, int(deg[s]))
                nreq[rp[s] + i] = k
                amb[s] |= a
    return ttau, nreq, amb


def _check_schedule(orc, g, lam, eps, delta=0.01):
    _, o = orc.aesc(g, eps, lam, seed=1, delta=delta)
    ttau, nreq, amb = _reference_schedule(g, lam, eps, delta)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    ok = ~amb[rows]
    assert np.array_equal(o["ttau"][ok], ttau[rows][ok])
    assert np.array_equal(o["nreq"][ok], nreq[ok])
    return ttau, amb


@pytest.mark.parametrize("name", ["toy", "er40", "c9star"])
def test_push_stop_rule_and_walk_pairs(orc, name):
    """Rules out: the stop test evaluated with the wrong level's hmax or volume, walks
    counted for edges already covered by the push (tau_st <= l), a missing max_t tau_st
    bound, and n_req computed at a level other than the stop level."""
    g = dict(_graphs())[name]
    lam = graphgen.spectral_lambda(g)
    seen_levels = set()
    for eps in (0.05, 0.1, 0.2, 0.3, 0.6, 1.0):
        ttau, amb = _check_schedule(orc, g, lam, eps)
        seen_levels |= set(ttau[~amb].tolist())
    # the sweep exercises more than one stop level on each graph
    assert len(seen_levels) >= 2, seen_levels


def _need_at(g, lam, delta, eps, s, level, hmax):
    """Walk pairs still needed at `level` of source s (floats; for the eps search only)."""
    rp, ci = g.row_ptr, g.col_idx
    deg = np.diff(rp)
    c = 32.0 * math.log(4.0 * (g.nnz // 2) / delta) / (eps * eps)
    need = 0
    for t in ci[rp[s]:rp[s + 1]]:
        tv = _tau_exact(int(deg[s]), int(deg[t]), lam, eps)[0]
        if tv > level:
            need += max(1, math.ceil(c * ((tv - level) * hmax / int(deg[s])) ** 2))
    return need


def _tie_cases(g, lam, delta, max_level=3):
    """(eps, source, level) with vol_l == need_l at the level where the rule stops.  For
    fixed (s, l), h_l does not depend on eps and need_l(eps) is non-increasing in eps (c
    falls as 1/eps^2 and every tau_st with it), so the eps interval on which need_l equals
    vol_l, if any, is found by bisecting its two ends; its geometric middle is the case."""
    n, rp, ci = g.n, g.row_ptr, g.col_idx
    deg = np.diff(rp)
    P = g.dense_adjacency() / deg[:, None]
    out = []
    for s in range(n):
        h = np.zeros(n)
        h[s] = 1.0
        for level in range(max_level + 1):
            supp = np.flatnonzero(h > 0)
            vol = int(deg[supp].sum())
            hmax = float(h.max())

            def first_at_most(target):  # smallest eps (on a log scale) with need <= target
                lo, hi = math.log(1e-3), math.log(50.0)
                if _need_at(g, lam, delta, math.exp(hi), s, level, hmax) > target:
                    return None
                for _ in range(80):
                    mid = 0.5 * (lo + hi)
                    if _need_at(g, lam, delta, math.exp(mid), s, level, hmax) <= target:
                        hi = mid
                    else:
                        lo = mid
                return hi

            a, b = first_at_most(vol), first_at_most(vol - 1)
            if a is not None and (b is None or b - a > 1e-3):
                eps = math.exp(0.5 * (a + (b if b is not None else math.log(50.0))))
                if _need_at(g, lam, delta, eps, s, level, hmax) == vol:
                    out.append((eps, s, level))
            h = P @ h
    return out


@pytest.mark.parametrize("name", ["er40", "c9star"])
def test_push_stop_rule_ties_stop(orc, name):
    """At vol_l == need_l the loop must stop ('push while vol < need').  Finds such ties by
    bisection over eps, keeps those where the exact reference schedule stops at that very
    level, and checks the oracle's push depth there; a rule written with '<=' would push on."""
    g = dict(_graphs())[name]
    lam = graphgen.spectral_lambda(g)
    delta = 0.01
    checked = 0
    for eps, s, level in _tie_cases(g, lam, delta):
        ttau, _, amb = _reference_schedule(g, lam, eps, delta)
        if amb[s] or ttau[s] != level:
            continue  # stopped earlier at this eps, or a count too close to call
        _, o = orc.aesc(g, float(eps), lam, seed=1, delta=delta)
        assert o["ttau"][g.row_ptr[s]] == level, (eps, s, level)
        checked += 1
        if checked >= 8:
            break
    assert checked >= 1, "no tie case found"


def test_walk_pair_limit(orc):
    """A directed edge whose NWalks count reaches 2^32 pairs is refused: walk keys carry a
    32-bit index, so more pairs would repeat walks and the count's independence would fail.
    Just below the limit the estimate runs."""
    g = graphgen.largest_component(graphgen.er_gnm(16, 30, 2))
    lam = graphgen.spectral_lambda(g)
    with pytest.raises(ValueError):
        orc.aesc(g, 1e-4, lam, seed=1, tilde_tau_max=0)
    sc, o = orc.aesc(g, 0.3, lam, seed=1, tilde_tau_max=0)
    assert o["nreq"].max() < 2 ** 32
