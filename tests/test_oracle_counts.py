"""Pins for the oracle's integer form of Alg. 1's Monte-Carlo statistic (source_counts):
the support of h_ttau and its values, the per-(edge, side, support vertex) visit counts,
and the Monte-Carlo sum formed from them.  Each is checked against something other than the
counting loop itself:

  * the support and h_ttau against exact rational matrix powers, h_l(x) = (P^l)[x, s];
  * the counts against walks re-run one by one through the separate path routine and
    tallied here, so a wrong edge index, a swapped side, a counted start position or a
    visit outside the support changes an entry;
  * the mean counts over many pairs against Chapman-Kolmogorov:
    E[c_side(x)] / n = sum_{b=1..L} (P^b)[start, x] for start = s (side 0) or t (side 1);
  * the sum over the support of h (c0 - c1) against the paper's per-pair loop (the MC the
    estimator itself accumulates), within the rounding of two FP64 summation orders.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen


def _small_graph():
    g = graphgen.largest_component(graphgen.er_gnm(24, 60, 11))
    return g, graphgen.spectral_lambda(g)


def _exact_powers(g, s, lmax):
    """Column s of P^l, l = 0..lmax, as exact fractions (P = D^-1 A): h_l(x) = (P^l)[x, s]."""
    deg = np.diff(g.row_ptr)
    h = [Fraction(0)] * g.n
    h[s] = Fraction(1)
    out = [h]
    for _ in range(lmax):
        nxt = []
        for x in range(g.n):
            acc = Fraction(0)
            for y in g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]:
                acc += h[int(y)]
            nxt.append(acc / int(deg[x]))
        h = nxt
        out.append(h)
    return out


def test_support_and_h_are_the_walk_vector(orc):
    """Rules out: a support taken from the wrong level (ttau +- 1), h values of another
    column or row of P^l, and a support list out of ascending order."""
    g, lam = _small_graph()
    checked = 0
    for s in range(0, g.n, 3):
        r = orc.source_counts(g, s, 0.2, lam, seed=2)
        tt = int(r["ttau"][0])
        assert np.all(r["ttau"] == tt)
        exact = _exact_powers(g, s, tt)[tt]
        supp = [x for x in range(g.n) if exact[x] != 0]
        assert r["supp"].tolist() == supp
        ref = np.array([float(exact[x]) for x in supp])
        np.testing.assert_allclose(r["h"], ref, rtol=1e-14, atol=0)
        checked += tt > 0
    assert checked >= 3  # some sources pushed at least one level


def test_counts_equal_walks_rerun_one_by_one(orc):
    """Every histogram entry equals the tally of the same walks re-run through the path
    routine: walk k of side sigma of edge (s, t) starts at s (sigma = 0) or t (sigma = 1), has
    key (s, t, sigma, k), and positions 1..L = tau - ttau count where h_ttau is nonzero."""
    g, lam = _small_graph()
    for s in (0, 5, 17):
        for kw in ({}, {"G": 8, "S": 24}):
            r = orc.source_counts(g, s, 0.35, lam, seed=7, **kw)
            pos = {int(x): p for p, x in enumerate(r["supp"])}
            row = g.col_idx[g.row_ptr[s]:g.row_ptr[s + 1]]
            assert r["hist"].shape == (row.size, 2, r["supp"].size)
            for i, t in enumerate(row):
                L = int(r["tau"][i] - r["ttau"][i])
                want = np.zeros((2, r["supp"].size), dtype=np.int64)
                for k in range(int(r["nreq"][i])):
                    for side in (0, 1):
                        hi, lo = orc.walk_key(7, s, int(t), side, k, kw.get("G", 1), kw.get("S", 0))
                        path = orc.walk_path(g, s if side == 0 else int(t), L, hi, lo)
                        for x in path[1:]:
                            if int(x) in pos:
                                want[side, pos[int(x)]] += 1
                assert np.array_equal(r["hist"][i], want), (s, i, kw)
                assert r["vis0"][i] == want[0].sum() and r["vis1"][i] == want[1].sum()


def test_mean_counts_follow_chapman_kolmogorov(orc):
    """With many pairs (small eps, the push held at two levels) the mean count per pair at
    each support vertex is close to sum_{b=1..L} P^b[start, x].  Rules out a swapped side, a
    start position counted (b = 0) or the last one dropped (b = L), and counts filed under the
    wrong support vertex.  Bound: one pair's count lies in [0, L] with mean mu, so its
    variance is at most L mu; six standard errors plus a small floor."""
    g, lam = _small_graph()
    s = 3
    r = orc.source_counts(g, s, 0.02, lam, seed=11, tilde_tau_max=2)
    assert int(r["ttau"][0]) == 2 and r["supp"].size > 4
    deg = np.diff(g.row_ptr).astype(float)
    A = np.zeros((g.n, g.n))
    for x in range(g.n):
        A[x, g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]] = 1.0
    P = A / deg[:, None]
    row = g.col_idx[g.row_ptr[s]:g.row_ptr[s + 1]]
    worst = 0.0
    for i, t in enumerate(row):
        n = int(r["nreq"][i])
        L = int(r["tau"][i] - r["ttau"][i])
        assert n > 5000 and L > 0
        for side, start in ((0, s), (1, int(t))):
            Pb = np.eye(g.n)
            mu = np.zeros(g.n)
            for _ in range(L):
                Pb = Pb @ P
                mu += Pb[start]
            mu = mu[r["supp"]]
            mean = r["hist"][i, side] / n
            tol = 6.0 * np.sqrt(L * np.maximum(mu, 1e-3) / n) + 1e-3
            z = np.abs(mean - mu) / tol
            worst = max(worst, float(z.max()))
            assert np.all(np.abs(mean - mu) <= tol), (i, side)
    assert worst > 0.0


def test_count_form_of_mc_matches_the_pair_loop(orc):
    """sum_x h(x) (c0(x) - c1(x)) over the ascending support equals the MC of the paper's
    per-pair loop up to FP64 rounding of the two summation orders: within 1e-13 of the sum of
    the absolute terms, sum_x h(x) (c0(x) + c1(x))."""
    g, lam = _small_graph()
    for s in range(g.n):
        r = orc.source_counts(g, s, 0.1, lam, seed=4)
        scale = (r["hist"][:, 0, :] + r["hist"][:, 1, :]) @ r["h"]
        assert np.all(np.abs(r["MCh"] - r["MC"]) <= 1e-13 * np.maximum(scale, 1e-300))
        # and the integer totals are the visit totals of the estimator
        assert np.array_equal(r["hist"][:, 0, :].sum(axis=1), r["vis0"])
        assert np.array_equal(r["hist"][:, 1, :].sum(axis=1), r["vis1"])


def test_counts_agree_with_the_all_edges_run(orc):
    """The per-edge outputs of one source are the all-edges oracle's entries of its row."""
    g, lam = _small_graph()
    _, o = orc.aesc(g, 0.25, lam, seed=9, G=4, S=26)
    for s in (1, 8, 20):
        r = orc.source_counts(g, s, 0.25, lam, seed=9, G=4, S=26)
        e0, e1 = g.row_ptr[s], g.row_ptr[s + 1]
        for k in ("tau", "ttau", "nreq", "D", "MC", "vis0", "vis1", "g"):
            assert np.array_equal(r[k], o[k][e0:e1]), k


def test_counts_reject_bad_sources(orc):
    g, lam = _small_graph()
    with pytest.raises(ValueError):
        orc.source_counts(g, -1, 0.2, lam, seed=1)
    with pytest.raises(ValueError):
        orc.source_counts(g, g.n, 0.2, lam, seed=1)
