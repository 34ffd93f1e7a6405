"""Pins for the oracle's walk generator (Alg. 2 with the Eq. (5) choice) against the
Markov chain it must sample: endpoint and visit frequencies against powers of P = D^-1 A."""
import numpy as np
import pytest
from scipy import stats

import graphgen


def _small_graph():
    # non-regular, non-bipartite, so P^L, P^(L-1) and P^(L+1) rows differ
    return graphgen.largest_component(graphgen.er_gnm(24, 50, 8))


def _P(g):
    A = g.dense_adjacency()
    return A / A.sum(axis=1, keepdims=True)


def _chi2_p(counts, probs):
    W = counts.sum()
    if np.any(counts[probs == 0] > 0):
        return 0.0  # mass where the chain cannot be
    exp = W * probs
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    chi2 = ((obs - ex) ** 2 / ex).sum()
    return stats.chi2.sf(chi2, len(obs) - 1)


@pytest.mark.parametrize("L", [1, 3, 4])
def test_endpoint_distribution_matches_PL(orc, L):
    g = _small_graph()
    P = _P(g)
    s = 0
    W = 60000
    ep, vi = orc.walks_histogram(g, np.full(W, s), L, seed=11)
    assert ep.sum() == W and vi.sum() == W * L
    PL = np.linalg.matrix_power(P, L)[s]
    assert _chi2_p(ep, PL) > 1e-5
    # the neighbouring step counts are rejected: positions are counted exactly
    for wrong in (L - 1, L + 1):
        if wrong < 0:
            continue
        Pw = np.linalg.matrix_power(P, wrong)[s]
        assert _chi2_p(ep, Pw) < 1e-12
    expv = W * sum(np.linalg.matrix_power(P, l)[s] for l in range(1, L + 1))
    assert np.abs(vi - expv).sum() / (W * L) < 0.02


def test_saba_lane_marginal_and_correlation(orc):
    # G > 1 correlates the members of a group but each member is still an exact walk
    g = _small_graph()
    P = _P(g)
    s, L, G, S = 3, 3, 64, 20
    n_groups = 6000
    ends = np.zeros(g.n, dtype=np.int64)
    for grp in range(n_groups):
        hi, lo = orc.walk_key(5, s, 0, 0, grp * G + 17, G, S)
        ends[orc.walk_path(g, s, L, hi, lo)[-1]] += 1
    assert _chi2_p(ends, np.linalg.matrix_power(P, L)[s]) > 1e-5

    def distinct(G_, S_):
        tot = 0
        for grp in range(200):
            e = set()
            for r in range(64):
                hi, lo = orc.walk_key(5, s, 0, 0, grp * 64 + r, G_, S_)
                e.add(int(orc.walk_path(g, s, L, hi, lo)[-1]))
            tot += len(e)
        return tot / 200

    assert distinct(64, 20) < 0.5 * distinct(1, 0)


def test_histogram_depends_only_on_source_multiset(orc):
    g = graphgen.largest_component(graphgen.er_gnm(500, 2000, 2))
    src = graphgen.uniform_sources(g, 20000, 3)
    a = orc.walks_histogram(g, src, 9, seed=7, G=8, S=22)
    b = orc.walks_histogram(g, np.sort(src), 9, seed=7, G=8, S=22)
    c = orc.walks_histogram(g, src[::-1], 9, seed=7, G=8, S=22, nthreads=1)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    d = orc.walks_histogram(g, src, 9, seed=8, G=8, S=22)
    assert not np.array_equal(a[1], d[1])


def test_long_walk_visits_stationary(orc):
    g = graphgen.largest_component(graphgen.er_gnm(60, 200, 9))
    d = g.degrees
    src = graphgen.uniform_sources(g, 3000, 1)
    _, vi = orc.walks_histogram(g, src, 400, seed=2)
    freq = vi / vi.sum()
    pi = d / d.sum()
    assert np.abs(freq - pi).sum() / 2 < 0.02


def test_isolated_source_rejected(orc):
    g = graphgen.from_edges([(0, 1)], 3)
    with pytest.raises(ValueError):
        orc.walks_histogram(g, np.array([2]), 3, seed=1)
