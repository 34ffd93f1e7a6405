"""Pins for the oracle's TGT+ reading (Alg. 1).

  * push-only mode must reproduce the truncated resistance r_tau, computed here
    spectrally (an independent route from the oracle's pull recursion);
  * the truncation tau keeps |r - r_tau| <= eps/2 against the exact resistance;
  * the pure Monte-Carlo mode is unbiased for r_tau (mean over seeds);
  * the full estimator meets the eps contract of Sec. 2.1 against exact SC.
"""
import numpy as np
import pytest

import graphgen
from oracle import exact_sc


def _graph(n=60, m=200, seed=21):
    g = graphgen.largest_component(graphgen.er_gnm(n, m, seed))
    return g, graphgen.spectral_lambda(g)


def test_push_only_equals_truncated_resistance(orc):
    g, lam = _graph()
    sc, o = orc.aesc(g, 0.2, lam, seed=1, push_all=True)
    ce = graphgen.canonical_edges(g)
    # tau of edge (u, v): the entry at CSR position of u->v
    taus = []
    for u, v in ce:
        row = g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]
        taus.append(int(o["tau"][g.row_ptr[u] + int(np.searchsorted(row, v))]))
    ref = exact_sc.truncated_resistance(g.row_ptr, g.col_idx, g.n, ce.tolist(), taus)
    np.testing.assert_allclose(sc, ref, rtol=1e-10)
    assert np.all(o["nreq"] == 0)


@pytest.mark.parametrize("eps", [0.05, 0.2, 0.5])
def test_tau_bound_against_exact(orc, eps):
    g, lam = _graph(80, 260, 4)
    sc, o = orc.aesc(g, eps, lam, seed=1, push_all=True)
    ex = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n)
    assert np.max(np.abs(sc - ex)) <= eps / 2
    # tau is symmetric in (s, t)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for e in range(0, g.nnz, 7):
        s, t = rows[e], g.col_idx[e]
        f = g.row_ptr[t] + int(np.searchsorted(g.col_idx[g.row_ptr[t]:g.row_ptr[t + 1]], s))
        assert o["tau"][e] == o["tau"][f]


def test_pure_monte_carlo_is_unbiased(orc):
    g, lam = _graph(16, 34, 5)
    eps = 0.6
    _, o0 = orc.aesc(g, eps, lam, seed=1, push_all=True)
    ce = graphgen.canonical_edges(g)
    taus = [int(o0["tau"][g.row_ptr[u] + int(np.searchsorted(g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]], v))])
            for u, v in ce]
    rt = exact_sc.truncated_resistance(g.row_ptr, g.col_idx, g.n, ce.tolist(), taus)
    K = 48
    est = np.stack([orc.aesc(g, eps, lam, seed=100 + k, tilde_tau_max=0)[0] for k in range(K)])
    _, o = orc.aesc(g, eps, lam, seed=1, tilde_tau_max=0)
    assert np.all(o["ttau"] == 0)
    z = (est.mean(axis=0) - rt) / (est.std(axis=0, ddof=1) / np.sqrt(K) + 1e-300)
    assert np.max(np.abs(z)) < 5.0
    assert 0.2 < np.mean(z * z) < 3.0


@pytest.mark.parametrize("G,S", [(1, 0), (64, 20)])
def test_eps_contract_er300(orc, G, S):
    g, lam = _graph(300, 1200, 3)
    eps = 0.1
    sc, o = orc.aesc(g, eps, lam, seed=1, G=G, S=S)
    ex = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n)
    assert np.max(np.abs(sc - ex)) <= eps
    # Foster: exact for SC, biased low only by the truncation (<= eps/2 per edge)
    assert (g.n - 1) - g.m * eps / 2 <= sc.sum() <= (g.n - 1) + g.m * eps / 4
    L = o["tau"] - o["ttau"]
    assert np.all(o["vis0"] <= o["nreq"] * np.maximum(L, 0))
    assert np.all(o["vis1"] <= o["nreq"] * np.maximum(L, 0))


def test_query_matches_all_edges(orc):
    g, lam = _graph(120, 500, 6)
    sc, o = orc.aesc(g, 0.15, lam, seed=9)
    ce = graphgen.canonical_edges(g)
    pick = np.random.default_rng(0).choice(g.m, 25, replace=False)
    q = ce[pick][:, ::-1].copy()  # reversed orientation is the same undirected edge
    sq, oq = orc.aesc(g, 0.15, lam, seed=9, query=q)
    assert np.array_equal(sq, sc[pick])


def test_tilde_tau_cap_and_seed_sensitivity(orc):
    g, lam = _graph(100, 400, 8)
    _, o = orc.aesc(g, 0.2, lam, seed=1, tilde_tau_max=1)
    assert np.all(o["ttau"] <= 1)
    a, _ = orc.aesc(g, 0.2, lam, seed=1)
    b, _ = orc.aesc(g, 0.2, lam, seed=2)
    assert not np.array_equal(a, b)
    c, _ = orc.aesc(g, 0.2, lam, seed=1, nthreads=1)
    assert np.array_equal(a, c)


@pytest.mark.slow
def test_er2000_eps_contract(orc):
    # ER n=2000, m=8000, seed 1, largest component, eps=0.3, plain walks
    g = graphgen.largest_component(graphgen.er_gnm(2000, 8000, 1))
    lam = graphgen.spectral_lambda(g)
    sc, _ = orc.aesc(g, 0.3, lam, seed=1)
    ex = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n)
    assert np.max(np.abs(sc - ex)) <= 0.3
    assert abs(ex.sum() - (g.n - 1)) < 1e-8 * g.n
