"""Pins for the exact spanning-centrality oracle (Sec. 2.1 definition of SC).

The pseudoinverse route is checked against things it does not compute itself:
closed forms, exact integer matrix-tree counts, brute-force enumeration,
Foster's theorem, bridges and networkx's independent resistance routine.
"""
import os
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import graphgen
from oracle import exact_sc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_toy():
    rows = []
    total = None
    with open(os.path.join(GOLDEN, "fig1_toy.txt")) as f:
        for line in f:
            if line.startswith("# spanning_trees"):
                total = int(line.split()[-1])
            if line.startswith("#") or not line.strip():
                continue
            u, v, a, b = map(int, line.split())
            rows.append(((u, v), Fraction(a, b)))
    return rows, total


def test_fig1_toy_graph():
    g = graphgen.toy_graph()
    rows, total = _load_toy()
    edges = graphgen.canonical_edges(g).tolist()
    assert [tuple(e) for e in edges] == [r[0] for r in rows]
    # K4 has 4^2 = 16 spanning trees (Cayley); each of its 6 edges lies in 16*3/6 = 8 of
    # them, so deleting A-D leaves 8 trees.
    assert total == 8 == exact_sc.spanning_tree_count(edges, 4)
    sc = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n)
    np.testing.assert_allclose(sc, [float(r[1]) for r in rows], rtol=0, atol=1e-12)
    assert exact_sc.sc_matrix_tree(edges, 4) == [r[1] for r in rows]
    assert sum(r[1] for r in rows) == 3  # Foster: n - 1


@pytest.mark.parametrize("n", [3, 5, 8, 13])
def test_closed_forms(n):
    # cycle C_n: (n-1)/n ; complete K_n: 2/n ; path (a tree): 1
    cyc = graphgen.from_edges([(i, (i + 1) % n) for i in range(n)], n)
    np.testing.assert_allclose(exact_sc.sc_pinv(cyc.row_ptr, cyc.col_idx, n), (n - 1) / n, atol=1e-12)
    kn = graphgen.from_edges([(i, j) for i in range(n) for j in range(i + 1, n)], n)
    np.testing.assert_allclose(exact_sc.sc_pinv(kn.row_ptr, kn.col_idx, n), 2.0 / n, atol=1e-12)
    path = graphgen.from_edges([(i, i + 1) for i in range(n - 1)], n)
    np.testing.assert_allclose(exact_sc.sc_pinv(path.row_ptr, path.col_idx, n), 1.0, atol=1e-12)


@pytest.mark.parametrize("a,b", [(1, 4), (2, 3), (3, 5), (4, 4)])
def test_complete_bipartite(a, b):
    n = a + b
    g = graphgen.from_edges([(i, a + j) for i in range(a) for j in range(b)], n)
    np.testing.assert_allclose(exact_sc.sc_pinv(g.row_ptr, g.col_idx, n), (a + b - 1) / (a * b), atol=1e-12)
    assert exact_sc.spanning_tree_count(graphgen.canonical_edges(g).tolist(), n) == a ** (b - 1) * b ** (a - 1)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 9])
def test_cayley_and_cycle_counts(n):
    kn = [(i, j) for i in range(n) for j in range(i + 1, n)]
    assert exact_sc.spanning_tree_count(kn, n) == n ** (n - 2)
    if n >= 3:
        assert exact_sc.spanning_tree_count([(i, (i + 1) % n) for i in range(n)], n) == n


def test_random_tree_all_ones():
    rng = np.random.default_rng(5)
    n = 40
    edges = [(i, int(rng.integers(0, i))) for i in range(1, n)]
    g = graphgen.from_edges(edges, n)
    np.testing.assert_allclose(exact_sc.sc_pinv(g.row_ptr, g.col_idx, n), 1.0, atol=1e-10)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_pinv_vs_enumeration_and_matrix_tree(seed):
    rng = np.random.default_rng(seed)
    n = 6
    while True:
        m = int(rng.integers(6, 12))
        g = graphgen.er_gnm(n, m, int(rng.integers(1 << 30)))
        g2 = graphgen.largest_component(g)
        if g2.n == n:
            break
    edges = graphgen.canonical_edges(g).tolist()
    enum, total = exact_sc.sc_enumerate(edges, n)
    mt = exact_sc.sc_matrix_tree(edges, n)
    assert enum == mt
    assert total == exact_sc.spanning_tree_count(edges, n)
    assert total == round(nx.number_of_spanning_trees(nx.Graph([tuple(e) for e in edges])))
    np.testing.assert_allclose(exact_sc.sc_pinv(g.row_ptr, g.col_idx, n), [float(x) for x in enum], atol=1e-12)


def test_foster_bridges_and_networkx():
    # two 5-cliques joined by one bridge plus a pendant path
    edges = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    edges += [(5 + i, 5 + j) for i in range(5) for j in range(i + 1, 5)]
    edges += [(4, 5), (9, 10), (10, 11)]
    n = 12
    g = graphgen.from_edges(edges, n)
    ce = graphgen.canonical_edges(g)
    sc = exact_sc.sc_pinv(g.row_ptr, g.col_idx, n)
    for (u, v), s in zip(ce.tolist(), sc):
        if (u, v) in [(4, 5), (9, 10), (10, 11)]:
            assert abs(s - 1.0) < 1e-12
        else:
            assert s < 1 - 1e-6
    assert abs(sc.sum() - (n - 1)) < 1e-9
    G = nx.Graph([tuple(e) for e in ce.tolist()])
    ref = [nx.resistance_distance(G, int(u), int(v)) for u, v in ce[:8]]
    np.testing.assert_allclose(sc[:8], ref, rtol=1e-9)


def test_foster_on_er():
    g = graphgen.largest_component(graphgen.er_gnm(400, 1600, 7))
    sc = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n)
    assert abs(sc.sum() - (g.n - 1)) < 1e-9 * g.n
    assert np.all(sc > 0) and np.all(sc <= 1 + 1e-12)


def test_truncated_resistance_limits():
    # r_tau -> r as tau grows (non-bipartite graph); r_0 = 1/d_s + 1/d_t
    g = graphgen.largest_component(graphgen.er_gnm(40, 120, 11))
    ce = graphgen.canonical_edges(g)[:10].tolist()
    d = g.degrees
    r0 = exact_sc.truncated_resistance(g.row_ptr, g.col_idx, g.n, ce, [0] * len(ce))
    np.testing.assert_allclose(r0, [1.0 / d[u] + 1.0 / d[v] for u, v in ce], rtol=1e-12)
    rbig = exact_sc.truncated_resistance(g.row_ptr, g.col_idx, g.n, ce, [400] * len(ce))
    np.testing.assert_allclose(rbig, exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n, ce), rtol=1e-8)
