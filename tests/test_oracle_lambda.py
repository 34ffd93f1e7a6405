"""Pins for the oracle's spectral input lambda = max(|lambda_2|, |lambda_n|) of D^-1/2 A D^-1/2
(CalculateTau in Alg. 1) against spectra known in closed form."""
import math

import numpy as np

import graphgen
from oracle import exact_sc


def _lam(g):
    return exact_sc.spectral_lambda(g.row_ptr, g.col_idx, g.n)


def test_complete_graph():
    # N = (J - I) / (n - 1): eigenvalues 1 and -1/(n-1)
    for n in (3, 5, 9):
        g = graphgen.from_edges([(i, j) for i in range(n) for j in range(i + 1, n)], n)
        lam, ev = _lam(g)
        assert abs(lam - 1.0 / (n - 1)) < 1e-13
        assert abs(ev[-1] - 1.0) < 1e-13


def test_odd_cycle():
    # N = A / 2 with eigenvalues cos(2 pi k / n); for odd n the extreme is cos(pi / n)
    for n in (5, 9, 21):
        g = graphgen.from_edges([(i, (i + 1) % n) for i in range(n)], n)
        assert abs(_lam(g)[0] - math.cos(math.pi / n)) < 1e-13


def test_petersen():
    # adjacency eigenvalues 3, 1, -2 -> N = A / 3: 1, 1/3, -2/3
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    g = graphgen.from_edges(outer + spokes + inner, 10)
    lam, ev = _lam(g)
    assert abs(lam - 2.0 / 3.0) < 1e-13
    assert np.allclose(sorted(set(np.round(ev, 9))), [-2 / 3, 1 / 3, 1.0])


def test_bipartite_reaches_one():
    # K_{2,3}: lambda_n = -1
    g = graphgen.from_edges([(a, b) for a in range(2) for b in range(2, 5)], 5)
    lam, ev = _lam(g)
    assert abs(lam - 1.0) < 1e-13 and abs(ev[0] + 1.0) < 1e-13
