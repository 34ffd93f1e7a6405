"""Pins for the eigenvector tail correction (the omega > 0 reading of CalculateTau, Alg. 1):
with every nontrivial eigenpair, the truncated series plus the correction is the exact
resistance for any truncation; with some of them, the rest obeys the tail bound of the
remaining spectrum."""
import numpy as np
import pytest

import graphgen
from oracle import exact_sc


def _graph():
    return graphgen.largest_component(graphgen.er_gnm(40, 110, 6))


def _edges(g):
    return [tuple(e) for e in graphgen.canonical_edges(g)]


def test_full_spectrum_closes_the_series():
    g = _graph()
    edges = _edges(g)
    exact = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n, edges)
    vals, vecs, rest = exact_sc.top_eigenpairs(g.row_ptr, g.col_idx, g.n, g.n - 1)
    assert rest == 0.0
    for tau in (0, 1, 4):
        taus = [tau] * len(edges)
        r_tau = exact_sc.truncated_resistance(g.row_ptr, g.col_idx, g.n, edges, taus)
        corr = exact_sc.eigen_tail_correction(g.row_ptr, g.col_idx, g.n, edges, taus, vals, vecs)
        np.testing.assert_allclose(r_tau + corr, exact, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("omega", [1, 3, 8])
def test_partial_spectrum_leaves_the_bounded_rest(omega):
    g = _graph()
    edges = _edges(g)
    d = np.diff(g.row_ptr)
    exact = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n, edges)
    vals, vecs, rest = exact_sc.top_eigenpairs(g.row_ptr, g.col_idx, g.n, omega)
    lam = exact_sc.spectral_lambda(g.row_ptr, g.col_idx, g.n)[0]
    assert rest <= lam + 1e-15 and len(vals) == omega
    for tau in (0, 2, 5):
        taus = [tau] * len(edges)
        r_tau = exact_sc.truncated_resistance(g.row_ptr, g.col_idx, g.n, edges, taus)
        corr = exact_sc.eigen_tail_correction(g.row_ptr, g.col_idx, g.n, edges, taus, vals, vecs)
        for i, (a, b) in enumerate(edges):
            bound = rest ** (tau + 1) * (1 / d[a] + 1 / d[b]) / (1 - rest)
            assert abs(exact[i] - r_tau[i] - corr[i]) <= bound + 1e-12
            # and it is tighter than the plain bound with lambda whenever rest < lambda
            assert abs(exact[i] - r_tau[i] - corr[i]) <= \
                lam ** (tau + 1) * (1 / d[a] + 1 / d[b]) / (1 - lam) + 1e-12


def test_top_eigenpairs_order_and_orthonormality():
    g = _graph()
    vals, vecs, rest = exact_sc.top_eigenpairs(g.row_ptr, g.col_idx, g.n, 5)
    assert np.all(np.diff(np.abs(vals)) <= 1e-15) and abs(vals[0]) <= 1.0 - 1e-9
    np.testing.assert_allclose(vecs.T @ vecs, np.eye(5), atol=1e-12)
    # orthogonal to the trivial eigenvector sqrt(d)
    sd = np.sqrt(np.diff(g.row_ptr).astype(float))
    assert np.max(np.abs(vecs.T @ sd)) < 1e-10
    assert rest <= abs(vals[-1]) + 1e-15
