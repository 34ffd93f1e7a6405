"""The seeded input generators that both sides use: deterministic per seed, canonical CSR
(sorted, symmetric, no self-loops or duplicates), and the sizes and degree structure they are
meant to have."""
import numpy as np
import pytest
from scipy import stats

import graphgen


def _canonical(g):
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == ci.size and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(ci != rows), "self-loop"
    for v in range(0, g.n, max(1, g.n // 200)):  # sampled rows: strictly increasing
        r = ci[rp[v]:rp[v + 1]]
        assert np.all(np.diff(r) > 0)
    # symmetric: the multiset of (u, v) equals that of (v, u)
    a = rows.astype(np.int64) * g.n + ci
    b = ci.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(a), np.sort(b))


GENS = {
    "er": lambda s: graphgen.er_gnm(3000, 12000, s),
    "rmat": lambda s: graphgen.rmat(12, 16, 0.57, 0.19, 0.19, s),
    "chung_lu": lambda s: graphgen.chung_lu(5000, 10, 2.5, s),
    "grid": lambda s: graphgen.grid_diagonals(40, 50, 0.05, s),
}


def test_circulant_is_canonical_and_regular():
    g = graphgen.circulant(1000, (1, 7, 100))
    _canonical(g)
    assert g.n == 1000 and g.m == 3000 and np.all(np.diff(g.row_ptr) == 6)
    # vertex 0 is joined to 1, 7, 100 and their negatives mod n
    assert list(g.col_idx[:6]) == [1, 7, 100, 900, 993, 999]
    # the direct build equals canonicalising the same edge list
    u = np.repeat(np.arange(1000), 3)
    v = (u + np.tile([1, 7, 100], 1000)) % 1000
    h = graphgen.canonical_csr(u, v, 1000)
    assert np.array_equal(g.row_ptr, h.row_ptr) and np.array_equal(g.col_idx, h.col_idx)
    with pytest.raises(ValueError):
        graphgen.circulant(10, (5,))


@pytest.mark.parametrize("name", list(GENS))
def test_deterministic_and_canonical(name):
    g1, g2, g3 = GENS[name](1), GENS[name](1), GENS[name](2)
    assert np.array_equal(g1.row_ptr, g2.row_ptr) and np.array_equal(g1.col_idx, g2.col_idx)
    assert not (g1.col_idx.size == g3.col_idx.size and np.array_equal(g1.col_idx, g3.col_idx))
    _canonical(g1)
    lc = graphgen.largest_component(g1)
    _canonical(lc)
    assert lc.n <= g1.n and lc.m <= g1.m


def test_sizes_and_degrees():
    er = graphgen.er_gnm(3000, 12000, 4)
    assert er.m == 12000 and er.n == 3000  # exactly m distinct edges
    rm = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 1)
    deg = np.diff(rm.row_ptr)
    assert rm.n == 4096 and rm.m <= 16 * 4096
    assert (deg == 0).sum() > 0  # R-MAT leaves isolated vertices
    top = np.sort(deg)[::-1][:41].sum() / deg.sum()
    assert top > 0.15  # heavy tail: the top 1% of vertices hold a large share of the entries
    gr = graphgen.grid_diagonals(40, 50, 0.05, 3)
    lattice = 40 * 49 + 50 * 39
    ndiag = gr.m - lattice
    assert 0 < ndiag < 0.1 * 39 * 49 and abs(ndiag - 0.05 * 39 * 49) < 4 * np.sqrt(0.05 * 39 * 49)


def test_chung_lu_follows_its_weights():
    g = graphgen.chung_lu(20000, 10, 2.5, 1)
    deg = np.diff(g.row_ptr).astype(float)
    w = np.power(np.arange(1, g.n + 1, dtype=float), -1.0 / 1.5)
    # vertex i receives 2M w_i / sum(w) endpoints on average (M = n k / 2 sampled pairs);
    # binned so that the Poisson noise averages out.  Duplicates only thin the hubs.
    expect = 2 * (20000 * 10 / 2) * w / w.sum()
    for lo, hi in ((100, 1000), (1000, 5000), (5000, 20000)):
        assert abs(deg[lo:hi].sum() / expect[lo:hi].sum() - 1) < 0.02, (lo, hi)
    assert 0.75 < deg[:10].sum() / expect[:10].sum() < 1.0
    assert stats.spearmanr(deg[:2000], w[:2000]).statistic > 0.9
    # mean degree near the target; self-loops and duplicates remove a little
    assert 9.5 < deg.mean() <= 10.0


def test_chung_lu_1e6_graph_figures():
    """The 10^6-vertex Chung-Lu graph of the estimator benchmark (seed 1): its largest
    component has the vertex and edge counts stated with the workload."""
    g = graphgen.largest_component(graphgen.chung_lu(1000000, 10, 2.5, 1))
    assert (g.n, g.m) == (990378, 4984862)


def test_uniform_sources_skip_isolated_vertices():
    g = graphgen.rmat(10, 4, 0.57, 0.19, 0.19, 3)
    s1 = graphgen.uniform_sources(g, 5000, 9)
    assert np.array_equal(s1, graphgen.uniform_sources(g, 5000, 9))
    assert np.all(np.diff(g.row_ptr)[s1] > 0)
