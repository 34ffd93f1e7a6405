"""Pins for the oracle's hashed uniform start vertices (the uniform random sources of the
synthetic walk benchmark, Sec. 5.4): they come from the non-isolated vertices only, uniformly,
depend on nothing but that set, the seed and the walk number, and the empty case is an error."""
import numpy as np
import pytest
from scipy import stats

import graphgen


def test_sources_are_uniform_over_the_non_isolated_vertices(orc):
    g = graphgen.rmat(10, 4, 0.57, 0.19, 0.19, 3)  # R-MAT leaves isolated vertices
    deg = np.diff(g.row_ptr)
    pool = np.flatnonzero(deg > 0)
    assert pool.size < g.n
    W = 400 * pool.size
    src = orc.uniform_sources(g, W, 7)
    assert np.all(deg[src] > 0)
    counts = np.bincount(src, minlength=g.n)[pool]
    assert counts.min() > 0
    assert stats.chisquare(counts).pvalue > 1e-5


def test_sources_depend_only_on_the_pool_seed_and_walk_number(orc):
    a = graphgen.from_edges([(0, 2), (2, 5), (5, 7)], 9)   # pool {0, 2, 5, 7}
    b = graphgen.from_edges([(0, 7), (2, 5), (0, 5)], 9)   # same pool, other edges
    sa, sb = orc.uniform_sources(a, 5000, 3), orc.uniform_sources(b, 5000, 3)
    assert np.array_equal(sa, sb)
    assert set(np.unique(sa)) == {0, 2, 5, 7}
    # walk j's draw does not depend on how many walks are drawn
    assert np.array_equal(orc.uniform_sources(a, 1234, 3), sa[:1234])
    assert not np.array_equal(orc.uniform_sources(a, 5000, 4), sa)


def test_two_vertex_pool_splits_evenly(orc):
    g = graphgen.from_edges([(3, 4)], 6)
    src = orc.uniform_sources(g, 20000, 11)
    assert set(np.unique(src)) == {3, 4}
    assert stats.binomtest(int((src == 3).sum()), src.size, 0.5).pvalue > 1e-5


def test_empty_pool(orc):
    g = graphgen.from_edges([], 4)
    assert orc.uniform_sources(g, 0, 1).size == 0
    with pytest.raises(ValueError):
        orc.uniform_sources(g, 5, 1)
