"""Pins for the oracle's ablation samplers (the neighbour-choice functions of Eq. (3), (4) and
Eq. (5) read literally) and its branching statistics (the Table 5 experiment)."""
import numpy as np
import pytest
from scipy import stats

import graphgen

KEYED, KEYED_MOD, STREAM_MOD, LITERAL = 0, 1, 2, 3


def _P(g):
    A = g.dense_adjacency()
    return A / A.sum(axis=1, keepdims=True)


def _chi2_p(counts, probs):
    W = counts.sum()
    if np.any(counts[probs == 0] > 0):
        return 0.0
    exp = W * probs
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    return stats.chi2.sf(((obs - ex) ** 2 / ex).sum(), len(obs) - 1)


def _cycle(n):
    return graphgen.from_edges([(i, (i + 1) % n) for i in range(n)], n)


def _circulant(n, offsets):
    return graphgen.from_edges([(i, (i + o) % n) for i in range(n) for o in offsets], n)


def test_xorshift32_published_value(orc):
    # Marsaglia (2003), "Xorshift RNGs": shifts (13, 17, 5) from y = 2463534242 give 723471715
    assert orc.xorshift32(2463534242) == 723471715
    # a bijection of the nonzero states: zero is a fixed point, nothing else maps to zero
    assert orc.xorshift32(0) == 0
    xs = np.random.default_rng(1).integers(1, 2**32, 2000, dtype=np.uint64)
    assert all(orc.xorshift32(int(x)) != 0 for x in xs)


@pytest.mark.parametrize("sampler", [KEYED_MOD, STREAM_MOD])
@pytest.mark.parametrize("L", [1, 3])
def test_modulo_samplers_sample_the_walk(orc, sampler, L):
    """Eq. (3) and Eq. (4) are proper random walks (the modulo bias is below 2^-20 for these
    degrees): endpoint frequencies follow the row of P^L, not of P^(L+1)."""
    g = graphgen.largest_component(graphgen.er_gnm(24, 50, 8))
    P = _P(g)
    W = 60000
    ep, vi = orc.walks_histogram(g, np.zeros(W, dtype=np.int32), L, seed=5, sampler=sampler)
    assert ep.sum() == W and vi.sum() == W * L
    assert _chi2_p(ep, np.linalg.matrix_power(P, L)[0]) > 1e-5
    assert _chi2_p(ep, np.linalg.matrix_power(P, L + 1)[0]) < 1e-12


def test_grouped_modulo_lanes_are_marginally_exact(orc):
    """With G > 1 each lane is still an exact walk under Eq. (4): lane r of every group."""
    g = graphgen.largest_component(graphgen.er_gnm(24, 50, 8))
    P = _P(g)
    L, G = 3, 64
    W = 64 * 1500
    ep, _ = orc.walks_histogram(g, np.zeros(W, dtype=np.int32), L, seed=9, G=G, S=20,
                                sampler=KEYED_MOD)
    assert _chi2_p(ep, np.linalg.matrix_power(P, L)[0]) > 1e-5


def test_literal_schedule_is_decided_by_the_seed_top_bits(orc):
    """Eq. (5) read literally: on a cycle every step takes floor(2 u / 2^32), the top bit of
    X_W XOR a fixed hash, so all walks from one source follow one of two paths; on a
    16-regular graph at most 16 paths.  The keyed schedule gives thousands."""
    W, L = 4096, 12
    src = np.zeros(W, dtype=np.int32)
    for g, cap in ((_cycle(50), 2), (_circulant(64, (1, 2, 3, 5, 7, 11, 13, 17)), 16)):
        reachable = int((np.linalg.matrix_power(_P(g), L)[0] > 0).sum())
        assert reachable > cap
        for sampler in (LITERAL, KEYED):
            # distinct end points bound the distinct paths from below, and a vector of 8
            # walks can never hold more distinct vertices than there are paths
            ends = int((orc.walks_histogram(g, src, L, 3, sampler=sampler)[0] > 0).sum())
            h = orc.distinct8(g, src, L, 3, sampler=sampler, order=0)
            if sampler == LITERAL:
                assert ends <= cap
                assert h[cap + 1:].sum() == 0
            else:  # the keyed schedule reaches (nearly) every reachable vertex
                assert ends >= 0.9 * reachable
                assert h[min(cap, 8) :].sum() > 0


def test_distinct8_brute_force(orc):
    """The branching statistics against a direct count from the walks' own paths."""
    g = graphgen.largest_component(graphgen.rmat(7, 4, 0.57, 0.19, 0.19, 2))
    rng = np.random.default_rng(4)
    pool = np.flatnonzero(np.diff(g.row_ptr) > 0)
    src = rng.choice(pool, 203).astype(np.int32)  # 25 full vectors and a partial one
    L, seed, G, S = 6, 7, 8, 24
    rank = np.zeros(len(src), dtype=np.int64)
    seen = {}
    for j, s in enumerate(src):
        rank[j] = seen.get(int(s), 0)
        seen[int(s)] = rank[j] + 1
    paths = []
    for j, s in enumerate(src):
        khi, klo = orc.walk_key(seed, int(s), 0, 0, int(rank[j]), G, S)
        paths.append(orc.walk_path(g, int(s), L, khi, klo))
    paths = np.array(paths)
    for order in (0, 1):
        idx = np.arange(len(src)) if order == 0 else np.lexsort((rank, src))
        want = np.zeros(9, dtype=np.int64)
        for v in range(0, len(src) - 7, 8):
            for l in range(1, L + 1):
                want[len(set(paths[idx[v:v + 8], l].tolist()))] += 1
        got = orc.distinct8(g, src, L, seed, G=G, S=S, order=order)
        assert np.array_equal(got, want), order
        assert got.sum() == (len(src) // 8) * L


def test_distinct8_special_cases(orc):
    # every walk from a degree-1 vertex takes the same first step
    g = graphgen.from_edges([(0, 1), (1, 2), (2, 3), (1, 3), (3, 4)], 5)
    h = orc.distinct8(g, np.zeros(64, dtype=np.int32), 1, 1, order=1)
    assert h[1] == 8 and h.sum() == 8
    # walks of L = 0 have no positions to count
    assert orc.distinct8(g, np.zeros(64, dtype=np.int32), 0, 1).sum() == 0


@pytest.mark.parametrize("beta", [4, 16, 100])
def test_distinct_count_follows_the_expected_distinct_items(orc, beta):
    """Sec. 5.5 (limitations): alpha independent choices among beta neighbours hold
    beta (1 - (1 - 1/beta)^alpha) distinct vertices on average.  The branching counter at the
    first step of independent walks (alpha = 8, one vector per 8 walks of a star's centre)
    follows it within a CLT bound; grouped walks (G = 64) fall far below it."""
    g = graphgen.from_edges([(0, i) for i in range(1, beta + 1)], beta + 1)
    W = 8 * 20000
    src = np.zeros(W, dtype=np.int32)
    h = orc.distinct8(g, src, 1, 13, order=1)
    k = np.arange(9)
    n = h.sum()
    mean = (h * k).sum() / n
    sd = np.sqrt((h * (k - mean) ** 2).sum() / n)
    expect = beta * (1 - (1 - 1 / beta) ** 8)
    assert abs(mean - expect) < 5 * sd / np.sqrt(n), (mean, expect)
    hg = orc.distinct8(g, src, 1, 13, G=64, S=20, order=1)
    assert (hg * k).sum() / hg.sum() < 0.5 * expect + 0.5
