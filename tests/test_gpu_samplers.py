"""GPU parity of the ablation samplers (Eq. (3), Eq. (4), Eq. (5) read literally, and the keyed
Eq. (5)) and of the branching statistics (the Table 5 experiment): histograms and distinct-vertex
counts must equal the oracle's bit for bit, in both execution modes."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

SAMPLERS = [0, 1, 2, 3]  # keyed, keyed modulo, per-walk stream modulo, literal


@pytest.fixture(scope="module")
def saba():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14056_amd as saba
    saba.load()
    return saba


GRAPHS = {
    "er": lambda: graphgen.largest_component(graphgen.er_gnm(500, 2000, 3)),
    "rmat12": lambda: graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 2),
}


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("sampler", SAMPLERS)
@pytest.mark.parametrize("G,S", [(1, 0), (64, 20)])
def test_sampler_histograms_and_branching_match_oracle(saba, orc, gname, sampler, G, S):
    import torch
    g = GRAPHS[gname]()
    L, seed = 9, 31
    print(f"sampler parity graph={gname} sampler={sampler} G={G} S={S}", flush=True)
    sg = saba.SabaGraph.from_graph(g)
    src = graphgen.uniform_sources(g, 12345, 7)  # ragged: a partial last vector of 8
    # walks of few sources, so that bouquet vectors hold walks of one start vertex
    few = np.repeat(src[:40], 97)[:3001]
    ep_o, vi_o = orc.walks_histogram(g, src, L, seed, G=G, S=S, sampler=sampler)
    d_naive = orc.distinct8(g, src, L, seed, G=G, S=S, sampler=sampler, order=0)
    d_bq = orc.distinct8(g, few, L, seed, G=G, S=S, sampler=sampler, order=1)
    t = torch.from_numpy(np.ascontiguousarray(src, dtype=np.int32)).cuda()
    tf = torch.from_numpy(np.ascontiguousarray(few, dtype=np.int32)).cuda()
    for mode in (saba.SABA_WALK_NAIVE, saba.SABA_WALK_BOUQUET, saba.SABA_WALK_NAIVE_LOG):
        for distinct in (False, True):
            r = saba.walks(sg, t, L, seed, group=G, spread=S, mode=mode, sampler=sampler,
                           distinct=distinct)
            assert np.array_equal(r.endpoint.cpu().numpy(), ep_o), (mode, distinct)
            assert np.array_equal(r.visits.cpu().numpy(), vi_o), (mode, distinct)
            if distinct and mode != saba.SABA_WALK_BOUQUET:  # both naive orders: list order
                assert np.array_equal(r.distinct.cpu().numpy(), d_naive)
    r = saba.walks(sg, tf, L, seed, group=G, spread=S, mode=saba.SABA_WALK_BOUQUET,
                   sampler=sampler, distinct=True)
    assert np.array_equal(r.distinct.cpu().numpy(), d_bq)
    assert r.distinct.sum().item() == (len(few) // 8) * L


def test_branching_reproduces_the_table5_ordering(saba, orc):
    """Grouped keys with the scaled choice (SABA) keep the 8 walks of a vector together far
    more than independent keys or the modulo choice do; the oracle agrees on every count."""
    import torch
    g = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 2)
    sg = saba.SabaGraph.from_graph(g)
    src = np.repeat(graphgen.uniform_sources(g, 64, 3), 256).astype(np.int32)
    t = torch.from_numpy(src).cuda()
    mean = {}
    for name, sampler, G, S in (("saba", 0, 64, 20), ("hash", 1, 1, 0), ("hash_grouped", 1, 64, 20),
                                ("stream", 2, 1, 0)):
        r = saba.walks(sg, t, 10, 5, group=G, spread=S, sampler=sampler, distinct=True)
        h = r.distinct.cpu().numpy()
        assert np.array_equal(h, orc.distinct8(g, src, 10, 5, G=G, S=S, sampler=sampler))
        mean[name] = (h * np.arange(9)).sum() / h.sum()
    assert mean["saba"] < 0.6 * min(mean["hash"], mean["hash_grouped"], mean["stream"])


def test_sampler_argument_checked(saba):
    import torch
    g = graphgen.toy_graph()
    sg = saba.SabaGraph.from_graph(g)
    with pytest.raises(saba.SabaError) as ei:
        saba.walks(sg, torch.zeros(4, dtype=torch.int32, device="cuda"), 3, 1, sampler=4)
    assert ei.value.name == "SABA_E_INVALID"
