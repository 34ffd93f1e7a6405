"""The walk entry point that allocates nothing (saba_walks_noalloc) against saba_walks: the
same histograms bit for bit on two calls in a row, the second smaller (on another graph), and
the limits of its fixed scratch region."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def saba():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14056_amd as saba
    saba.load()
    return saba


def _both(saba, g, W, L, seed, src_seed, **kw):
    import torch
    sg = saba.SabaGraph.from_graph(g)
    src = torch.from_numpy(graphgen.uniform_sources(g, W, src_seed)).cuda()
    ref = saba.walks(sg, src, L, seed, **kw)
    ep = torch.full((g.n,), -7, dtype=torch.int64, device="cuda")  # overwritten by the call
    vi = torch.full((g.n,), -7, dtype=torch.int64, device="cuda")
    r = saba.walks_noalloc(sg, src, L, seed, ep, vi, **kw)
    torch.cuda.synchronize()
    assert r.endpoint.data_ptr() == ep.data_ptr() and r.visits.data_ptr() == vi.data_ptr()
    return ref, r


def test_noalloc_matches_walks_twice(saba):
    import torch
    # first call: 2^22 walks of 16 steps, so the fixed region holds the visit log only in
    # chunks; second call: a smaller graph and a short ragged list (the region keeps the first
    # call's contents)
    g1 = graphgen.rmat(16, 16, 0.57, 0.19, 0.19, 3)
    print(f"noalloc call 1: rmat16 n={g1.n} W=2^22 L=16", flush=True)
    ref, r = _both(saba, g1, 1 << 22, 16, 5, 1)
    assert torch.equal(ref.endpoint, r.endpoint) and torch.equal(ref.visits, r.visits)
    assert int(r.visits.sum()) == (1 << 22) * 16
    g2 = graphgen.largest_component(graphgen.er_gnm(900, 3000, 4))
    print(f"noalloc call 2: er n={g2.n} W=3001 L=7 G=64 S=20", flush=True)
    ref, r = _both(saba, g2, 3001, 7, 9, 2, group=64, spread=20)
    assert torch.equal(ref.endpoint, r.endpoint) and torch.equal(ref.visits, r.visits)
    assert int(r.endpoint.sum()) == 3001


def test_noalloc_limits(saba):
    import torch
    g = graphgen.largest_component(graphgen.er_gnm(500, 2000, 6))
    sg = saba.SabaGraph.from_graph(g)
    ep = torch.empty(g.n, dtype=torch.int64, device="cuda")
    vi = torch.empty(g.n, dtype=torch.int64, device="cuda")
    # 2^27 walks: the walk order alone (4 bytes a walk) exceeds the 256 MiB region
    src = torch.zeros(1 << 27, dtype=torch.int32, device="cuda")
    with pytest.raises(saba.SabaError) as e:
        saba.walks_noalloc(sg, src, 4, 1, ep, vi)
    assert e.value.name == "SABA_E_INVALID"
    del src
    # other modes are refused
    src = torch.from_numpy(graphgen.uniform_sources(g, 100, 1)).cuda()
    with pytest.raises(saba.SabaError):
        saba.walks(sg, src, 4, 1, mode=saba.SABA_WALK_NAIVE, endpoint=ep, visits=vi,
                   _entry="saba_walks_noalloc")
    with pytest.raises(saba.SabaError):
        saba.walks(sg, None, 4, 1, n_walks=100, endpoint=ep, visits=vi,
                   _entry="saba_walks_noalloc")
    # the region is still usable
    r = saba.walks_noalloc(sg, src, 4, 1, ep, vi)
    ref = saba.walks(sg, src, 4, 1)
    assert torch.equal(ref.visits, r.visits) and torch.equal(ref.endpoint, r.endpoint)
