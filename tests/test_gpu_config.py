"""Execution knobs and the walk autotuner: every setting gives bit-identical walks and
estimates (they only change how the work is spread over the GPU)."""
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


def test_walk_knobs_do_not_change_results(saba, orc):
    import torch
    g = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 2)
    sg = saba.SabaGraph.from_graph(g)
    src = graphgen.uniform_sources(g, 200001, 3)  # several tiles per block, ragged
    t = torch.from_numpy(src).cuda()
    ep_o, vi_o = orc.walks_histogram(g, src, 13, 9, G=8, S=24)
    for wpl in (1, 2, 4):
        for blocks in (7, 64, 1024, 4096):
            saba.set_config(sg, walks_per_lane=wpl, walk_blocks=blocks)
            r = saba.walks(sg, t, 13, 9, group=8, spread=24)
            assert np.array_equal(r.endpoint.cpu().numpy(), ep_o), (wpl, blocks)
            assert np.array_equal(r.visits.cpu().numpy(), vi_o), (wpl, blocks)
    # visit-log chunks counted on the second stream while the next chunk walks (ragged last
    # chunk; 2 chunks, an odd count, and more chunks than the double buffer)
    for ch in (2, 3, 7, 64):
        for wpl, blocks in ((2, 1024), (1, 64)):
            saba.set_config(sg, walks_per_lane=wpl, walk_blocks=blocks, walk_chunks=ch)
            r = saba.walks(sg, t, 13, 9, group=8, spread=24, time_kernels=True)
            assert np.array_equal(r.endpoint.cpu().numpy(), ep_o), (ch, wpl, blocks)
            assert np.array_equal(r.visits.cpu().numpy(), vi_o), (ch, wpl, blocks)
            assert r.stats["kernel_ms"] > 0 and r.stats["count_ms"] > 0
    best = saba.autotune_walks(sg, t, 13, 9)
    assert best["walks_per_lane"] in (1, 2, 4) and best["walk_blocks"] in (1024, 2048, 4096, 8192)
    assert best["walk_chunks"] in (1, 4, 8)
    assert saba.get_config(sg) == best
    r = saba.walks(sg, t, 13, 9, group=8, spread=24)
    assert np.array_equal(r.visits.cpu().numpy(), vi_o)


def test_estimator_knobs_do_not_change_results(saba):
    import torch
    g = graphgen.largest_component(graphgen.chung_lu(3000, 8, 2.3, 5))
    lam = graphgen.spectral_lambda(g)
    sg = saba.SabaGraph.from_graph(g)
    ref, _ = saba.aesc(sg, 0.2, lam, 4, tau_cap=64)
    for wq in (0, 1, 2):  # stride, queues, staged tiles (support bitmaps in LDS)
        for wb, pb in ((1, 1), (3, 17), (512, 4096), (8192, 64)):
            saba.set_config(sg, est_walk_blocks=wb, est_push_blocks=pb, est_walk_queue=wq)
            sc, _ = saba.aesc(sg, 0.2, lam, 4, tau_cap=64)
            assert torch.equal(sc, ref), (wq, wb, pb)
            # the queue counters are cleared per launch: a second call gives the same
            sc, _ = saba.aesc(sg, 0.2, lam, 4, tau_cap=64, batch_sources=333)
            assert torch.equal(sc, ref), (wq, wb, pb, "batched")


def test_batch_streams_do_not_change_results(saba):
    """Two pool sets with the levels of the next batch on a second stream give the results
    and the per-call totals of the batches run in order: even and odd batch counts, one
    batch (nothing to overlap), a query, a source range, and the walk-pair timing."""
    import torch
    g = graphgen.largest_component(graphgen.chung_lu(3000, 8, 2.3, 5))
    lam = graphgen.spectral_lambda(g)
    sg = saba.SabaGraph.from_graph(g)
    keys = ("walks", "walk_steps", "push_edge_visits", "sources", "batches", "max_tau",
            "max_ttau", "warnings")
    ce = graphgen.canonical_edges(g)
    pick = np.random.default_rng(8).choice(g.m, 300, replace=False)
    q = torch.from_numpy(np.ascontiguousarray(ce[pick])).cuda()
    for bsrc, wq in ((0, 1), (250, 2), (333, 1), (1500, 2)):
        outs = {}
        for streams in (1, 2, 0):
            saba.set_config(sg, est_walk_queue=wq, est_batch_streams=streams)
            sc, st = saba.aesc(sg, 0.2, lam, 4, tau_cap=64, batch_sources=bsrc,
                               time_kernels=True)
            qs, qst = saba.aesc_query(sg, q, 0.2, lam, 4, tau_cap=64, batch_sources=bsrc)
            gs = torch.zeros(sg.nnz, dtype=torch.float64, device="cuda")
            saba.aesc_sources(sg, gs, 100, 2100, 0.2, lam, 4, tau_cap=64, batch_sources=bsrc)
            assert st["kernel_ms"] > 0 and st["total_ms"] >= st["kernel_ms"]
            outs[streams] = (sc, {k: st[k] for k in keys}, qs, {k: qst[k] for k in keys}, gs)
        for streams in (2, 0):
            a, b = outs[1], outs[streams]  # 0: the default, in order
            assert torch.equal(a[0], b[0]), (bsrc, streams)
            assert a[1] == b[1], (bsrc, streams)
            assert torch.equal(a[2], b[2]) and a[3] == b[3], (bsrc, streams, "query")
            assert torch.equal(a[4], b[4]), (bsrc, streams, "sources")
    saba.set_config(sg)


def test_staged_schedule_falls_back_beyond_the_lds(saba):
    """A graph of 1.39e6 vertices, whose support bitmap (174 KB) exceeds a block's LDS: the
    staged schedule falls back to the work queues and gives the results of the other
    schedules, bit for bit."""
    import torch
    g = graphgen.largest_component(graphgen.er_gnm(1400000, 3500000, 3))
    assert (g.n + 31) // 32 * 4 > 160 * 1024
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    ce = graphgen.canonical_edges(g)
    pick = np.random.default_rng(4).choice(g.m, 64, replace=False)
    q = torch.from_numpy(np.ascontiguousarray(ce[pick])).cuda()
    outs = []
    for wq in (0, 1, 2):
        saba.set_config(sg, est_walk_queue=wq)
        sc, st = saba.aesc_query(sg, q, 0.3, 0.0, 2, tau_cap=24)
        outs.append((sc, st["walk_steps"]))
    for sc, steps in outs[1:]:
        assert torch.equal(sc, outs[0][0]) and steps == outs[0][1]


def test_estimator_autotuner(saba):
    """saba_autotune_aesc picks a candidate grid, keeps it in the handle, and the sample's
    outputs and later results equal the untuned ones."""
    import torch
    gs = [graphgen.largest_component(graphgen.er_gnm(800, 3200, 2)),
          graphgen.largest_component(graphgen.chung_lu(2000, 8, 2.3, 3))]
    mg = saba.SabaGraph.from_graphs(gs)
    lams = [graphgen.spectral_lambda(g) for g in gs]
    reqs = [dict(graph=k, eps=0.25, lam=lams[k], seed=5, m=g.m) for k, g in enumerate(gs)]
    ref, _ = saba.aesc_batch(mg, reqs)
    best = saba.autotune_aesc(mg, reqs)
    assert best["est_walk_blocks"] in (512, 1024, 2048, 4096)
    assert best["est_push_blocks"] in (1024, 2048, 4096, 8192)
    assert best["est_walk_queue"] in (0, 1, 2)
    assert best["est_batch_streams"] in (1, 2)
    assert saba.get_config(mg) == best
    out, _ = saba.aesc_batch(mg, reqs)
    for a, b in zip(out, ref):
        assert torch.equal(a, b)
    with pytest.raises(saba.SabaError) as ei:
        saba.autotune_aesc(mg, [])
    assert ei.value.name == "SABA_E_INVALID"


def test_results_do_not_depend_on_the_stream(saba):
    """Walks and estimates issued on a side stream (default priority) equal those on the
    current stream, bit for bit."""
    import torch
    g = graphgen.largest_component(graphgen.chung_lu(3000, 8, 2.3, 7))
    lam = graphgen.spectral_lambda(g)
    sg = saba.SabaGraph.from_graph(g)
    src = torch.from_numpy(graphgen.uniform_sources(g, 50000, 2)).cuda()
    r0 = saba.walks(sg, src, 11, 3)
    a0, _ = saba.aesc(sg, 0.25, lam, 3)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r1 = saba.walks(sg, src, 11, 3, stream=side)
        a1, _ = saba.aesc(sg, 0.25, lam, 3, stream=side)
    side.synchronize()
    assert torch.equal(r0.endpoint, r1.endpoint) and torch.equal(r0.visits, r1.visits)
    assert torch.equal(a0, a1)


def test_config_rejects_bad_values(saba):
    sg = saba.SabaGraph.from_graph(graphgen.toy_graph())
    for kw in ({"walks_per_lane": 3}, {"walk_blocks": -1}, {"est_push_blocks": 1 << 20},
               {"walk_chunks": 65}, {"walk_chunks": -1}, {"est_walk_queue": 3},
               {"est_batch_streams": 3}, {"est_batch_streams": -1}):
        with pytest.raises(saba.SabaError) as ei:
            saba.set_config(sg, **kw)
        assert ei.value.name == "SABA_E_INVALID"


def test_bouquet_autotuner_respects_the_budget(saba):
    """saba_autotune_bouquet returns the fastest (G, S) whose 8-walk vectors keep at least the
    budget of distinct vertices on the sample; the returned mean is the branching statistic of
    the same walks, and the schedule is not kept in the handle."""
    import torch
    g = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 2)
    sg = saba.SabaGraph.from_graph(g)
    src = torch.from_numpy(np.repeat(graphgen.uniform_sources(g, 512, 3), 256).astype(np.int32)).cuda()
    before = saba.get_config(sg)
    picks = {}
    for budget in (7.5, 4.0, 1.0):
        b = saba.autotune_bouquet(sg, src, 12, 5, budget)
        assert b["distinct_mean"] >= budget and b["ms"] > 0
        r = saba.walks(sg, src, 12, 5, group=b["group"], spread=b["spread"], distinct=True)
        h = r.distinct.cpu().numpy()
        assert abs((h * np.arange(9)).sum() / h.sum() - b["distinct_mean"]) < 1e-12
        picks[budget] = b
    assert saba.get_config(sg) == before
    # a looser budget admits every schedule a tighter one does
    assert picks[1.0]["distinct_mean"] <= 8.0
    with pytest.raises(saba.SabaError):
        saba.autotune_bouquet(sg, src, 12, 5, 9.0)
