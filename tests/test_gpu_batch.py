"""Batched estimation (saba_aesc_batch over a multi-graph handle): every request's result must
be bit-identical to the same request run alone on a handle that holds only its graph, and so
agree with the oracle (Alg. 1 applied to each graph separately)."""
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


@pytest.fixture(scope="module")
def graphs():
    gs = [
        graphgen.largest_component(graphgen.er_gnm(300, 1200, 3)),
        graphgen.largest_component(graphgen.chung_lu(3000, 8, 2.3, 5)),
        graphgen.toy_graph(),
        graphgen.largest_component(graphgen.grid_diagonals(12, 15, 0.05, 2)),
        graphgen.largest_component(graphgen.er_gnm(120, 500, 6)),
    ]
    lams = [graphgen.spectral_lambda(g) for g in gs]
    return gs, lams


def _alone(saba, g, lam, eps, seed, edges=None, **kw):
    import torch
    sg = saba.SabaGraph.from_graph(g)
    if edges is None:
        sc, _ = saba.aesc(sg, eps, lam, seed, **kw)
    else:
        sc, _ = saba.aesc_query(sg, torch.from_numpy(edges).cuda(), eps, lam, seed, **kw)
    return sc.cpu().numpy()


def test_multi_graph_all_edges_equal_alone(saba, orc, graphs):
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    assert mg.info()["ngraphs"] == len(gs)
    eps = [0.3, 0.2, 0.1, 0.3, 0.15]
    reqs = [{"graph": k, "eps": eps[k], "lam": lams[k], "seed": 7, "m": gs[k].m, "tau_cap": 64}
            for k in range(len(gs))]
    outs, st = saba.aesc_batch(mg, reqs)
    assert st["sources"] == sum(g.n for g in gs)
    for k, g in enumerate(gs):
        alone = _alone(saba, g, lams[k], eps[k], 7, tau_cap=64)
        assert np.array_equal(outs[k].cpu().numpy(), alone), k
    so, _ = orc.aesc(gs[0], eps[0], lams[0], 7, tau_cap=64)
    np.testing.assert_allclose(outs[0].cpu().numpy(), so, rtol=1e-12, atol=1e-15)
    so, _ = orc.aesc(gs[3], eps[3], lams[3], 7, tau_cap=64)
    np.testing.assert_allclose(outs[3].cpu().numpy(), so, rtol=1e-12, atol=1e-15)


def test_mixed_requests_equal_alone_in_any_order(saba, graphs):
    import torch
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    rng = np.random.default_rng(4)
    reqs, expect = [], []
    for k in (0, 1, 1, 4, 0, 3):
        g = gs[k]
        ce = graphgen.canonical_edges(g)
        e = np.ascontiguousarray(ce[rng.choice(g.m, min(g.m, 17), replace=False)])
        eps = float(rng.choice([0.1, 0.2, 0.3]))
        seed = int(rng.integers(1, 4))
        reqs.append({"graph": k, "eps": eps, "lam": lams[k], "seed": seed,
                     "edges": torch.from_numpy(e).cuda(), "tau_cap": 64})
        expect.append(_alone(saba, g, lams[k], eps, seed, edges=e, tau_cap=64))
    # an all-edges request sharing parameters with a query request of the same graph
    reqs.append({"graph": 0, "eps": reqs[0]["eps"], "lam": lams[0], "seed": reqs[0]["seed"],
                 "m": gs[0].m, "tau_cap": 64})
    expect.append(_alone(saba, gs[0], lams[0], reqs[0]["eps"], reqs[0]["seed"], tau_cap=64))
    outs, _ = saba.aesc_batch(mg, reqs)
    for o, e in zip(outs, expect):
        assert np.array_equal(o.cpu().numpy(), e)
    perm = rng.permutation(len(reqs))
    outs2, _ = saba.aesc_batch(mg, [reqs[i] for i in perm], batch_sources=13)
    for j, i in enumerate(perm):
        assert np.array_equal(outs2[j].cpu().numpy(), expect[i])


def test_batch_errors(saba, graphs):
    import torch
    gs, lams = graphs
    disc = graphgen.from_edges([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)], 6)
    mg = saba.SabaGraph.from_graphs([gs[2], disc])
    with pytest.raises(saba.SabaError) as ei:
        saba.aesc_batch(mg, [{"graph": 1, "eps": 0.2, "lam": 0.5, "seed": 1, "m": disc.m}])
    assert ei.value.name == "SABA_E_DISCONNECTED"
    with pytest.raises(saba.SabaError) as ei:
        saba.aesc_batch(mg, [{"graph": 2, "eps": 0.2, "lam": 0.5, "seed": 1, "m": 1}])
    assert ei.value.name == "SABA_E_INVALID"
    with pytest.raises(saba.SabaError) as ei:
        saba.aesc_batch(mg, [{"graph": 0, "eps": 0.2, "lam": lams[2], "seed": 1,
                              "edges": torch.tensor([[0, 3]], dtype=torch.int32, device="cuda")}])
    assert ei.value.name == "SABA_E_NOT_EDGE"
    # the single-graph calls refuse a multi-graph handle
    with pytest.raises(saba.SabaError):
        saba.aesc(mg, 0.2, lams[2], 1)
    # an edge leaving its graph is rejected at upload
    with pytest.raises(saba.SabaError) as ei:
        lib = saba.load()
        import ctypes
        rp = np.array([0, 1, 2, 3], dtype=np.int32)
        ci = np.array([1, 0, 0], dtype=np.int32)  # vertex 2 (graph 1) points into graph 0
        off = np.array([0, 2, 3], dtype=np.int32)
        h = ctypes.c_void_p()
        from paper_2410_14056_amd._binding import _check
        _check(lib.saba_graph_create_multi(rp.ctypes.data_as(ctypes.c_void_p),
                                           ci.ctypes.data_as(ctypes.c_void_p), 3, 3, 2,
                                           off.ctypes.data_as(ctypes.c_void_p), 0, None,
                                           ctypes.byref(h)))
    assert ei.value.name == "SABA_E_GRAPH"
    # still usable
    outs, _ = saba.aesc_batch(mg, [{"graph": 0, "eps": 0.2, "lam": lams[2], "seed": 1, "m": 5}])
    assert outs[0].numel() == 5


def test_256_graph_batch_full_size_sampled_edges_match_oracle(saba, orc):
    """The batched benchmark's workload at full size (256 graphs, 26 million vertices, a seeded
    1% of every graph's edges as its query, tau capped at 128, the grids' lambda from the
    device) in its launch configuration: one saba_aesc_batch call with the knobs autotuned on
    every 16th request.  Requests of several graphs of each kind equal the same request run
    alone, and 8 edges of the median-size graph of each kind match the oracle (Alg. 1 on that
    graph, those edges only)."""
    import torch
    import bench
    print("256-graph batch at full size: building the graphs", flush=True)
    graphs, lams0, epss, qnp = bench.batch_workload(256, 0.01)
    mg = saba.SabaGraph.from_graphs(graphs, trusted=True)
    print("256-graph batch: lambda of the grids on the device", flush=True)
    lams = bench.device_lambdas(saba, mg, lams0)
    assert all(0.0 < l < 1.0 for l in lams)
    reqs = [{"graph": k, "eps": epss[k], "lam": lams[k], "seed": 1,
             "edges": torch.from_numpy(qnp[k]).cuda(), "tau_cap": 128} for k in range(len(graphs))]
    print("256-graph batch: autotuning on the benchmark's sample", flush=True)
    saba.autotune_aesc(mg, bench.tuning_sample(reqs))
    print(f"256-graph batch: one batched call over {sum(len(q) for q in qnp)} query edges",
          flush=True)
    outs, _ = saba.aesc_batch(mg, reqs)
    print("256-graph batch: requests alone", flush=True)
    for k in (0, 1, 2, 127, 128, 129, 253, 254, 255):
        alone = _alone(saba, graphs[k], lams[k], epss[k], 1, edges=qnp[k], tau_cap=128)
        assert np.array_equal(outs[k].cpu().numpy(), alone), k
    for kind in range(3):
        ks = [k for k in range(len(graphs)) if k % 3 == kind]
        k = sorted(ks, key=lambda j: graphs[j].n)[len(ks) // 2]
        sel = np.linspace(0, len(qnp[k]) - 1, 8).astype(int)
        print(f"256-graph batch, oracle check: graph {k} kind {kind} n={graphs[k].n} eps={epss[k]}", flush=True)
        so, _ = orc.aesc(graphs[k], epss[k], lams[k], 1, query=qnp[k][sel], tau_cap=128)
        np.testing.assert_allclose(outs[k].cpu().numpy()[sel], so, rtol=1e-12, atol=1e-15)


def test_small_grid_certified_only_with_enough_tau(saba):
    """A small graph of the batched workload's grid generator (5 x 5 grid with 5% random
    diagonals, not bipartite): at tau <= 128 the truncation bound exceeds eps / 2, so the
    benchmark reports such requests as uncertified; with the cap raised above the largest
    CalculateTau the estimates meet eps against exact SC."""
    import bench
    from oracle import exact_sc
    g = graphgen.largest_component(graphgen.grid_diagonals(5, 5, 0.05, 1))
    assert not graphgen.is_bipartite(g)
    lam = graphgen.spectral_lambda(g)
    ce = graphgen.canonical_edges(g)
    eps = 0.3
    bound, ok = bench.truncation_bound(g, ce, lam, eps, 128)
    assert not ok and bound > eps / 2
    bound, ok = bench.truncation_bound(g, ce, lam, eps, 1 << 20)
    assert ok and bound <= eps / 2
    sg = saba.SabaGraph.from_graph(g)
    sc, st = saba.aesc(sg, eps, lam, 3, tau_cap=1 << 20)
    assert not (st["warnings"] & 1)
    ex = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n)
    err = np.abs(sc.cpu().numpy() - ex)
    print(f"grid 5x5: lambda {lam:.5f} max tau {st['max_tau']} max error {err.max():.4f}", flush=True)
    assert err.max() <= eps
