"""Query server (saba_server_*): continuous batching must not change any result.  Every served
request is compared bit for bit with the same request run alone through saba_aesc_query on a
handle holding only its graph, under batch sizes and lane counts that force its sources to be
split across batches and streams, and with requests arriving while others run."""
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
        graphgen.largest_component(graphgen.grid_diagonals(12, 15, 0.05, 2)),
        graphgen.toy_graph(),
    ]
    lams = [graphgen.spectral_lambda(g) for g in gs]
    return gs, lams


def _requests(gs, lams, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        k = int(rng.integers(len(gs)))
        g = gs[k]
        ce = graphgen.canonical_edges(g)
        q = int(rng.integers(1, min(g.m, 40) + 1))
        e = ce[rng.choice(g.m, q, replace=False)].copy()
        flip = rng.random(q) < 0.5  # either orientation is a valid query
        e[flip] = e[flip][:, ::-1]
        reqs.append({"graph": k, "edges": np.ascontiguousarray(e, dtype=np.int32),
                     "eps": float(rng.choice([0.1, 0.2, 0.3])), "seed": int(rng.integers(1, 4)),
                     "tau_cap": 64})
    return reqs


def _alone(saba, gs, lams, r):
    import torch
    sg = saba.SabaGraph.from_graph(gs[r["graph"]])
    sc, _ = saba.aesc_query(sg, torch.from_numpy(r["edges"]).cuda(), r["eps"], lams[r["graph"]],
                            r["seed"], tau_cap=r["tau_cap"])
    return sc.cpu().numpy()


def _submit(srv, lams, r):
    return srv.submit(r["graph"], r["edges"], r["eps"], lams[r["graph"]], r["seed"],
                      tau_cap=r["tau_cap"])


@pytest.mark.parametrize("schedule", [0, 2])
def test_served_results_equal_alone(saba, orc, graphs, schedule):
    """Served results equal each request alone, with the served handle on the stride
    schedule or on the staged one (two lanes each launching LDS-staged walk-pair kernels)."""
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    saba.set_config(mg, est_walk_queue=schedule)
    reqs = _requests(gs, lams, 14, 1)
    expect = [_alone(saba, gs, lams, r) for r in reqs]
    with saba.SabaServer(mg, lanes=2, max_batch_sources=5) as srv:
        tickets = [_submit(srv, lams, r) for r in reqs]
        for t, r, e in zip(tickets, reqs, expect):
            sc, res = srv.wait(t)
            assert res["status"] == 0
            assert res["instances"] == len(np.unique(r["edges"]))
            assert res["batches"] >= 1 and res["latency_ms"] >= res["queue_ms"] >= 0.0
            assert np.array_equal(sc.cpu().numpy(), e)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0 and st["queued_edges"] == 0
        assert st["instances"] == sum(len(np.unique(r["edges"])) for r in reqs)
        assert st["batches"] >= 2
    # and the oracle (Alg. 1 for the first graph, all edges) agrees on the served values
    r0 = next(r for r in reqs if r["graph"] == 0)
    so, _ = orc.aesc(gs[0], r0["eps"], lams[0], r0["seed"], tau_cap=64, query=r0["edges"])
    np.testing.assert_allclose(expect[reqs.index(r0)], so, rtol=1e-12, atol=1e-15)


def test_served_eigenpair_requests_equal_alone(saba, graphs):
    """omega > 0 requests (the eigenpair form, radius left to the library) mixed with plain ones:
    each served result equals the same request alone on a handle holding only its graph."""
    import torch
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    reqs = _requests(gs, lams, 12, 7)
    for i, r in enumerate(reqs):
        r["omega"] = 3 if i % 2 == 0 else 0
    expect = []
    for r in reqs:
        sg = saba.SabaGraph.from_graph(gs[r["graph"]])
        lam = 0.0 if r["omega"] else lams[r["graph"]]
        sc, _ = saba.aesc_query(sg, torch.from_numpy(r["edges"]).cuda(), r["eps"], lam, r["seed"],
                                tau_cap=r["tau_cap"], omega=r["omega"])
        expect.append(sc.cpu().numpy())
    with saba.SabaServer(mg, lanes=2, max_batch_sources=5) as srv:
        tickets = [srv.submit(r["graph"], r["edges"], r["eps"],
                              0.0 if r["omega"] else lams[r["graph"]], r["seed"],
                              tau_cap=r["tau_cap"], omega=r["omega"]) for r in reqs]
        for t, r, e in zip(tickets, reqs, expect):
            sc, res = srv.wait(t)
            assert res["status"] == 0
            assert np.array_equal(sc.cpu().numpy(), e), r["omega"]
    # the correction is there: the same request without it differs
    r = next(x for x in reqs if x["omega"])
    plain = _alone(saba, gs, lams, r)
    assert not np.array_equal(plain, expect[reqs.index(r)])


def test_staggered_arrivals_and_lanes(saba, graphs):
    """Requests submitted while others run, waited for out of order, on three lanes with tiny
    batches, plus duplicate pairs in one request: still identical to running alone."""
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    reqs = _requests(gs, lams, 12, 2)
    dup = dict(reqs[0])
    dup["edges"] = np.ascontiguousarray(np.concatenate([reqs[0]["edges"],
                                                        reqs[0]["edges"][::-1, ::-1]]))
    reqs.append(dup)
    expect = [_alone(saba, gs, lams, r) for r in reqs]
    got = {}
    with saba.SabaServer(mg, lanes=3, max_batch_sources=3) as srv:
        live = []
        for i, r in enumerate(reqs):
            live.append((i, _submit(srv, lams, r)))
            if i % 4 == 3:  # wait for an earlier one while later ones keep arriving
                j, t = live.pop(0)
                got[j] = srv.wait(t)[0].cpu().numpy()
        for j, t in reversed(live):
            got[j] = srv.wait(t)[0].cpu().numpy()
    for i, e in enumerate(expect):
        assert np.array_equal(got[i], e), i
    q0 = len(reqs[0]["edges"])
    assert np.array_equal(got[len(reqs) - 1][:q0], got[len(reqs) - 1][q0:][::-1])


def test_backpressure_and_errors(saba, graphs):
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    big = graphgen.canonical_edges(gs[1])[:200]
    with saba.SabaServer(mg, lanes=1, max_queued_edges=250, arena_edges=300) as srv:
        t0 = srv.submit(1, big, 0.1, lams[1], 1, tau_cap=64)
        # the queue holds 200 edges until that request finishes: 100 more exceed the bound
        with pytest.raises(saba.SabaError) as ei:
            srv.submit(1, big[:100], 0.1, lams[1], 1, tau_cap=64)
        assert ei.value.name == "SABA_E_BUSY"
        sc0, _ = srv.wait(t0)
        t1 = srv.submit(1, big[:100], 0.1, lams[1], 1, tau_cap=64)
        sc1, _ = srv.wait(t1)
        assert np.array_equal(sc1.cpu().numpy(), sc0.cpu().numpy()[:100])
        assert srv.stats()["rejected"] == 1
        with pytest.raises(saba.SabaError) as ei:
            srv.submit(0, np.array([[0, 0]], dtype=np.int32), 0.2, lams[0], 1)
        assert ei.value.name == "SABA_E_NOT_EDGE"
        with pytest.raises(saba.SabaError) as ei:  # more pairs than the arena holds
            srv.submit(1, graphgen.canonical_edges(gs[1])[:301], 0.2, lams[1], 1)
        assert ei.value.name == "SABA_E_INVALID"
        with pytest.raises(saba.SabaError) as ei:
            srv.submit(7, big[:1], 0.2, 0.5, 1)
        assert ei.value.name == "SABA_E_INVALID"
        with pytest.raises(saba.SabaError) as ei:
            srv.wait(987654)
        assert ei.value.name == "SABA_E_INVALID"
        t = srv.submit(2, np.zeros((0, 2), dtype=np.int32), 0.2, lams[2], 1)
        sc, res = srv.wait(t, timeout_ms=0)
        assert sc.numel() == 0 and res["status"] == 0


def test_destroy_with_requests_in_flight(saba, graphs):
    """Destroying a busy server cancels what has not started and returns."""
    gs, lams = graphs
    mg = saba.SabaGraph.from_graphs(gs)
    srv = saba.SabaServer(mg, lanes=2, max_batch_sources=2)
    for r in _requests(gs, lams, 20, 3):
        _submit(srv, lams, r)
    srv.close()
    # the handle is still usable afterwards
    import torch
    e = torch.from_numpy(graphgen.canonical_edges(gs[3])[:2].copy()).cuda()
    sg = saba.SabaGraph.from_graph(gs[3])
    sc, _ = saba.aesc_query(sg, e, 0.2, lams[3], 1)
    assert sc.numel() == 2


def test_16_graph_server_full_size_served_match_alone_and_oracle(saba, orc):
    """The serving benchmark's 16 resident graphs at full size (Chung-Lu, n = 10^4 .. 10^6) under
    its server settings (2 lanes, 32 GiB of source scratch): a burst of 16 requests of 1-512
    edges (one of them on the 10^6-vertex graph) served together equals each request run alone,
    also with the served handle on the staged walk-pair schedule (both lanes then launch
    LDS-staged kernels for graphs of different sizes at once), and 6 edges of the largest
    graph's request and of another match the oracle."""
    import os
    import torch
    import bench
    print("16-graph server at full size: building the graphs", flush=True)
    gs, lams = bench.serve_workload()
    ces = [graphgen.canonical_edges(g) for g in gs]
    rng = np.random.default_rng(11)
    reqs = []
    for j in range(16):
        k = 15 if j == 0 else int(rng.integers(len(gs)))
        q = int(rng.integers(1, 513))
        pick = np.sort(rng.choice(ces[k].shape[0], q, replace=False))
        reqs.append({"graph": k, "edges": np.ascontiguousarray(ces[k][pick]),
                     "eps": float(rng.choice([0.1, 0.2, 0.3])), "seed": 1, "tau_cap": 4096})
    mg = saba.SabaGraph.from_graphs(gs, trusted=True)
    with saba.SabaServer(mg, lanes=2, mem_budget=32 << 30) as srv:
        tickets = [_submit(srv, lams, r) for r in reqs]
        served = [srv.wait(t)[0].cpu().numpy() for t in tickets]
    print("16-graph server at full size: the staged walk-pair schedule", flush=True)
    saba.set_config(mg, est_walk_queue=2)
    with saba.SabaServer(mg, lanes=2, mem_budget=32 << 30) as srv:
        tickets = [_submit(srv, lams, r) for r in reqs]
        for t, sc in zip(tickets, served):
            assert np.array_equal(srv.wait(t)[0].cpu().numpy(), sc)
    saba.set_config(mg)
    handles = {}
    for r, sc in zip(reqs, served):
        k = r["graph"]
        if k not in handles:
            handles[k] = saba.SabaGraph.from_graph(gs[k], trusted=True)
        alone, _ = saba.aesc_query(handles[k], torch.from_numpy(r["edges"]).cuda(), r["eps"],
                                   lams[k], 1, tau_cap=4096)
        assert np.array_equal(sc, alone.cpu().numpy()), k
    for j in (0, 1):
        r = reqs[j]
        sel = np.arange(min(6, r["edges"].shape[0]))
        print(f"16-graph server, oracle check: graph {r['graph']} n={gs[r['graph']].n} eps={r['eps']}", flush=True)
        so, _ = orc.aesc(gs[r["graph"]], r["eps"], lams[r["graph"]], 1, query=r["edges"][sel],
                         tau_cap=4096, nthreads=min(16, os.cpu_count() or 1))
        np.testing.assert_allclose(served[j][sel], so, rtol=1e-12, atol=1e-15)
