"""Error paths forced from the host: an allocation failure injected at every point of a walk
call, an estimator call, a spectrum call and a server start leaves each handle usable, and the
next call gives the results of a clean run, bit for bit."""
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
    yield saba
    saba.fail_allocation(0)


@pytest.fixture(scope="module")
def graph():
    return graphgen.largest_component(graphgen.chung_lu(4000, 8, 2.3, 9))


def _fail_then_recover(saba, fresh, run, same):
    """For n = 1, 2, ...: a fresh handle, the n-th allocation failing; the call either
    succeeds (fewer allocations than n) or reports SABA_E_NOMEM, and the next call on the
    same handle matches the clean result."""
    ref = run(fresh())
    failures = 0
    for n in range(1, 40):
        h = fresh()
        saba.fail_allocation(n)
        try:
            out = run(h)
            saba.fail_allocation(0)
            assert same(out, ref), n
            break  # the call needed fewer than n allocations: every point has been covered
        except saba.SabaError as e:
            saba.fail_allocation(0)
            assert e.name == "SABA_E_NOMEM", (n, e)
            failures += 1
        assert same(run(h), ref), n
    assert failures >= 1


def test_walks_recover(saba, graph):
    import torch
    src = torch.from_numpy(graphgen.uniform_sources(graph, 30000, 4)).cuda()

    def run(h):
        r = saba.walks(h, src, 9, 2)
        return r.endpoint.clone(), r.visits.clone()

    _fail_then_recover(saba, lambda: saba.SabaGraph.from_graph(graph), run,
                       lambda a, b: torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]))


def test_estimator_recovers(saba, graph):
    import torch
    lam = graphgen.spectral_lambda(graph)
    e = graphgen.canonical_edges(graph)[::7]
    q = torch.from_numpy(np.ascontiguousarray(e)).cuda()

    def run(h):
        a, _ = saba.aesc(h, 0.25, lam, 6, batch_sources=64)  # several batches
        b, _ = saba.aesc_query(h, q, 0.25, lam, 6)
        return a, b

    _fail_then_recover(saba, lambda: saba.SabaGraph.from_graph(graph), run,
                       lambda x, y: torch.equal(x[0], y[0]) and torch.equal(x[1], y[1]))


def test_spectrum_and_eigen_estimator_recover(saba, graph):
    import torch

    def run(h):
        r = saba.graph_spectrum(h, 3)
        a, _ = saba.aesc(h, 0.25, 0.0, 6, omega=3)
        return r["values"], r["vectors"], a

    _fail_then_recover(saba, lambda: saba.SabaGraph.from_graph(graph), run,
                       lambda x, y: np.array_equal(x[0], y[0]) and torch.equal(x[1], y[1])
                       and torch.equal(x[2], y[2]))


def test_server_start_recovers(saba, graph):
    """A server whose arena or lane pools cannot be allocated is torn down cleanly (lanes,
    streams, pools), and a server started afterwards on the same handle serves correctly."""
    h = saba.SabaGraph.from_graphs([graph])
    failures = 0
    for n in range(1, 40):
        saba.fail_allocation(n)
        try:
            srv = saba.SabaServer(h, mem_budget=1 << 28)
        except saba.SabaError as err:
            saba.fail_allocation(0)
            assert err.name == "SABA_E_NOMEM", (n, err)
            failures += 1
            continue
        saba.fail_allocation(0)
        srv.close()
        break
    assert failures >= 2  # the arena and at least one lane pool
    e = graphgen.canonical_edges(graph)[:50]
    lam = graphgen.spectral_lambda(graph)
    with saba.SabaServer(h, mem_budget=1 << 28) as srv:
        sc, _ = srv.wait(srv.submit(0, e, 0.3, lam, 1))
    import torch
    ref, _ = saba.aesc_query(saba.SabaGraph.from_graph(graph),
                             torch.from_numpy(np.ascontiguousarray(e)).cuda(), 0.3, lam, 1)
    assert torch.equal(sc, ref)


def test_fail_allocation_argument(saba):
    with pytest.raises(saba.SabaError) as ei:
        saba.fail_allocation(-1)
    assert ei.value.name == "SABA_E_INVALID"


def test_walk_index_limits(saba, orc):
    """Walk keys carry a 32-bit walk index: 2^32 walks from uniform starts, or a directed edge
    needing 2^32 walk pairs, are refused (SABA_E_OVERFLOW) before any walk runs; the handle
    stays usable.  The oracle refuses the same estimator case."""
    g = graphgen.largest_component(graphgen.er_gnm(40, 120, 3))
    lam = graphgen.spectral_lambda(g)
    sg = saba.SabaGraph.from_graph(g)
    with pytest.raises(saba.SabaError) as e:
        saba.walks(sg, None, 4, 1, n_walks=1 << 32)
    assert e.value.name == "SABA_E_OVERFLOW"
    # eps = 1e-4 with pure Monte Carlo: c = 32 ln(4m/delta) / eps^2 > 3e10 pairs per edge
    with pytest.raises(saba.SabaError) as e:
        saba.aesc(sg, 1e-4, lam, 1, tilde_tau_max=0)
    assert e.value.name == "SABA_E_OVERFLOW"
    with pytest.raises(ValueError):
        orc.aesc(g, 1e-4, lam, 1, tilde_tau_max=0)
    r = saba.walks(sg, None, 4, 1, n_walks=1000)
    assert int(r.visits.sum()) == 4000
