"""On-device lambda (saba_graph_lambda) against the oracle's dense eigendecomposition, and the
estimator with lambda left to the library against the same run with lambda passed in."""
import numpy as np
import pytest

import graphgen
from oracle import exact_sc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def saba():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14056_amd as saba
    saba.load()
    return saba


GRAPHS = {
    "er300": lambda: graphgen.largest_component(graphgen.er_gnm(300, 1200, 3)),
    "er2000": lambda: graphgen.largest_component(graphgen.er_gnm(2000, 8000, 1)),
    "chung_lu3000": lambda: graphgen.largest_component(graphgen.chung_lu(3000, 8, 2.3, 5)),
    "toy": graphgen.toy_graph,
    "petersen": lambda: graphgen.from_edges(
        [(i, (i + 1) % 5) for i in range(5)] + [(i, i + 5) for i in range(5)] +
        [(5 + i, 5 + (i + 2) % 5) for i in range(5)], 10),
}


@pytest.mark.parametrize("gname", list(GRAPHS))
def test_lambda_matches_dense_eigendecomposition(saba, gname):
    g = GRAPHS[gname]()
    print(f"lambda parity graph={gname} n={g.n}", flush=True)
    lam, ev = exact_sc.spectral_lambda(g.row_ptr, g.col_idx, g.n)
    sg = saba.SabaGraph.from_graph(g)
    r = saba.graph_lambda(sg, max_iters=400)
    assert r["converged"] == 1
    # Ritz values lie inside the spectrum of N on the complement of sqrt(d) ...
    assert ev[0] - 1e-12 <= r["lambdan"] and r["lambda2"] <= ev[-2] + 1e-12
    # ... and converge to its extremes
    assert abs(r["lambda2"] - ev[-2]) < 1e-8 and abs(r["lambdan"] - ev[0]) < 1e-8
    assert abs(r["lambda"] - lam) < 1e-8
    assert r["lambda_bound"] >= lam - 1e-12
    # deterministic
    assert saba.graph_lambda(sg, max_iters=400) == r


def test_lambda_per_graph_of_a_multi_graph_handle(saba):
    gs = [GRAPHS[k]() for k in ("er300", "toy", "chung_lu3000")]
    mg = saba.SabaGraph.from_graphs(gs)
    for k, g in enumerate(gs):
        alone = saba.graph_lambda(saba.SabaGraph.from_graph(g))
        assert saba.graph_lambda(mg, index=k) == alone


def test_estimator_with_lambda_left_to_the_library(saba):
    import torch
    g = GRAPHS["er300"]()
    sg = saba.SabaGraph.from_graph(g)
    lb = saba.graph_lambda(sg)["lambda_bound"]
    auto, _ = saba.aesc(sg, 0.2, 0.0, 3, tau_cap=64)
    given, _ = saba.aesc(sg, 0.2, min(lb, 1 - 1e-12), 3, tau_cap=64)
    assert torch.equal(auto, given)
    # the radius the library took is the dense one up to the Lanczos residual (the estimator's
    # parity at a given lambda is covered by the estimator tests)
    lam, _ = exact_sc.spectral_lambda(g.row_ptr, g.col_idx, g.n)
    assert lam - 1e-12 <= lb <= lam + 1e-6
    # the server resolves it too
    e = graphgen.canonical_edges(g)[:9]
    with saba.SabaServer(saba.SabaGraph.from_graphs([g])) as srv:
        sc, _ = srv.wait(srv.submit(0, e, 0.2, 0.0, 3, tau_cap=64))
    q, _ = saba.aesc_query(sg, torch.from_numpy(e.copy()).cuda(), 0.2, min(lb, 1 - 1e-12), 3,
                           tau_cap=64)
    assert torch.equal(sc, q)


def test_lambda_errors(saba):
    disc = graphgen.from_edges([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)], 6)
    with pytest.raises(saba.SabaError) as ei:
        saba.graph_lambda(saba.SabaGraph.from_graph(disc))
    assert ei.value.name == "SABA_E_DISCONNECTED"
    with pytest.raises(saba.SabaError) as ei:
        saba.graph_lambda(saba.SabaGraph.from_graph(graphgen.toy_graph()), index=1)
    assert ei.value.name == "SABA_E_INVALID"


def test_lambda_chung_lu_1e6_against_arpack(saba):
    """The 10^6-vertex graph of the estimator benchmark: Lanczos on the device against ARPACK."""
    g = graphgen.largest_component(graphgen.chung_lu(1000000, 10, 2.5, 1))
    ref = graphgen.spectral_lambda(g)
    r = saba.graph_lambda(saba.SabaGraph.from_graph(g, trusted=True), max_iters=1000)
    print(f"lambda chung-lu 1e6 device={r!r} arpack={ref!r}", flush=True)
    assert abs(r["lambda"] - ref) < 1e-6
    assert r["lambda_bound"] >= ref - 1e-9
