"""The eigenpair form of CalculateTau (Alg. 1's omega > 0) on the device.

saba_graph_spectrum is checked against the oracle's dense eigendecomposition (eigenvalues,
eigenvectors up to sign within the Davis-Kahan bound of the reported residual, the radius of
the rest of the spectrum) and against closed forms on graphs with repeated eigenvalues.  The
estimator with omega > 0 is checked against the oracle's truncated series plus its eigen tail
correction: tau and the deterministic and Monte-Carlo parts bit for bit (both sides take tau
from the same radius), the correction within the eigenvector error.
"""
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
    "er1500": lambda: graphgen.largest_component(graphgen.er_gnm(1500, 6000, 1)),
    "chung_lu2000": lambda: graphgen.largest_component(graphgen.chung_lu(2000, 8, 2.3, 5)),
}


def _dense(g, omega):
    return exact_sc.top_eigenpairs(g.row_ptr, g.col_idx, g.n, omega)


def _gap(g, vals):
    """Distance of each kept eigenvalue to the rest of the spectrum of N."""
    _, ev = exact_sc.spectral_lambda(g.row_ptr, g.col_idx, g.n)
    out = []
    for v in vals:
        others = ev[np.abs(ev - v) > 1e-12]
        out.append(np.min(np.abs(others - v)))
    return np.array(out)


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("omega", [1, 4, 8])
def test_spectrum_matches_dense_eigendecomposition(saba, gname, omega):
    g = GRAPHS[gname]()
    print(f"spectrum parity graph={gname} n={g.n} omega={omega}", flush=True)
    vals, vecs, rest = _dense(g, omega)
    sg = saba.SabaGraph.from_graph(g)
    r = saba.graph_spectrum(sg, omega)
    assert r["pairs"] == omega and r["converged"] == 1
    assert r["max_residual"] <= 1e-10
    np.testing.assert_allclose(r["values"], vals, rtol=0, atol=1e-10)
    u = r["vectors"].cpu().numpy()
    gap = _gap(g, vals)
    for k in range(omega):
        s = np.sign(u[k] @ vecs[:, k])
        err = np.linalg.norm(u[k] - s * vecs[:, k])
        # sin(angle) <= residual / gap (Davis-Kahan); the norm of the difference is within
        # sqrt(2) of it
        assert err <= 2.0 * r["max_residual"] / gap[k] + 1e-12, (k, err, gap[k])
    np.testing.assert_allclose(u @ u.T, np.eye(omega), atol=1e-12)
    assert abs(r["lambda_rest"] - rest) < 1e-8
    assert r["lambda_rest_bound"] >= rest - 1e-12
    # deterministic
    r2 = saba.graph_spectrum(sg, omega)
    assert np.array_equal(r2["values"], r["values"])
    assert np.array_equal(r2["vectors"].cpu().numpy(), u)


def _cycle(n):
    return graphgen.from_edges([(i, (i + 1) % n) for i in range(n)], n)


def test_spectrum_repeated_eigenvalues(saba):
    """One start vector reaches one direction of each eigenspace: on the Petersen graph
    (theta = 1/3 five times, -2/3 four times) two pairs are found, and the deflated run sees
    the other copies of -2/3 as the radius of the rest; on an odd cycle (cos(2 pi k / n) twice
    each) the rest keeps the second copy of -cos(pi / n)."""
    pet = graphgen.from_edges([(i, (i + 1) % 5) for i in range(5)] + [(i, i + 5) for i in range(5)] +
                              [(5 + i, 5 + (i + 2) % 5) for i in range(5)], 10)
    r = saba.graph_spectrum(saba.SabaGraph.from_graph(pet), 3)
    assert r["pairs"] == 2
    np.testing.assert_allclose(r["values"], [-2 / 3, 1 / 3, 0.0], atol=1e-12)
    assert abs(r["lambda_rest"] - 2 / 3) < 1e-10
    n = 21
    r = saba.graph_spectrum(saba.SabaGraph.from_graph(_cycle(n)), 2)
    assert r["pairs"] == 2
    np.testing.assert_allclose(r["values"], [-np.cos(np.pi / n), np.cos(2 * np.pi / n)],
                               atol=1e-12)
    assert abs(r["lambda_rest"] - np.cos(np.pi / n)) < 1e-10


def test_spectrum_full_set_leaves_nothing(saba):
    g = graphgen.largest_component(graphgen.er_gnm(12, 30, 2))
    r = saba.graph_spectrum(saba.SabaGraph.from_graph(g), g.n - 1)
    vals, _, rest = _dense(g, g.n - 1)
    assert rest == 0.0 and r["pairs"] == g.n - 1
    np.testing.assert_allclose(r["values"], vals, atol=1e-12)
    assert r["lambda_rest_bound"] < 1e-10


def _canon_taus(g, tau_csr):
    e = graphgen.canonical_edges(g)
    pos = np.array([g.row_ptr[u] + np.searchsorted(g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]], v)
                    for u, v in e])
    return e, tau_csr[pos]


def _corr_tol(g, e, taus, vals, vecs, res):
    """Per-edge bound on how far the device's correction may sit from the oracle's: each
    eigenvector is within 2 res / gap of the true one (Davis-Kahan), each eigenvalue within
    res, and the correction is smooth in both."""
    d = np.diff(g.row_ptr).astype(np.float64)
    a, b = e[:, 0], e[:, 1]
    gap = _gap(g, vals)
    tol = np.full(len(e), 1e-15)
    for k, th in enumerate(vals):
        y = vecs[:, k] / np.sqrt(d)
        delta = np.abs(y[a] - y[b])
        eta = (2.0 * res / gap[k]) * (1 / np.sqrt(d[a]) + 1 / np.sqrt(d[b]))
        p = np.abs(th) ** (taus + 1.0)
        dp = (taus + 1.0) * np.abs(th) ** taus / (1 - th) + p / (1 - th) ** 2
        tol += (2 * delta * eta + eta ** 2) * p / (1 - th) + delta ** 2 * dp * res
    return tol


def _omega_case(saba, orc, g, omega, eps, seed, **kw):
    vals, vecs, rest = _dense(g, omega)
    sg = saba.SabaGraph.from_graph(g)
    res = saba.graph_spectrum(sg, omega, vectors=False)["max_residual"]
    o_gpu, _ = saba.aesc_edge_stats(sg, eps, rest, seed, omega=omega, **kw)
    okw = dict(kw)
    if "group" in okw:
        okw["G"], okw["S"] = okw.pop("group"), okw.pop("spread")
    sc_o, o_orc = orc.aesc(g, eps, rest, seed=seed, **okw)
    gpu = {k: v.cpu().numpy() for k, v in o_gpu.items()}
    for k in ("tau", "ttau", "nreq", "vis0", "vis1"):
        assert np.array_equal(gpu[k], o_orc[k]), k
    assert np.array_equal(gpu["D"], o_orc["D"])
    e, taus = _canon_taus(g, o_orc["tau"])
    corr = exact_sc.eigen_tail_correction(g.row_ptr, g.col_idx, g.n, e, taus, vals, vecs)
    tol = 1e-12 * np.abs(sc_o) + _corr_tol(g, e, taus, vals, vecs, res)
    assert np.all(np.abs(gpu["sc"] - (sc_o + corr)) <= tol)
    return sg, gpu, sc_o, corr, e, taus, rest


@pytest.mark.parametrize("omega", [2, 6])
def test_estimator_push_all_with_eigen_correction(saba, orc, omega):
    """Deterministic levels only: the estimate is the truncated series plus the kept pairs'
    tail, so it misses the exact resistance by at most the rest's tail bound."""
    g = GRAPHS["er300"]()
    sg, gpu, sc_o, corr, e, taus, rest = _omega_case(saba, orc, g, omega, 0.05, 4, push_all=True,
                                                      tau_cap=256)
    exact = exact_sc.sc_pinv(g.row_ptr, g.col_idx, g.n, [tuple(x) for x in e])
    d = np.diff(g.row_ptr)
    bound = rest ** (taus + 1) * (1 / d[e[:, 0]] + 1 / d[e[:, 1]]) / (1 - rest)
    assert np.all(np.abs(exact - gpu["sc"]) <= bound + 1e-12)


@pytest.mark.parametrize("kw", [{}, {"group": 64, "spread": 20}])
def test_estimator_walks_with_eigen_correction(saba, orc, kw):
    g = GRAPHS["er300"]()
    print(f"omega estimator parity {kw}", flush=True)
    sg, gpu, sc_o, corr, e, taus, rest = _omega_case(saba, orc, g, 4, 0.15, 7, **kw)
    # the correction is not negligible next to the estimate's own error scale
    assert np.max(np.abs(corr)) > 1e-7


def test_query_equals_all_edges_and_library_radius(saba):
    import torch
    g = GRAPHS["chung_lu2000"]()
    sg = saba.SabaGraph.from_graph(g)
    r = saba.graph_spectrum(sg, 5)
    lam = min(r["lambda_rest_bound"], 1 - 1e-12)
    auto, st_a = saba.aesc(sg, 0.2, 0.0, 3, omega=5)
    given, _ = saba.aesc(sg, 0.2, lam, 3, omega=5)
    assert torch.equal(auto, given)
    e = graphgen.canonical_edges(g)
    rng = np.random.default_rng(2)
    pick = rng.choice(len(e), 300, replace=False)
    q = e[pick].copy()
    q[::2] = q[::2, ::-1]  # both orientations
    qs, _ = saba.aesc_query(sg, torch.from_numpy(np.ascontiguousarray(q)).cuda(), 0.2, 0.0, 3,
                            omega=5)
    assert torch.equal(qs.cpu(), auto.cpu()[pick])
    # fewer walk steps than the plain series: tau comes from a smaller radius
    _, st_0 = saba.aesc(sg, 0.2, 0.0, 3)
    assert st_a["walk_steps"] < st_0["walk_steps"]


def test_batch_mixes_omega_and_plain_requests(saba):
    import torch
    g = GRAPHS["er300"]()
    sg = saba.SabaGraph.from_graph(g)
    lam = graphgen.spectral_lambda(g)
    reqs = [dict(graph=0, eps=0.2, lam=lam, seed=5, m=g.m),
            dict(graph=0, eps=0.2, lam=lam, seed=5, m=g.m, omega=3)]
    out, _ = saba.aesc_batch(sg, reqs)
    a, _ = saba.aesc(sg, 0.2, lam, 5)
    b, _ = saba.aesc(sg, 0.2, lam, 5, omega=3)
    assert torch.equal(out[0], a) and torch.equal(out[1], b)
    assert not torch.equal(a, b)


def test_omega_errors(saba):
    import torch
    g = GRAPHS["er300"]()
    sg = saba.SabaGraph.from_graph(g)
    for bad in (-1, 65):
        with pytest.raises(saba.SabaError) as ei:
            saba.aesc(sg, 0.2, 0.5, 1, omega=bad)
        assert ei.value.name == "SABA_E_INVALID"
    with pytest.raises(saba.SabaError) as ei:
        saba.graph_spectrum(sg, 0)
    assert ei.value.name == "SABA_E_INVALID"
    toy = saba.SabaGraph.from_graph(graphgen.toy_graph())
    with pytest.raises(saba.SabaError) as ei:
        saba.aesc(toy, 0.2, 0.0, 1, omega=graphgen.toy_graph().n)
    assert ei.value.name == "SABA_E_INVALID"
    disc = graphgen.from_edges([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)], 6)
    with pytest.raises(saba.SabaError) as ei:
        saba.graph_spectrum(saba.SabaGraph.from_graph(disc), 1)
    assert ei.value.name == "SABA_E_DISCONNECTED"
    e = graphgen.canonical_edges(g)[:4]
    with saba.SabaServer(saba.SabaGraph.from_graphs([g])) as srv:
        with pytest.raises(saba.SabaError) as ei:
            srv.submit(0, e, 0.2, 0.5, 3, omega=65)
        assert ei.value.name == "SABA_E_INVALID"


def test_spectrum_chung_lu_1e6(saba):
    """The 10^6-vertex graph of the estimator benchmark: eight pairs converge, the rest of the
    spectrum is smaller than lambda, and every kept |theta| is at least the rest's radius."""
    g = graphgen.largest_component(graphgen.chung_lu(1000000, 10, 2.5, 1))
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    r = saba.graph_spectrum(sg, 8, vectors=False)
    lam = saba.graph_lambda(sg, max_iters=1000)
    print(f"spectrum chung-lu 1e6 {dict((k, v) for k, v in r.items() if k != 'vectors')} "
          f"lambda={lam['lambda']}", flush=True)
    assert r["converged"] == 1 and r["pairs"] == 8
    assert abs(abs(r["values"][0]) - lam["lambda"]) < 1e-8
    assert r["lambda_rest"] < lam["lambda"]
    assert np.all(np.abs(r["values"]) >= r["lambda_rest"] - 1e-8)
