"""Exact spanning centrality, the target of the estimator's epsilon contract.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU library.

Definitions followed:
  * SC(e) = fraction of spanning trees of G that contain e
    = 1 - T(G minus e) / T(G)   (Sec. 2.1, the formula for SC).
  * By Kirchhoff's matrix-tree theorem (invoked in Sec. 2.1 for the exact
    algorithm) T(G) is any cofactor of the Laplacian L = D - A, and SC(e) for
    e = {u, v} equals the effective resistance (e_u - e_v)^T L^+ (e_u - e_v).
  * Truncated resistance r_tau (the quantity TGT+ estimates before walks,
    Alg. 1): sum over l = 0..tau of y^T N^l y with y = e_s/sqrt(d_s) - e_t/sqrt(d_t)
    and N = D^{-1/2} A D^{-1/2}, evaluated here with dense matrix powers of the
    transition matrix P = D^{-1} A.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def _dense_laplacian(row_ptr, col_idx, n):
    A = np.zeros((n, n), dtype=np.float64)
    for u in range(n):
        for i in range(row_ptr[u], row_ptr[u + 1]):
            A[u, col_idx[i]] = 1.0
    return np.diag(A.sum(axis=1)) - A, A


def canonical_edge_list(row_ptr, col_idx, n):
    out = []
    for u in range(n):
        for i in range(row_ptr[u], row_ptr[u + 1]):
            v = int(col_idx[i])
            if v > u:
                out.append((u, v))
    return out


def sc_pinv(row_ptr, col_idx, n, edges=None):
    """Effective resistance of each edge from the FP64 Moore-Penrose pseudoinverse of L."""
    L, _ = _dense_laplacian(row_ptr, col_idx, n)
    Lp = np.linalg.pinv(L, hermitian=True)
    if edges is None:
        edges = canonical_edge_list(row_ptr, col_idx, n)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    u, v = e[:, 0], e[:, 1]
    return Lp[u, u] + Lp[v, v] - 2.0 * Lp[u, v]


def bareiss_det(M):
    """Exact determinant of an integer matrix (fraction-free Bareiss elimination)."""
    A = [[int(x) for x in row] for row in M]
    k = len(A)
    if k == 0:
        return 1
    sign = 1
    prev = 1
    for i in range(k - 1):
        if A[i][i] == 0:
            piv = next((r for r in range(i + 1, k) if A[r][i] != 0), None)
            if piv is None:
                return 0
            A[i], A[piv] = A[piv], A[i]
            sign = -sign
        for r in range(i + 1, k):
            for cidx in range(i + 1, k):
                A[r][cidx] = (A[r][cidx] * A[i][i] - A[r][i] * A[i][cidx]) // prev
            A[r][i] = 0
        prev = A[i][i]
    return sign * A[k - 1][k - 1]


def spanning_tree_count(edges, n):
    """T(G) by the matrix-tree theorem: determinant of the Laplacian with row/col 0 removed."""
    L = [[0] * n for _ in range(n)]
    for u, v in edges:
        if u == v:
            continue
        L[u][u] += 1
        L[v][v] += 1
        L[u][v] -= 1
        L[v][u] -= 1
    red = [row[1:] for row in L[1:]]
    return bareiss_det(red)


def sc_matrix_tree(edges, n):
    """SC(e) = 1 - T(G minus e)/T(G) as exact fractions."""
    edges = [tuple(e) for e in edges]
    T = spanning_tree_count(edges, n)
    out = []
    for i in range(len(edges)):
        rest = edges[:i] + edges[i + 1:]
        out.append(1 - Fraction(spanning_tree_count(rest, n), T))
    return out


def sc_enumerate(edges, n):
    """SC by brute force: enumerate every (n-1)-subset of edges, keep the spanning trees."""
    edges = [tuple(e) for e in edges]
    m = len(edges)
    count = [0] * m
    total = 0
    for subset in itertools.combinations(range(m), n - 1):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        ok = True
        for i in subset:
            a, b = find(edges[i][0]), find(edges[i][1])
            if a == b:
                ok = False
                break
            parent[a] = b
        if ok:
            total += 1
            for i in subset:
                count[i] += 1
    return [Fraction(c, total) for c in count], total


def truncated_resistance(row_ptr, col_idx, n, edges, taus):
    """r_tau(s,t) = sum_{l=0}^{tau} y^T N^l y, y = e_s/sqrt(d_s) - e_t/sqrt(d_t),
    evaluated spectrally: N = U diag(mu) U^T gives sum_k c_k^2 sum_{l<=tau} mu_k^l with
    c = U^T y (one tau per edge)."""
    _, A = _dense_laplacian(row_ptr, col_idx, n)
    d = A.sum(axis=1)
    inv = 1.0 / np.sqrt(d)
    N = inv[:, None] * A * inv[None, :]
    mu, U = np.linalg.eigh(N)
    out = np.zeros(len(edges))
    for i, ((s, t), tau) in enumerate(zip(edges, taus)):
        c = U[s, :] * inv[s] - U[t, :] * inv[t]
        geo = np.array([sum(mk ** l for l in range(int(tau) + 1)) for mk in mu])
        out[i] = float(np.sum(c * c * geo))
    return out


def spectral_lambda(row_ptr, col_idx, n):
    """lambda = max(|lambda_2|, |lambda_n|) of N = D^{-1/2} A D^{-1/2} (the spectral input of
    CalculateTau in Alg. 1), written out as the definition: a dense symmetric eigen-
    decomposition of N (a connected graph has lambda_1 = 1).  Returns (lambda, eigenvalues
    in ascending order)."""
    _, A = _dense_laplacian(row_ptr, col_idx, n)
    s = 1.0 / np.sqrt(A.sum(axis=1))
    ev = np.linalg.eigvalsh(s[:, None] * A * s[None, :])
    return float(max(abs(ev[-2]), abs(ev[0]))), ev


def top_eigenpairs(row_ptr, col_idx, n, omega):
    """The omega eigenpairs of N = D^{-1/2} A D^{-1/2} of largest |eigenvalue| other than the
    trivial one (eigenvalue 1, vector sqrt(d)/sqrt(2m)), by a dense symmetric eigen-
    decomposition; and lambda_rest, the largest |eigenvalue| of the others.  Returns
    (values[omega], vectors[n, omega], lambda_rest)."""
    _, A = _dense_laplacian(row_ptr, col_idx, n)
    s = 1.0 / np.sqrt(A.sum(axis=1))
    mu, U = np.linalg.eigh(s[:, None] * A * s[None, :])
    keep = np.arange(n - 1)  # eigh sorts ascending: the trivial eigenvalue 1 is the last
    order = keep[np.argsort(-np.abs(mu[keep]), kind="stable")]
    top, rest = order[:omega], order[omega:]
    lam_rest = float(np.max(np.abs(mu[rest]))) if len(rest) else 0.0
    return mu[top], U[:, top], lam_rest


def eigen_tail_correction(row_ptr, col_idx, n, edges, taus, values, vectors):
    """The part of the truncation remainder r - r_tau that the given eigenpairs carry:
    sum_k c_k mu_k^(tau+1) / (1 - mu_k), c_k = (u_k(s)/sqrt(d_s) - u_k(t)/sqrt(d_t))^2,
    the geometric tail of the spectral series of the truncated resistance (one tau per
    edge; the power by repeated multiplication)."""
    d = np.diff(np.asarray(row_ptr)).astype(np.float64)
    out = np.zeros(len(edges))
    for i, ((a, b), tau) in enumerate(zip(edges, taus)):
        acc = 0.0
        for k, mk in enumerate(values):
            c = vectors[a, k] / np.sqrt(d[a]) - vectors[b, k] / np.sqrt(d[b])
            p = mk
            for _ in range(int(tau)):
                p = p * mk
            acc += c * c * p / (1.0 - mk)
        out[i] = acc
    return out
