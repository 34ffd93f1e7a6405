"""Synthetic graph generators and CSR canonicalisation (host side, NumPy).

Every generator is seeded and returns a :class:`Graph` in canonical form:
undirected, symmetric int32 CSR, rows sorted ascending, no self-loops and no
duplicate entries.  The paper evaluates on SNAP social/collaboration graphs
(Sec. 5, Table 2), which are not available here; these generators stand in for
them (heavy-tailed R-MAT and Chung-Lu graphs, homogeneous Erdos-Renyi graphs,
and slow-mixing grids).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph


@dataclass
class Graph:
    """Canonical undirected graph in CSR form (int32 row_ptr[n+1], col_idx[2m])."""

    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def to_scipy(self) -> sp.csr_matrix:
        data = np.ones(self.nnz, dtype=np.float64)
        return sp.csr_matrix((data, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def dense_adjacency(self) -> np.ndarray:
        return self.to_scipy().toarray()


def canonical_csr(u: np.ndarray, v: np.ndarray, n: int, name: str = "", meta=None) -> Graph:
    """Symmetrise an edge list, drop self-loops and duplicates, sort rows."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * np.int64(n) + b)
    rows = (key // n).astype(np.int64)
    cols = (key % n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(row_ptr.astype(np.int32), cols, name=name, meta=dict(meta or {}))


def from_edges(edges, n: int, name: str = "") -> Graph:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return canonical_csr(e[:, 0], e[:, 1], n, name=name)


def largest_component(g: Graph) -> Graph:
    """Keep the largest connected component, relabelled in ascending old-id order."""
    ncomp, labels = csgraph.connected_components(g.to_scipy(), directed=False)
    if ncomp == 1:
        return g
    sizes = np.bincount(labels)
    keep = labels == int(np.argmax(sizes))
    newid = -np.ones(g.n, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    sel = keep[rows]
    h = canonical_csr(newid[rows[sel]], newid[g.col_idx[sel]], int(keep.sum()), name=g.name, meta=g.meta)
    h.meta["lcc_of_n"] = g.n
    return h


def er_gnm(n: int, m: int, seed: int) -> Graph:
    """Uniform G(n, m): m distinct unordered pairs drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    chosen = np.zeros(0, dtype=np.int64)
    while chosen.size < m:
        need = m - chosen.size
        a = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        b = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        ok = a != b
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        key = lo * n + hi
        # keep first occurrences in draw order so the result is a uniform subset
        _, first = np.unique(key, return_index=True)
        key = key[np.sort(first)]
        key = key[~np.isin(key, chosen)]
        chosen = np.concatenate([chosen, key[:need]])
    return canonical_csr(chosen // n, chosen % n, n, name=f"er_n{n}_m{m}_s{seed}",
                         meta={"gen": "er_gnm", "n": n, "m": m, "seed": seed})


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         permute: bool = False) -> Graph:
    """R-MAT generator: each of edge_factor * 2^scale edges descends `scale` quadrant levels."""
    n = 1 << scale
    M = edge_factor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(M, dtype=np.int64)
    dst = np.zeros(M, dtype=np.int64)
    ab, abc = a + b, a + b + c
    chunk = 1 << 22
    for lo in range(0, M, chunk):
        hi = min(M, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.int64)
        d = np.zeros(hi - lo, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(hi - lo)
            sbit = (r >= ab).astype(np.int64)
            dbit = (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64)
            s = (s << 1) | sbit
            d = (d << 1) | dbit
        src[lo:hi] = s
        dst[lo:hi] = d
    if permute:
        perm = rng.permutation(n)
        src, dst = perm[src], perm[dst]
    return canonical_csr(src, dst, n, name=f"rmat_s{scale}_ef{edge_factor}_s{seed}",
                         meta={"gen": "rmat", "scale": scale, "edge_factor": edge_factor,
                               "abc": (a, b, c), "seed": seed, "permute": permute})


def chung_lu(n: int, avg_degree: float, exponent: float, seed: int) -> Graph:
    """Chung-Lu (edge-sampling variant): n*avg_degree/2 pairs, endpoints drawn prop. to
    w_i = (i+1)^(-1/(exponent-1)); then symmetrised and deduplicated."""
    rng = np.random.default_rng(seed)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (exponent - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    M = int(round(n * avg_degree / 2))
    u = np.searchsorted(cdf, rng.random(M), side="right")
    v = np.searchsorted(cdf, rng.random(M), side="right")
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    return canonical_csr(u, v, n, name=f"cl_n{n}_k{avg_degree}_b{exponent}_s{seed}",
                         meta={"gen": "chung_lu", "n": n, "avg_degree": avg_degree,
                               "exponent": exponent, "seed": seed})


def grid_diagonals(rows: int, cols: int, frac: float, seed: int) -> Graph:
    """rows x cols 4-neighbour grid plus a random diagonal in a fraction `frac` of cells."""
    rng = np.random.default_rng(seed)
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    us = [idx[:, :-1].ravel(), idx[:-1, :].ravel()]
    vs = [idx[:, 1:].ravel(), idx[1:, :].ravel()]
    cells = (rows - 1) * (cols - 1)
    pick = rng.random(cells) < frac
    tl = idx[:-1, :-1].ravel()[pick]
    br = idx[1:, 1:].ravel()[pick]
    tr = idx[:-1, 1:].ravel()[pick]
    bl = idx[1:, :-1].ravel()[pick]
    flip = rng.random(int(pick.sum())) < 0.5
    us.append(np.where(flip, tr, tl))
    vs.append(np.where(flip, bl, br))
    return canonical_csr(np.concatenate(us), np.concatenate(vs), rows * cols,
                         name=f"grid{rows}x{cols}_d{frac}_s{seed}",
                         meta={"gen": "grid_diagonals", "rows": rows, "cols": cols,
                               "frac": frac, "seed": seed})


def circulant(n: int, steps=(1, 2)) -> Graph:
    """Circulant graph C_n(steps): vertex i is joined to i - s and i + s (mod n) for every s in
    `steps` (0 < s < n/2, distinct).  Every vertex has degree 2 |steps|.  The CSR is built
    directly, without the edge-list canonicalisation, so graphs of 10^7-10^8 vertices take
    seconds (large vertex counts for bucket-count limits)."""
    st = sorted({int(x) for x in steps})
    if not st or st[0] <= 0 or 2 * st[-1] >= n:
        raise ValueError("steps must lie in 0 < s < n/2")
    k = 2 * len(st)
    if (n + 1) * k >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    off = np.array([-x for x in st] + st, dtype=np.int64)
    col = np.empty((n, k), dtype=np.int32)
    base = np.arange(n, dtype=np.int64)
    for j, o in enumerate(off):
        col[:, j] = (base + o) % n
    col.sort(axis=1)
    row_ptr = (np.arange(n + 1, dtype=np.int64) * k).astype(np.int32)
    return Graph(row_ptr, col.reshape(-1), name=f"circulant{n}_{'_'.join(map(str, st))}",
                 meta={"gen": "circulant", "n": n, "steps": st})


def toy_graph() -> Graph:
    """The 4-vertex, 5-edge sample graph of Fig. 1: A,D of degree 2, B,C of degree 3
    (K4 minus the edge A-D). Vertex ids: A=0, B=1, C=2, D=3."""
    return from_edges([(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)], 4, name="fig1_toy")


def canonical_edges(g: Graph) -> np.ndarray:
    """Undirected edges (u < v) in lexicographic order, shape [m, 2] int32."""
    rows = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.row_ptr))
    sel = rows < g.col_idx
    return np.stack([rows[sel], g.col_idx[sel]], axis=1).astype(np.int32)


def uniform_sources(g: Graph, n_walks: int, seed: int) -> np.ndarray:
    """Walk start vertices drawn uniformly from the non-isolated vertices (int32)."""
    pool = np.flatnonzero(np.diff(g.row_ptr) > 0).astype(np.int32)
    rng = np.random.default_rng(seed)
    return pool[rng.integers(0, pool.size, size=n_walks, dtype=np.int64)]


def is_bipartite(g: Graph) -> bool:
    color = -np.ones(g.n, dtype=np.int8)
    for s in range(g.n):
        if color[s] >= 0:
            continue
        color[s] = 0
        stack = [s]
        while stack:
            x = stack.pop()
            for y in g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]:
                if color[y] < 0:
                    color[y] = 1 - color[x]
                    stack.append(int(y))
                elif color[y] == color[x]:
                    return False
    return True


def spectral_lambda(g: Graph) -> float:
    """max(|lambda_2|, |lambda_n|) of D^{-1/2} A D^{-1/2} (the estimator's spectral input).

    Dense eigvalsh for small graphs, ARPACK otherwise."""
    d = g.degrees.astype(np.float64)
    if np.any(d == 0):
        raise ValueError("spectral_lambda needs a graph without isolated vertices")
    inv = 1.0 / np.sqrt(d)
    A = g.to_scipy()
    N = sp.diags(inv) @ A @ sp.diags(inv)
    if g.n <= 3000:
        ev = np.linalg.eigvalsh(N.toarray())
        ev = np.sort(ev)
        return float(max(abs(ev[-2]), abs(ev[0])))
    from scipy.sparse.linalg import eigsh
    vals = eigsh(N, k=3, which="LM", return_eigenvectors=False, tol=1e-10, maxiter=100000)
    vals = np.sort(np.abs(vals))[::-1]
    # the largest magnitude is the trivial eigenvalue 1 of a connected graph
    return float(vals[1])
