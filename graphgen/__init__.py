"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the oracle.

This package only builds inputs: graphs in canonical CSR form, walk start
vertices and the spectral constant that the estimator takes as a parameter.
It contains none of the method's arithmetic (no hashing, no sampling rule,
no estimator), so both sides of a parity check can consume it.
"""
from .generators import (  # noqa: F401
    Graph,
    canonical_csr,
    largest_component,
    er_gnm,
    rmat,
    chung_lu,
    grid_diagonals,
    toy_graph,
    circulant,
    from_edges,
    uniform_sources,
    spectral_lambda,
    canonical_edges,
    is_bipartite,
)
