"""MI355X (gfx950) random-bouquet walks and TGT+ spanning-centrality estimation.

The computation lives in libsaba.so (HIP kernels behind the C-ABI declared in
include/saba.h); this package is its Python binding.
"""
from ._binding import (  # noqa: F401
    EXPORTS,
    SABA_SAMPLER_KEYED,
    SABA_SAMPLER_KEYED_MOD,
    SABA_SAMPLER_LITERAL,
    SABA_SAMPLER_STREAM_MOD,
    SABA_SOURCES_EXPLICIT,
    SABA_SOURCES_UNIFORM,
    SABA_WALK_BOUQUET,
    SABA_WALK_NAIVE,
    SABA_WALK_NAIVE_LOG,
    SabaError,
    SabaGraph,
    SabaServer,
    WalkResult,
    aesc,
    aesc_batch,
    aesc_counts,
    aesc_edge_stats,
    aesc_query,
    autotune_aesc,
    autotune_bouquet,
    autotune_walks,
    fail_allocation,
    get_config,
    set_config,
    graph_lambda,
    graph_spectrum,
    probe_random_reads,
    load,
    walks,
    walks_noalloc,
)
