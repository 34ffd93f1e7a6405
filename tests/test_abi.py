"""CPU checks of the boundary: the library loads and exports every symbol the header declares."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "saba.h")
LIB = os.path.join(ROOT, "paper_2410_14056_amd", "libsaba.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(saba_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ("saba_version", "saba_last_error", "saba_graph_create", "saba_graph_destroy",
                 "saba_graph_create_multi", "saba_graph_info", "saba_walks", "saba_aesc",
                 "saba_aesc_query", "saba_aesc_edge_stats", "saba_aesc_batch",
                 "saba_server_create", "saba_server_submit", "saba_server_wait",
                 "saba_server_stats", "saba_server_destroy", "saba_graph_lambda",
                 "saba_graph_get_config", "saba_graph_set_config", "saba_autotune_walks",
                 "saba_probe_random_reads"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (saba_\w+)", out))
    assert set(declared()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_reports_version():
    import paper_2410_14056_amd as saba
    lib = saba.load()
    assert lib.saba_version() == 5
    for name in saba.EXPORTS:
        assert hasattr(lib, name)
    assert set(saba.EXPORTS) == set(declared())


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2410_14056_amd import _binding
    with pytest.raises(RuntimeError):
        _binding._lib = None
        try:
            _binding.load(str(tmp_path / "missing.so"))
        finally:
            _binding._lib = None


def test_structs_match_header_layout():
    import ctypes
    from paper_2410_14056_amd import _binding as b
    # saba_walk_params: int64, int32, 3 x uint32, 2 x int32, pointer, 2 x int32, pointer -> 56
    assert ctypes.sizeof(b.WalkParams) == 56
    # saba_aesc_params: 3 doubles, 3 uint32, 5 int32, int64, 2 int32 -> 72 bytes
    assert ctypes.sizeof(b.AescParams) == 72
    assert ctypes.sizeof(b.Stats) == 80
    assert ctypes.sizeof(b.GraphInfo) == 48
    # saba_aesc_request: 2 x int32, params (72), pointer, int64, pointer -> 104 bytes
    assert ctypes.sizeof(b.AescRequest) == 104
    assert ctypes.sizeof(b.SpectrumParams) == 24
    assert ctypes.sizeof(b.SpectrumResult) == 40
    assert ctypes.sizeof(b.BatchOptions) == 16


def test_server_structs_match_the_c_compiler(tmp_path):
    """sizeof and field offsets as gcc lays the header's structs out, against the binding."""
    import ctypes
    from paper_2410_14056_amd import _binding as b
    checks = {
        "saba_server_options": (b.ServerOptions, ["mem_budget", "max_queued_edges", "arena_edges",
                                                  "lanes", "max_batch_sources"]),
        "saba_server_request": (b.ServerRequest, ["graph", "params", "edges", "q", "d_sc"]),
        "saba_server_result": (b.ServerResult, ["status", "batches", "instances", "queue_ms",
                                                "latency_ms"]),
        "saba_server_stats_t": (b.ServerStats, [f for f, _ in b.ServerStats._fields_]),
        "saba_aesc_request": (b.AescRequest, ["graph", "params", "d_edges", "q", "d_sc"]),
        "saba_aesc_params": (b.AescParams, ["eps", "delta", "seed", "tau_cap", "mem_budget",
                                            "omega", "reserved"]),
        "saba_spectrum_params": (b.SpectrumParams, ["graph", "omega", "max_iters", "seed", "tol"]),
        "saba_spectrum_result": (b.SpectrumResult, ["lambda_rest", "lambda_rest_bound",
                                                    "max_residual", "pairs", "iterations",
                                                    "converged"]),
        "saba_stats": (b.Stats, ["walks", "warnings", "kernel_ms", "count_ms"]),
        "saba_walk_params": (b.WalkParams, ["n_walks", "length", "mode", "d_sources", "sampler",
                                            "source_mode", "d_distinct"]),
        "saba_batch_options": (b.BatchOptions, ["mem_budget", "batch_sources", "time_kernels"]),
        "saba_lambda_params": (b.LambdaParams, ["graph", "max_iters", "tol", "seed"]),
        "saba_exec_config": (b.ExecConfig, ["walks_per_lane", "walk_blocks", "est_walk_blocks",
                                            "est_push_blocks", "walk_chunks",
                                            "est_walk_queue", "est_batch_streams"]),
        "saba_lambda_result": (b.LambdaResult, ["lambda_bound", "residual", "iterations",
                                                "converged"]),
        "saba_count_source": (b.CountSource, [f for f, _ in b.CountSource._fields_]),
        "saba_bouquet_choice": (b.BouquetChoice, [f for f, _ in b.BouquetChoice._fields_]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "saba.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                         text=True, check=True).stdout.splitlines())
    for cname, (cls, fields) in checks.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in fields:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_server_entry_points_reject_null_handles():
    """Host-side argument checks of the server calls (no device is touched)."""
    import ctypes
    import paper_2410_14056_amd as saba
    from paper_2410_14056_amd import _binding as b
    lib = saba.load()
    out = ctypes.c_void_p(123)
    assert lib.saba_server_create(None, None, ctypes.byref(out)) == -1
    assert out.value is None
    t = ctypes.c_uint64()
    assert lib.saba_server_submit(None, None, ctypes.byref(t)) == -1
    assert lib.saba_server_wait(None, ctypes.c_uint64(1), 0, None) == -1
    assert lib.saba_server_stats(None, None) == -1
    assert lib.saba_server_destroy(None) == 0
    assert b"NULL" in lib.saba_last_error() or lib.saba_last_error() == b""
