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
                 "saba_aesc_query", "saba_aesc_edge_stats", "saba_aesc_batch"):
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
    assert lib.saba_version() == 1
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
    # saba_walk_params: int64, int32, 3 x uint32, 2 x int32, pointer -> 40 bytes
    assert ctypes.sizeof(b.WalkParams) == 40
    # saba_aesc_params: 3 doubles, 3 uint32, 5 int32, int64 -> 64 bytes
    assert ctypes.sizeof(b.AescParams) == 64
    assert ctypes.sizeof(b.Stats) == 80
    assert ctypes.sizeof(b.GraphInfo) == 48
    # saba_aesc_request: 2 x int32, params (64), pointer, int64, pointer -> 96 bytes
    assert ctypes.sizeof(b.AescRequest) == 96
    assert ctypes.sizeof(b.BatchOptions) == 16
