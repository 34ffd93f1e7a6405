"""ctypes binding of libsaba.so: argument marshalling only.

Every computation happens in the HIP library; torch provides device memory and
streams.  Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsaba.so")

SABA_OK = 0
SABA_DEVICE_PTRS = 1
SABA_TRUSTED = 2
SABA_WALK_NAIVE = 0
SABA_WALK_BOUQUET = 1
SABA_WALK_NAIVE_LOG = 2
SABA_SAMPLER_KEYED = 0
SABA_SAMPLER_KEYED_MOD = 1
SABA_SAMPLER_STREAM_MOD = 2
SABA_SAMPLER_LITERAL = 3
SABA_SOURCES_EXPLICIT, SABA_SOURCES_UNIFORM = 0, 1

_ERRORS = {
    -1: "SABA_E_INVALID", -2: "SABA_E_NOMEM", -3: "SABA_E_HIP", -4: "SABA_E_GRAPH",
    -5: "SABA_E_DISCONNECTED", -6: "SABA_E_BIPARTITE", -7: "SABA_E_NOT_EDGE",
    -8: "SABA_E_OVERFLOW", -9: "SABA_E_NODEVICE", -10: "SABA_E_BUSY", -11: "SABA_E_TIMEOUT",
    -12: "SABA_E_CANCELLED",
}
SABA_E_INVALID = -1
SABA_E_OVERFLOW = -8
SABA_E_BUSY = -10
SABA_E_TIMEOUT = -11


class SabaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = _ERRORS.get(code, str(code))


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("m", ctypes.c_int64),
                ("d_max", ctypes.c_int32), ("n_isolated", ctypes.c_int32),
                ("connected", ctypes.c_int32), ("bipartite", ctypes.c_int32),
                ("ngraphs", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("walks", ctypes.c_int64), ("walk_steps", ctypes.c_int64),
                ("push_edge_visits", ctypes.c_int64), ("sources", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("max_tau", ctypes.c_int32),
                ("max_ttau", ctypes.c_int32), ("warnings", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("kernel_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("count_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class WalkParams(ctypes.Structure):
    _fields_ = [("n_walks", ctypes.c_int64), ("length", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("group", ctypes.c_uint32), ("spread", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32), ("d_sources", ctypes.c_void_p),
                ("sampler", ctypes.c_int32), ("source_mode", ctypes.c_int32),
                ("d_distinct", ctypes.c_void_p)]


class AescParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("delta", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("seed", ctypes.c_uint32), ("group", ctypes.c_uint32), ("spread", ctypes.c_uint32),
                ("tau_cap", ctypes.c_int32), ("tilde_tau_max", ctypes.c_int32),
                ("push_all", ctypes.c_int32), ("batch_sources", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32), ("mem_budget", ctypes.c_int64),
                ("omega", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class AescRequest(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("reserved", ctypes.c_int32), ("params", AescParams),
                ("d_edges", ctypes.c_void_p), ("q", ctypes.c_int64), ("d_sc", ctypes.c_void_p)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_int64), ("batch_sources", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_int64), ("max_queued_edges", ctypes.c_int64),
                ("arena_edges", ctypes.c_int64), ("lanes", ctypes.c_int32),
                ("max_batch_sources", ctypes.c_int32)]


class ServerRequest(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("reserved", ctypes.c_int32), ("params", AescParams),
                ("edges", ctypes.c_void_p), ("q", ctypes.c_int64), ("d_sc", ctypes.c_void_p)]


class ServerResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batches", ctypes.c_int32),
                ("instances", ctypes.c_int64), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "rejected", "completed", "failed", "batches", "instances", "walk_steps",
        "queued_edges", "queued_requests", "peak_queued_edges")] + [("busy_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LambdaParams(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("seed", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class LambdaResult(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lambda_bound", ctypes.c_double),
                ("lambda2", ctypes.c_double), ("lambdan", ctypes.c_double),
                ("residual", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


class SpectrumParams(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("omega", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("seed", ctypes.c_uint32), ("tol", ctypes.c_double)]


class SpectrumResult(ctypes.Structure):
    _fields_ = [("lambda_rest", ctypes.c_double), ("lambda_rest_bound", ctypes.c_double),
                ("max_residual", ctypes.c_double), ("pairs", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CountSource(ctypes.Structure):
    _fields_ = [("source", ctypes.c_int32), ("degree", ctypes.c_int32), ("ttau", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("support", ctypes.c_int64),
                ("supp_off", ctypes.c_int64), ("edge_off", ctypes.c_int64),
                ("hist_off", ctypes.c_int64)]


class BouquetChoice(ctypes.Structure):
    _fields_ = [("group", ctypes.c_uint32), ("spread", ctypes.c_uint32),
                ("distinct_mean", ctypes.c_double), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ExecConfig(ctypes.Structure):
    _fields_ = [("walks_per_lane", ctypes.c_int32), ("walk_blocks", ctypes.c_int32),
                ("est_walk_blocks", ctypes.c_int32), ("est_push_blocks", ctypes.c_int32),
                ("walk_chunks", ctypes.c_int32), ("est_walk_queue", ctypes.c_int32),
                ("est_batch_streams", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol the header declares
EXPORTS = ["saba_version", "saba_last_error", "saba_graph_create", "saba_graph_create_multi",
           "saba_graph_destroy", "saba_graph_info", "saba_walks", "saba_aesc", "saba_aesc_query",
           "saba_aesc_edge_stats", "saba_aesc_batch", "saba_server_create", "saba_server_submit",
           "saba_server_wait", "saba_server_stats", "saba_server_destroy", "saba_graph_lambda",
           "saba_graph_get_config", "saba_graph_set_config", "saba_autotune_walks",
           "saba_probe_random_reads", "saba_graph_spectrum", "saba_autotune_aesc",
           "saba_debug_fail_allocation", "saba_aesc_counts", "saba_walks_noalloc",
           "saba_autotune_bouquet", "saba_aesc_sources", "saba_aesc_combine"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsaba.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.saba_version.restype = ctypes.c_int
    L.saba_last_error.restype = ctypes.c_char_p
    L.saba_graph_create.argtypes = [P, P, i32, i64, u32, P, ctypes.POINTER(P)]
    L.saba_graph_create_multi.argtypes = [P, P, i32, i64, i32, P, u32, P, ctypes.POINTER(P)]
    L.saba_graph_destroy.argtypes = [P]
    L.saba_graph_info.argtypes = [P, ctypes.POINTER(GraphInfo)]
    L.saba_walks.argtypes = [P, ctypes.POINTER(WalkParams), P, P, ctypes.POINTER(Stats), P]
    L.saba_walks_noalloc.argtypes = [P, ctypes.POINTER(WalkParams), P, P, ctypes.POINTER(Stats),
                                     P]
    L.saba_aesc.argtypes = [P, ctypes.POINTER(AescParams), P, ctypes.POINTER(Stats), P]
    L.saba_aesc_query.argtypes = [P, ctypes.POINTER(AescParams), P, i64, P, ctypes.POINTER(Stats), P]
    L.saba_aesc_edge_stats.argtypes = [P, ctypes.POINTER(AescParams), P, P, P, P, P, P, P, P, P,
                                       ctypes.POINTER(Stats), P]
    L.saba_aesc_counts.argtypes = [P, ctypes.POINTER(AescParams), P, i32, P, P, P, P, P, P, P,
                                   P, P, P, ctypes.POINTER(Stats), P]
    L.saba_aesc_sources.argtypes = [P, ctypes.POINTER(AescParams), i32, i32, P,
                                    ctypes.POINTER(Stats), P]
    L.saba_aesc_combine.argtypes = [P, P, P, P]
    L.saba_aesc_batch.argtypes = [P, P, i32, ctypes.POINTER(BatchOptions), ctypes.POINTER(Stats), P]
    L.saba_server_create.argtypes = [P, ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]
    L.saba_server_submit.argtypes = [P, ctypes.POINTER(ServerRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.saba_server_wait.argtypes = [P, ctypes.c_uint64, i32, ctypes.POINTER(ServerResult)]
    L.saba_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.saba_server_destroy.argtypes = [P]
    L.saba_graph_lambda.argtypes = [P, ctypes.POINTER(LambdaParams), ctypes.POINTER(LambdaResult), P]
    L.saba_graph_get_config.argtypes = [P, ctypes.POINTER(ExecConfig)]
    L.saba_graph_set_config.argtypes = [P, ctypes.POINTER(ExecConfig)]
    L.saba_autotune_walks.argtypes = [P, ctypes.POINTER(WalkParams), ctypes.POINTER(ExecConfig), P]
    L.saba_autotune_bouquet.argtypes = [P, ctypes.POINTER(WalkParams), ctypes.c_double,
                                        ctypes.POINTER(BouquetChoice), P]
    L.saba_autotune_aesc.argtypes = [P, P, i32, ctypes.POINTER(BatchOptions),
                                     ctypes.POINTER(ExecConfig), P]
    L.saba_debug_fail_allocation.argtypes = [i32]
    L.saba_graph_spectrum.argtypes = [P, ctypes.POINTER(SpectrumParams), P, P,
                                      ctypes.POINTER(SpectrumResult), P]
    L.saba_probe_random_reads.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), P]
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_char_p if name == "saba_last_error" else ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != SABA_OK:
        msg = load().saba_last_error().decode(errors="replace")
        raise SabaError(rc, msg)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class SabaGraph:
    """A graph resident in device memory (saba_graph_create / saba_graph_destroy)."""

    def __init__(self, row_ptr, col_idx, trusted: bool = False, stream=None):
        lib = load()
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        n = rp.size - 1
        h = ctypes.c_void_p()
        flags = SABA_TRUSTED if trusted else 0
        _check(lib.saba_graph_create(rp.ctypes.data_as(ctypes.c_void_p),
                                     ci.ctypes.data_as(ctypes.c_void_p), n, ci.size, flags,
                                     _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.n = n
        self.nnz = ci.size
        self.offsets = [0, n]

    @classmethod
    def from_graph(cls, g, **kw):
        return cls(g.row_ptr, g.col_idx, **kw)

    @classmethod
    def from_graphs(cls, graphs, trusted: bool = False, stream=None):
        """Several graphs side by side in one handle (saba_graph_create_multi); graph k keeps
        its own vertex ids in estimator requests."""
        lib = load()
        offs = [0]
        rps, cis = [], []
        nnz = 0
        for g in graphs:
            rps.append(np.asarray(g.row_ptr[:-1], dtype=np.int64) + nnz)
            cis.append(np.asarray(g.col_idx, dtype=np.int64) + offs[-1])
            nnz += int(g.col_idx.size)
            offs.append(offs[-1] + int(g.row_ptr.size - 1))
        rp = np.ascontiguousarray(np.concatenate(rps + [np.array([nnz])]), dtype=np.int32)
        ci = np.ascontiguousarray(np.concatenate(cis) if cis else np.zeros(0), dtype=np.int32)
        off = np.ascontiguousarray(offs, dtype=np.int32)
        self = cls.__new__(cls)
        h = ctypes.c_void_p()
        flags = SABA_TRUSTED if trusted else 0
        _check(lib.saba_graph_create_multi(rp.ctypes.data_as(ctypes.c_void_p),
                                           ci.ctypes.data_as(ctypes.c_void_p), offs[-1], nnz,
                                           len(graphs), off.ctypes.data_as(ctypes.c_void_p), flags,
                                           _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.n = offs[-1]
        self.nnz = nnz
        self.offsets = list(offs)
        self.graph_m = [int(g.col_idx.size) // 2 for g in graphs]
        return self

    @property
    def handle(self):
        return self._h

    def n_of(self, index: int = 0) -> int:
        """Vertex count of graph `index` of the handle."""
        return self.offsets[index + 1] - self.offsets[index]

    def info(self) -> dict:
        out = GraphInfo()
        _check(load().saba_graph_info(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in GraphInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().saba_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class WalkResult:
    endpoint: torch.Tensor
    visits: torch.Tensor
    stats: dict
    distinct: torch.Tensor | None = None


def walks(graph: SabaGraph, sources: torch.Tensor | None, length: int, seed: int, group: int = 1,
          spread: int = 0, mode: int = SABA_WALK_BOUQUET, time_kernels: bool = False,
          endpoint: torch.Tensor | None = None, visits: torch.Tensor | None = None,
          stream=None, sampler: int = SABA_SAMPLER_KEYED,
          distinct: bool = False, n_walks: int | None = None,
          _entry: str = "saba_walks") -> WalkResult:
    """saba_walks: endpoint / visit histograms of the walks started at `sources` (int32,
    device), or, with sources=None, of n_walks walks from uniform sources the library draws
    (SABA_SOURCES_UNIFORM); with distinct=True also the branching statistics (int64 [9])."""
    if sources is None:
        assert n_walks is not None and n_walks >= 0
        nw, sptr, smode, dev = int(n_walks), None, SABA_SOURCES_UNIFORM, torch.device("cuda")
    else:
        assert sources.is_cuda and sources.dtype == torch.int32 and sources.is_contiguous()
        nw, sptr, smode, dev = sources.numel(), sources.data_ptr(), SABA_SOURCES_EXPLICIT, sources.device
    if endpoint is None:
        endpoint = torch.empty(graph.n, dtype=torch.int64, device=dev)
    if visits is None:
        visits = torch.empty(graph.n, dtype=torch.int64, device=dev)
    dist = torch.empty(9, dtype=torch.int64, device=dev) if distinct else None
    p = WalkParams(nw, int(length), seed & 0xFFFFFFFF, int(group), int(spread),
                   int(mode), int(bool(time_kernels)), sptr, int(sampler), smode,
                   None if dist is None else dist.data_ptr())
    st = Stats()
    _check(getattr(load(), _entry)(graph.handle, ctypes.byref(p), _ptr(endpoint), _ptr(visits),
                                   ctypes.byref(st), _stream_ptr(stream)))
    return WalkResult(endpoint, visits, st.as_dict(), dist)


def walks_noalloc(graph: SabaGraph, sources: torch.Tensor, length: int, seed: int,
                  endpoint: torch.Tensor, visits: torch.Tensor, group: int = 1, spread: int = 0,
                  stream=None, sampler: int = SABA_SAMPLER_KEYED) -> WalkResult:
    """saba_walks_noalloc: saba_walks in bouquet mode from explicit sources, with the caller's
    output tensors and the library's fixed device scratch (no allocation in the call)."""
    return walks(graph, sources, length, seed, group=group, spread=spread,
                 mode=SABA_WALK_BOUQUET, endpoint=endpoint, visits=visits, stream=stream,
                 sampler=sampler, _entry="saba_walks_noalloc")


def probe_random_reads(log2_records: int = 26, steps: int = 256, stream=None) -> dict:
    """saba_probe_random_reads: dependent random 16-byte reads per second."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check(load().saba_probe_random_reads(int(log2_records), int(steps), ctypes.byref(rate),
                                          ctypes.byref(ms), _stream_ptr(stream)))
    return {"reads_per_s": rate.value, "ms": ms.value, "log2_records": log2_records,
            "steps": steps}


def get_config(graph: SabaGraph) -> dict:
    c = ExecConfig()
    _check(load().saba_graph_get_config(graph.handle, ctypes.byref(c)))
    return c.as_dict()


def set_config(graph: SabaGraph, walks_per_lane: int = 0, walk_blocks: int = 0,
               est_walk_blocks: int = 0, est_push_blocks: int = 0, walk_chunks: int = 0,
               est_walk_queue: int = 0, est_batch_streams: int = 0):
    """saba_graph_set_config: execution knobs of the handle (0 = default); never changes a
    result."""
    c = ExecConfig(int(walks_per_lane), int(walk_blocks), int(est_walk_blocks),
                   int(est_push_blocks), int(walk_chunks), int(est_walk_queue),
                   int(est_batch_streams))
    _check(load().saba_graph_set_config(graph.handle, ctypes.byref(c)))


def autotune_bouquet(graph: SabaGraph, sources: torch.Tensor, length: int, seed: int,
                     min_distinct: float, stream=None) -> dict:
    """saba_autotune_bouquet: the fastest key schedule (G, S) on this sample whose walks keep at
    least min_distinct distinct vertices per 8-walk vector on average (not kept in the handle:
    the schedule changes which walks are drawn)."""
    assert sources.is_cuda and sources.dtype == torch.int32 and sources.is_contiguous()
    p = WalkParams(sources.numel(), int(length), seed & 0xFFFFFFFF, 1, 0, SABA_WALK_BOUQUET, 0,
                   sources.data_ptr(), SABA_SAMPLER_KEYED, SABA_SOURCES_EXPLICIT, None)
    b = BouquetChoice()
    _check(load().saba_autotune_bouquet(graph.handle, ctypes.byref(p), float(min_distinct),
                                        ctypes.byref(b), _stream_ptr(stream)))
    return b.as_dict()


def autotune_walks(graph: SabaGraph, sources: torch.Tensor, length: int, seed: int,
                   group: int = 1, spread: int = 0, stream=None) -> dict:
    """saba_autotune_walks: times the bouquet walk kernel on this sample under each candidate
    setting, keeps the fastest in the handle and returns it."""
    assert sources.is_cuda and sources.dtype == torch.int32 and sources.is_contiguous()
    p = WalkParams(sources.numel(), int(length), seed & 0xFFFFFFFF, int(group), int(spread),
                   SABA_WALK_BOUQUET, 1, sources.data_ptr(), 0, 0, None)
    c = ExecConfig()
    _check(load().saba_autotune_walks(graph.handle, ctypes.byref(p), ctypes.byref(c),
                                      _stream_ptr(stream)))
    return c.as_dict()


def graph_lambda(graph: SabaGraph, index: int = 0, max_iters: int = 0, tol: float = 0.0,
                 seed: int = 1, stream=None) -> dict:
    """saba_graph_lambda: lambda of graph `index` of the handle by Lanczos on the device."""
    p = LambdaParams(int(index), int(max_iters), float(tol), seed & 0xFFFFFFFF, 0)
    r = LambdaResult()
    _check(load().saba_graph_lambda(graph.handle, ctypes.byref(p), ctypes.byref(r),
                                    _stream_ptr(stream)))
    return r.as_dict()


def graph_spectrum(graph: SabaGraph, omega: int, index: int = 0, max_iters: int = 0,
                   tol: float = 0.0, seed: int = 1, vectors: bool = True, stream=None) -> dict:
    """saba_graph_spectrum: the omega nontrivial eigenpairs of D^-1/2 A D^-1/2 of largest
    |theta| for graph `index` of the handle, and the radius of the rest of the spectrum.
    Returns the result fields plus "values" (numpy, by decreasing |theta|) and "vectors"
    (a [omega, n] float64 CUDA tensor of unit eigenvectors, or None)."""
    import numpy as np
    n = graph.n_of(index)
    p = SpectrumParams(int(index), int(omega), int(max_iters), seed & 0xFFFFFFFF, float(tol))
    vals = (ctypes.c_double * max(int(omega), 1))()
    vec = None
    if vectors and omega > 0:
        vec = torch.empty((int(omega), n), dtype=torch.float64, device="cuda")
    r = SpectrumResult()
    _check(load().saba_graph_spectrum(graph.handle, ctypes.byref(p), vals,
                                      vec.data_ptr() if vec is not None else None,
                                      ctypes.byref(r), _stream_ptr(stream)))
    d = r.as_dict()
    d["values"] = np.array(vals[:max(int(omega), 0)], dtype=np.float64)
    d["vectors"] = vec
    return d


def fail_allocation(n: int):
    """saba_debug_fail_allocation: the n-th scratch allocation from now on fails (0 disarms)."""
    _check(load().saba_debug_fail_allocation(int(n)))


def _aesc_params(eps, lam, seed, delta=0.01, group=1, spread=0, tau_cap=0, tilde_tau_max=-1,
                 push_all=False, batch_sources=0, time_kernels=False, mem_budget=0, omega=0):
    return AescParams(float(eps), float(delta), float(lam), seed & 0xFFFFFFFF, int(group),
                      int(spread), int(tau_cap), int(tilde_tau_max), int(bool(push_all)),
                      int(batch_sources), int(bool(time_kernels)), int(mem_budget), int(omega), 0)


def aesc(graph: SabaGraph, eps: float, lam: float, seed: int, device="cuda", stream=None, **kw):
    """saba_aesc: spanning-centrality estimates of all edges in canonical order (double, device)."""
    p = _aesc_params(eps, lam, seed, **kw)
    sc = torch.empty(graph.nnz // 2, dtype=torch.float64, device=device)
    st = Stats()
    _check(load().saba_aesc(graph.handle, ctypes.byref(p), _ptr(sc), ctypes.byref(st),
                            _stream_ptr(stream)))
    return sc, st.as_dict()


def aesc_query(graph: SabaGraph, edges: torch.Tensor, eps: float, lam: float, seed: int,
               stream=None, **kw):
    """saba_aesc_query: estimates of the query edges (int32 [q, 2], device)."""
    assert edges.is_cuda and edges.dtype == torch.int32 and edges.is_contiguous()
    q = edges.numel() // 2
    p = _aesc_params(eps, lam, seed, **kw)
    sc = torch.empty(q, dtype=torch.float64, device=edges.device)
    st = Stats()
    _check(load().saba_aesc_query(graph.handle, ctypes.byref(p), _ptr(edges), q, _ptr(sc),
                                  ctypes.byref(st), _stream_ptr(stream)))
    return sc, st.as_dict()


def aesc_edge_stats(graph: SabaGraph, eps: float, lam: float, seed: int, device="cuda",
                    stream=None, **kw):
    """saba_aesc_edge_stats: per-directed-edge internals plus the all-edges estimates."""
    p = _aesc_params(eps, lam, seed, **kw)
    nnz = graph.nnz
    out = {
        "sc": torch.empty(nnz // 2, dtype=torch.float64, device=device),
        "tau": torch.empty(nnz, dtype=torch.int32, device=device),
        "ttau": torch.empty(nnz, dtype=torch.int32, device=device),
        "nreq": torch.empty(nnz, dtype=torch.int64, device=device),
        "D": torch.empty(nnz, dtype=torch.float64, device=device),
        "MC": torch.empty(nnz, dtype=torch.float64, device=device),
        "vis0": torch.empty(nnz, dtype=torch.int64, device=device),
        "vis1": torch.empty(nnz, dtype=torch.int64, device=device),
        "g": torch.empty(nnz, dtype=torch.float64, device=device),
    }
    st = Stats()
    _check(load().saba_aesc_edge_stats(
        graph.handle, ctypes.byref(p), _ptr(out["sc"]), _ptr(out["tau"]), _ptr(out["ttau"]),
        _ptr(out["nreq"]), _ptr(out["D"]), _ptr(out["MC"]), _ptr(out["vis0"]), _ptr(out["vis1"]),
        _ptr(out["g"]), ctypes.byref(st), _stream_ptr(stream)))
    return out, st.as_dict()


def aesc_sources(graph: SabaGraph, g: torch.Tensor, src_begin: int, src_end: int, eps: float,
                 lam: float, seed: int, stream=None, **kw) -> dict:
    """saba_aesc_sources: directed estimates of the edges out of sources [src_begin, src_end),
    written into g (float64 [nnz], device) at their CSR positions; returns the stats."""
    assert g.is_cuda and g.dtype == torch.float64 and g.numel() == graph.nnz
    p = _aesc_params(eps, lam, seed, **kw)
    st = Stats()
    _check(load().saba_aesc_sources(graph.handle, ctypes.byref(p), int(src_begin), int(src_end),
                                    _ptr(g), ctypes.byref(st), _stream_ptr(stream)))
    return st.as_dict()


def aesc_combine(graph: SabaGraph, g: torch.Tensor, stream=None) -> torch.Tensor:
    """saba_aesc_combine: SC of all edges in canonical order from directed estimates g."""
    assert g.is_cuda and g.dtype == torch.float64 and g.numel() == graph.nnz
    sc = torch.empty(graph.nnz // 2, dtype=torch.float64, device=g.device)
    _check(load().saba_aesc_combine(graph.handle, _ptr(g), _ptr(sc), _stream_ptr(stream)))
    return sc


def aesc_counts(graph: SabaGraph, sources, eps: float, lam: float, seed: int, device="cuda",
                stream=None, histograms: bool = True, **kw):
    """saba_aesc_counts: the integer visit counts of the walk pairs of the given sources.

    Returns (per-source list, dict of device tensors, stats).  Each list entry is a dict with
    source, degree, ttau, support, edge_off and, with histograms, the entries supp/h (support,
    h_ttau there) and hist (int64 [degree, 2, support]) as views into the packed tensors; the
    dict holds the packed supp, h, hist and the per-edge tau, nreq, D, MC, vis0, vis1, g
    (entry edge_off + i).  histograms=False stops after the sizing call (per-edge outputs
    and the layout only)."""
    L = load()
    p = _aesc_params(eps, lam, seed, **kw)
    K = len(sources)
    lay = (CountSource * K)()
    for k, v in enumerate(sources):
        lay[k].source = int(v)
    st = Stats()
    s = _stream_ptr(stream)
    _check(L.saba_aesc_counts(graph.handle, ctypes.byref(p), lay, K, None, None, None, None,
                              None, None, None, None, None, None, ctypes.byref(st), s))
    last = lay[K - 1]
    ns = last.supp_off + last.support
    ne = last.edge_off + last.degree
    nh = last.hist_off + 2 * last.degree * last.support
    out = {
        "tau": torch.empty(ne, dtype=torch.int32, device=device),
        "nreq": torch.empty(ne, dtype=torch.int64, device=device),
        "D": torch.empty(ne, dtype=torch.float64, device=device),
        "MC": torch.empty(ne, dtype=torch.float64, device=device),
        "vis0": torch.empty(ne, dtype=torch.int64, device=device),
        "vis1": torch.empty(ne, dtype=torch.int64, device=device),
        "g": torch.empty(ne, dtype=torch.float64, device=device),
    }
    edge_ptrs = [_ptr(out[k]) for k in ("tau", "nreq", "D", "MC", "vis0", "vis1", "g")]
    if histograms:
        out["supp"] = torch.empty(ns, dtype=torch.int32, device=device)
        out["h"] = torch.empty(ns, dtype=torch.float64, device=device)
        out["hist"] = torch.empty(nh, dtype=torch.int64, device=device)
        _check(L.saba_aesc_counts(graph.handle, ctypes.byref(p), lay, K, _ptr(out["supp"]),
                                  _ptr(out["h"]), _ptr(out["hist"]), *edge_ptrs,
                                  ctypes.byref(st), s))
    else:
        _check(L.saba_aesc_counts(graph.handle, ctypes.byref(p), lay, K, None, None, None,
                                  *edge_ptrs, ctypes.byref(st), s))
    per = []
    for k in range(K):
        c = lay[k]
        d, z = c.degree, c.support
        e = {"source": c.source, "degree": d, "ttau": c.ttau, "support": z,
             "edge_off": c.edge_off}
        if histograms:
            e["supp"] = out["supp"][c.supp_off:c.supp_off + z]
            e["h"] = out["h"][c.supp_off:c.supp_off + z]
            e["hist"] = out["hist"][c.hist_off:c.hist_off + 2 * d * z].view(d, 2, z)
        per.append(e)
    return per, out, st.as_dict()


def aesc_batch(graph: SabaGraph, requests, mem_budget: int = 0, batch_sources: int = 0,
               time_kernels: bool = False, device="cuda", stream=None):
    """saba_aesc_batch.  Each request is a dict with keys graph (index), eps, lam, seed and
    optionally edges (int32 [q, 2] device tensor of the graph's own ids; omitted = all edges),
    m (edge count of the graph, needed for all-edges requests) and the estimator keywords of
    aesc().  Returns (list of result tensors, stats)."""
    lib = load()
    arr, outs, keep = _batch_requests(requests, device)
    opt = BatchOptions(int(mem_budget), int(batch_sources), int(bool(time_kernels)))
    st = Stats()
    _check(lib.saba_aesc_batch(graph.handle, ctypes.cast(arr, ctypes.c_void_p), len(requests),
                               ctypes.byref(opt), ctypes.byref(st), _stream_ptr(stream)))
    return outs, st.as_dict()


def autotune_aesc(graph: SabaGraph, requests, mem_budget: int = 0, batch_sources: int = 0,
                  device="cuda", stream=None) -> dict:
    """saba_autotune_aesc: times the estimator on the sample `requests` (as for aesc_batch)
    under each candidate grid, keeps the fastest in the handle and returns it."""
    arr, outs, keep = _batch_requests(requests, device)
    opt = BatchOptions(int(mem_budget), int(batch_sources), 1)
    c = ExecConfig()
    _check(load().saba_autotune_aesc(graph.handle, ctypes.cast(arr, ctypes.c_void_p),
                                     len(requests), ctypes.byref(opt), ctypes.byref(c),
                                     _stream_ptr(stream)))
    return c.as_dict()


def _batch_requests(requests, device):
    """The AescRequest array of aesc_batch's request dicts, the result tensors and the edge
    tensors that must stay alive during the call."""
    arr = (AescRequest * max(1, len(requests)))()
    outs = []
    keep = []
    for i, r in enumerate(requests):
        kw = {k: v for k, v in r.items() if k not in ("graph", "eps", "lam", "seed", "edges", "m")}
        p = _aesc_params(r["eps"], r["lam"], r["seed"], **kw)
        edges = r.get("edges")
        if edges is None:
            q = -1
            out = torch.empty(int(r["m"]), dtype=torch.float64, device=device)
            eptr = None
        else:
            assert edges.is_cuda and edges.dtype == torch.int32 and edges.is_contiguous()
            q = edges.numel() // 2
            out = torch.empty(q, dtype=torch.float64, device=edges.device)
            eptr = edges.data_ptr()
            keep.append(edges)
        arr[i].graph = int(r.get("graph", 0))
        arr[i].params = p
        arr[i].d_edges = eptr
        arr[i].q = q
        arr[i].d_sc = out.data_ptr() if out.numel() else None
        outs.append(out)
    return arr, outs, keep


class SabaServer:
    """Query server over a resident handle (saba_server_*): requests are admitted as they
    arrive and their sources run in shared batches on `lanes` concurrent streams."""

    def __init__(self, graph: SabaGraph, lanes: int = 0, mem_budget: int = 0,
                 max_queued_edges: int = 0, arena_edges: int = 0, max_batch_sources: int = 0,
                 device="cuda"):
        lib = load()
        self.graph = graph  # the handle must outlive the server
        self.device = device
        opt = ServerOptions(int(mem_budget), int(max_queued_edges), int(arena_edges), int(lanes),
                            int(max_batch_sources))
        h = ctypes.c_void_p()
        _check(lib.saba_server_create(graph.handle, ctypes.byref(opt), ctypes.byref(h)))
        self.handle = h
        self._out = {}

    def submit(self, graph: int, edges, eps: float, lam: float, seed: int, **kw) -> int:
        """Submit query pairs (host int32 array [q, 2] of the graph's own ids); returns a
        ticket.  Raises SabaError (name SABA_E_BUSY when the admission queue is full)."""
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        q = e.shape[0]
        out = torch.empty(q, dtype=torch.float64, device=self.device)
        # the block may have been freed with work still pending on torch's stream; the
        # server writes it from its own stream
        torch.cuda.current_stream(out.device).synchronize()
        r = ServerRequest()
        r.graph = int(graph)
        r.params = _aesc_params(eps, lam, seed, **kw)
        r.edges = e.ctypes.data if q else None
        r.q = q
        r.d_sc = out.data_ptr() if q else None
        t = ctypes.c_uint64()
        _check(load().saba_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._out[t.value] = out
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(results tensor, result dict) once the request has finished; None on time-out."""
        res = ServerResult()
        rc = load().saba_server_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_ms),
                                     ctypes.byref(res))
        if rc == SABA_E_TIMEOUT:
            return None
        out = self._out.pop(ticket, None)
        _check(rc)
        return out, res.as_dict()

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().saba_server_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().saba_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self._out.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
