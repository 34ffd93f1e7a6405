"""CPU oracle for the random-bouquet walks and the TGT+ AESC estimator.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library: the C part (saba_oracle.c) is its own implementation of the hash,
the neighbour choice, the walk keys, the walks and the estimator, and
exact_sc.py computes exact spanning centrality.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "saba_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i32, u32, i64, f64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
        P = ctypes.c_void_p
        L.orc_murmur2.argtypes = [P, i32, u32]
        L.orc_murmur2.restype = u32
        L.orc_hash_words.argtypes = [P, i32, u32]
        L.orc_hash_words.restype = u32
        L.orc_hash2_batch.argtypes = [P, P, i64, u32, P]
        L.orc_hash2_batch.restype = None
        L.orc_choice.argtypes = [u32, u32]
        L.orc_choice.restype = u32
        L.orc_walk_key.argtypes = [u32, u32, u32, u32, ctypes.c_uint64, u32, u32, P, P]
        L.orc_walk_key.restype = None
        L.orc_walk_path.argtypes = [P, P, i32, i32, u32, u32, P]
        L.orc_walk_path.restype = i32
        L.orc_walks_histogram.argtypes = [P, P, i32, P, i64, i32, u32, u32, u32, i32, P, P, i32]
        L.orc_walks_histogram.restype = i32
        L.orc_distinct8.argtypes = [P, P, i32, P, i64, i32, u32, u32, u32, i32, i32, P]
        L.orc_distinct8.restype = i32
        L.orc_uniform_sources.argtypes = [P, i32, i64, u32, P]
        L.orc_uniform_sources.restype = i32
        L.orc_xorshift32.argtypes = [u32]
        L.orc_xorshift32.restype = u32
        L.orc_aesc.argtypes = [P, P, i32, f64, f64, f64, u32, u32, u32, i32, i32, i32, P, i64, P,
                               P, P, P, P, P, P, P, P, i32]
        L.orc_aesc.restype = i32
        L.orc_cconst_export.argtypes = [f64, f64, i64]
        L.orc_cconst_export.restype = f64
        L.orc_nwalks_export.argtypes = [i32, f64, i32, f64]
        L.orc_nwalks_export.restype = i64
        L.orc_tau_export.argtypes = [i32, i32, f64, f64, i32]
        L.orc_tau_export.restype = i32
        L.orc_source_counts.argtypes = [P, P, i32, i32, f64, f64, f64, u32, u32, u32, i32, i32,
                                        i32, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_source_counts.restype = i64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def murmur2(data: bytes, seed: int) -> int:
    buf = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)
    return int(lib().orc_murmur2(_p(buf), len(data), seed & 0xFFFFFFFF))


def hash_words(words, seed: int) -> int:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    return int(lib().orc_hash_words(_p(w), int(w.size), seed & 0xFFFFFFFF))


def hash2_batch(a, b, seed: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    out = np.zeros(a.size, dtype=np.uint32)
    lib().orc_hash2_batch(_p(a), _p(b), int(a.size), seed & 0xFFFFFFFF, _p(out))
    return out


def choice(u: int, d: int) -> int:
    return int(lib().orc_choice(u & 0xFFFFFFFF, d))


def walk_key(seed, a0, a1, a2, k, G=1, S=0):
    hi = ctypes.c_uint32()
    lo = ctypes.c_uint32()
    lib().orc_walk_key(seed, a0, a1, a2, k, G, S, ctypes.byref(hi), ctypes.byref(lo))
    return int(hi.value), int(lo.value)


def walk_path(g, start, L, key_hi, key_lo):
    path = np.zeros(L + 1, dtype=np.int32)
    rc = lib().orc_walk_path(_p(g.row_ptr), _p(g.col_idx), int(start), int(L), key_hi, key_lo,
                             _p(path))
    if rc != 0:
        raise ValueError("walk from an isolated vertex")
    return path


SAMPLER_KEYED, SAMPLER_KEYED_MOD, SAMPLER_STREAM_MOD, SAMPLER_LITERAL = 0, 1, 2, 3


def walks_histogram(g, sources, L, seed, G=1, S=0, nthreads=0, sampler=SAMPLER_KEYED):
    """Endpoint and visit histograms (int64[n] each) of the walks started at `sources`."""
    src = np.ascontiguousarray(sources, dtype=np.int32)
    ep = np.zeros(g.n, dtype=np.int64)
    vi = np.zeros(g.n, dtype=np.int64)
    rc = lib().orc_walks_histogram(_p(g.row_ptr), _p(g.col_idx), g.n, _p(src), int(src.size),
                                   int(L), seed, G, S, int(sampler), _p(ep), _p(vi),
                                   int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_walks_histogram failed ({rc})")
    return ep, vi


def uniform_sources(g, n_walks, seed):
    """Hashed uniform start vertices over the non-isolated vertices (int32[n_walks])."""
    out = np.zeros(int(n_walks), dtype=np.int32)
    rc = lib().orc_uniform_sources(_p(g.row_ptr), g.n, int(n_walks), seed & 0xFFFFFFFF, _p(out))
    if rc != 0:
        raise ValueError(f"orc_uniform_sources failed ({rc})")
    return out


def distinct8(g, sources, L, seed, G=1, S=0, sampler=SAMPLER_KEYED, order=1):
    """Branching statistics: hist[k] = (8-walk vector, position) pairs with k distinct
    vertices; order 0 = the given order, 1 = by start vertex then rank (bouquet order)."""
    src = np.ascontiguousarray(sources, dtype=np.int32)
    hist = np.zeros(9, dtype=np.int64)
    rc = lib().orc_distinct8(_p(g.row_ptr), _p(g.col_idx), g.n, _p(src), int(src.size), int(L),
                             seed, G, S, int(sampler), int(order), _p(hist))
    if rc != 0:
        raise ValueError(f"orc_distinct8 failed ({rc})")
    return hist


def xorshift32(x):
    return int(lib().orc_xorshift32(x & 0xFFFFFFFF))


def cconst(eps, delta, m):
    return float(lib().orc_cconst_export(eps, delta, m))


def nwalks(L, hmax, ds, c):
    return int(lib().orc_nwalks_export(L, hmax, ds, c))


def tau(ds, dt, lam, eps, tau_cap=1 << 20):
    return int(lib().orc_tau_export(ds, dt, lam, eps, tau_cap))


def aesc(g, eps, lam, seed, delta=0.01, G=1, S=0, tau_cap=1 << 20, tilde_tau_max=-1,
         push_all=False, query=None, nthreads=0):
    """TGT+ as read.  Returns (sc, per-directed-edge dict).

    sc is over canonical edges (u < v, lexicographic) when query is None, else over the
    query edges.  The dict holds tau, ttau, nreq, D, MC, vis0, vis1, g indexed by CSR
    position (entries of directed edges that were not needed are unspecified)."""
    nnz = g.nnz
    out = {
        "tau": np.full(nnz, -1, dtype=np.int32),
        "ttau": np.full(nnz, -1, dtype=np.int32),
        "nreq": np.zeros(nnz, dtype=np.int64),
        "D": np.zeros(nnz, dtype=np.float64),
        "MC": np.zeros(nnz, dtype=np.float64),
        "vis0": np.zeros(nnz, dtype=np.int64),
        "vis1": np.zeros(nnz, dtype=np.int64),
        "g": np.zeros(nnz, dtype=np.float64),
    }
    if query is None:
        qarr = None
        qn = 0
        sc = np.zeros(g.m, dtype=np.float64)
    else:
        qarr = np.ascontiguousarray(query, dtype=np.int32).reshape(-1, 2)
        qn = qarr.shape[0]
        sc = np.zeros(qn, dtype=np.float64)
    rc = lib().orc_aesc(_p(g.row_ptr), _p(g.col_idx), g.n, float(eps), float(delta), float(lam),
                        seed, G, S, int(tau_cap), int(tilde_tau_max), int(bool(push_all)),
                        None if qarr is None else _p(qarr), qn, _p(sc),
                        _p(out["tau"]), _p(out["ttau"]), _p(out["nreq"]), _p(out["D"]),
                        _p(out["MC"]), _p(out["vis0"]), _p(out["vis1"]), _p(out["g"]),
                        int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_aesc failed ({rc})")
    return sc, out


def source_counts(g, s, eps, lam, seed, delta=0.01, G=1, S=0, tau_cap=1 << 20, tilde_tau_max=-1,
                  push_all=False):
    """The integer visit counts of source s (Alg. 1's inner loop, per edge, side and support
    vertex).  Returns a dict:
      supp  int32[ns]   support of h_ttau, ascending;  h  float64[ns]  h_ttau there;
      hist  int64[d_s, 2, ns]  visits of the side-0 / side-1 walks of edge i (row order);
      MCh   float64[d_s]  sum over the support, ascending, of h * (c0 - c1);
      tau, ttau, nreq, D, MC, vis0, vis1, g  per edge of the row of s."""
    L = lib()
    args0 = (_p(g.row_ptr), _p(g.col_idx), g.n, int(s), float(eps), float(delta), float(lam),
             seed, G, S, int(tau_cap), int(tilde_tau_max), int(bool(push_all)))
    if not 0 <= int(s) < g.n:
        raise ValueError(f"source {s} out of range")
    d = int(g.row_ptr[s + 1] - g.row_ptr[s])
    out = {
        "tau": np.zeros(d, dtype=np.int32), "ttau": np.zeros(d, dtype=np.int32),
        "nreq": np.zeros(d, dtype=np.int64), "D": np.zeros(d, dtype=np.float64),
        "MC": np.zeros(d, dtype=np.float64), "vis0": np.zeros(d, dtype=np.int64),
        "vis1": np.zeros(d, dtype=np.int64), "g": np.zeros(d, dtype=np.float64),
    }
    edge_keys = ["tau", "ttau", "nreq", "D", "MC", "vis0", "vis1", "g"]
    ns = L.orc_source_counts(*args0, None, None, None, None, *[_p(out[k]) for k in edge_keys])
    if ns < 0:
        raise ValueError(f"orc_source_counts failed ({ns})")
    out.update({
        "supp": np.zeros(ns, dtype=np.int32), "h": np.zeros(ns, dtype=np.float64),
        "hist": np.zeros((d, 2, ns), dtype=np.int64), "MCh": np.zeros(d, dtype=np.float64),
    })
    keys = ["supp", "h", "hist", "MCh"] + edge_keys
    r = L.orc_source_counts(*args0, *[_p(out[k]) for k in keys])
    if r != ns:
        raise ValueError(f"orc_source_counts failed ({r})")
    return out

