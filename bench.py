#!/usr/bin/env python3
"""Benchmark of the random-bouquet walk generator on one MI355X.

Workload: R-MAT scale 20, edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), seed 1,
symmetrised and deduplicated, int32 CSR; 2^24 walks of 64 steps from uniform
non-isolated sources (seed 1), hash-keyed neighbour choice, bouquet execution.
A step is one saba_walks call: source bucketing, key set-up, the walks and the
int64 endpoint / visit histograms (Sec. 5.4's synthetic benchmark).

Prints one JSON line.  `roofline` prices the walk kernel at 3 random 64-byte
sectors per walk step (vertex record, adjacency entry, visit counter) against
the 8 TB/s HBM peak; `cpu_baseline` times the CPU oracle on a bounded slice of
the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-steps/s and AESC edges/s at ε=0.1 (1 GPU); p50/p99 query latency"
BYTES_PER_STEP = 192  # 3 random 64 B sectors: vertex record, adjacency entry, visit counter
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "walk_bouquet_rmat20_counters.json")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("saba_internal.hpp", "walks.hip"):
        with open(os.path.join(ROOT, "paper_2410_14056_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(mode: str, walks: int, steps: int):
    """HBM bytes per launch of the walk kernel from committed rocprofv3 counters, if they
    were taken on the current kernel source; else None."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except OSError:
        return None
    rec = c.get(mode)
    if not rec or c.get("kernel_source_sha") != kernel_source_sha():
        return None
    if rec.get("walks") != walks or rec.get("length") != steps:
        return None
    return float(rec["hbm_bytes_per_dispatch"])


def cpu_baseline(g, L, seed, target_s=12.0):
    """The oracle as it stands, on all host cores, on a slice of the walks."""
    import numpy as np
    import graphgen
    import oracle
    cores = os.cpu_count() or 1
    nw = 1 << 18
    src = graphgen.uniform_sources(g, nw, seed + 1000)
    t0 = time.perf_counter()
    oracle.walks_histogram(g, src, L, seed, nthreads=cores)
    dt = time.perf_counter() - t0
    if dt < target_s / 4:
        nw = int(min(1 << 24, nw * max(1.0, target_s / max(dt, 1e-3))))
        src = graphgen.uniform_sources(g, nw, seed + 1000)
        t0 = time.perf_counter()
        oracle.walks_histogram(g, src, L, seed, nthreads=cores)
        dt = time.perf_counter() - t0
    return {"value": nw * L / dt, "unit": "walk-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{nw} walks x {L} steps from uniform sources on the same graph "
                      f"({dt:.1f} s wall, OpenMP over walks)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["bouquet", "naive"], default="bouquet")
    ap.add_argument("--group", type=int, default=1)
    ap.add_argument("--spread", type=int, default=0)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--walks-log2", type=int, default=24)
    ap.add_argument("--length", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the walk path shards by splitting the walk range, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import graphgen
    import paper_2410_14056_amd as saba

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    saba.load()
    t_gen = time.perf_counter()
    g = graphgen.rmat(args.scale, 16, 0.57, 0.19, 0.19, 1)
    W, L, seed = 1 << args.walks_log2, args.length, 1
    src_np = graphgen.uniform_sources(g, W, 1)
    t_gen = time.perf_counter() - t_gen
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    src = torch.from_numpy(src_np).cuda()
    mode = saba.SABA_WALK_BOUQUET if args.mode == "bouquet" else saba.SABA_WALK_NAIVE
    ep = torch.empty(g.n, dtype=torch.int64, device="cuda")
    vi = torch.empty(g.n, dtype=torch.int64, device="cuda")

    def step():
        return saba.walks(sg, src, L, seed, group=args.group, spread=args.spread, mode=mode,
                          time_kernels=True, endpoint=ep, visits=vi)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        kms.append(r.stats["kernel_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert int(vi.sum().item()) == W * L and int(ep.sum().item()) == W

    steps_total = W * L * args.steps
    value = steps_total / dt
    k_ms = float(np.mean(kms))
    achieved = BYTES_PER_STEP * W * L / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.mode, W, L)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"rmat{args.scale}_ef16_walks_2^{args.walks_log2}x{L}",
            "graph": f"R-MAT scale {args.scale}, edge factor 16, a=0.57 b=0.19 c=0.19, seed 1, "
                     "symmetrised, deduplicated, int32 CSR",
            "n": g.n, "nnz": g.nnz, "walks": W, "length": L, "sources": "uniform non-isolated, seed 1",
            "mode": args.mode, "group": args.group, "spread": args.spread,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "walk_bouquet_kernel" if mode == saba.SABA_WALK_BOUQUET else "walk_naive_kernel",
            "kernel_ms": k_ms,
            "bytes_per_step": BYTES_PER_STEP,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, L, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
