#!/usr/bin/env python3
"""Benchmark of the random-bouquet walk generator and the TGT+ estimator on one MI355X.

Headline (`value`): walk-steps/s.  Workload: R-MAT scale 20, edge factor 16,
(a, b, c) = (0.57, 0.19, 0.19), seed 1, symmetrised and deduplicated, int32 CSR;
2^24 walks of 64 steps from uniform non-isolated sources (seed 1), hash-keyed
neighbour choice, bouquet execution, G = 1.  A step is one saba_walks call:
source bucketing, key set-up, the walks and the int64 endpoint / visit
histograms (the synthetic benchmark of Sec. 5.4).

Secondary legs of the default run:
  walks_side_by_side  naive generation and grouped bouquets (G = 64, S = 20) on the same starts;
  er2000              all edges of ER n = 2000, m = 8000 at eps = 0.3 (latency);
  aesc                edges/s of the TGT+ estimator at eps = 0.1 on the Chung-Lu graph
                      n = 10^6, average degree 10, exponent 2.5, seed 1, largest component,
                      over a seeded 1% sample of its edges (saba_aesc_query; the paper
                      estimates its largest graph the same way, from a fixed 5% of the edges);
  aesc_all_edges      all edges of the same graph (sum of the estimates against n - 1);
  serve               16 resident graphs, Poisson requests: an offered load with backpressure
                      and a sustained load at 70% of the served capacity; p50_ms / p99_ms are
                      the sustained phase's.

`roofline` prices the dominant kernel with its algorithmic bytes (64 B sectors), with the
128 B line the L2 fetches and the measured random-read ceiling beside it; `cpu_baseline`
times the CPU oracle on a bounded slice of the same workload.
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
HBM_PEAK_GBS = 8000.0
# walk kernel, algorithmic bytes per step in 64 B sectors (the HBM3E access unit): one random
# sector for the 16-byte walk entry of the next vertex, plus the 4 B coalesced visit-log store
WALK_KERNEL_BYTES_PER_STEP = 68
# the same step priced at what gfx950 moves for it: its L2 fetches whole 128 B lines for every
# read (the request-size counters TCC_EA0_RDREQ_{32B,64B,128B} show only 128 B read requests,
# for a plain copy and for the random walk-entry reads alike)
WALK_KERNEL_BYTES_PER_STEP_LINE = 132
# naive walk kernel: the vertex record and the adjacency entry (two random sectors) and a
# random 8 B counter update (a third sector) per step
WALK_STEP_BYTES = 192
# estimator walk kernel: one random 64 B sector for the walk entry of the next vertex per step
# (the support bitmaps, and the h values of frequently hit vertices, are meant to stay cached);
# and the same step at the 128 B line the L2 fetches
AESC_STEP_BYTES = 64
AESC_STEP_BYTES_LINE = 128
TRAFFIC_BASIS = ("bytes the L2 requested from the memory fabric (FETCH_SIZE x 2.0 + WRITE_SIZE, "
                 "each scaled by a plain 1 GiB copy), served by HBM or the 256 MB Infinity Cache")
COUNTERS = os.path.join(ROOT, "profiles", "walk_bouquet_log_kernel_rmat20_counters.json")


EST_COUNTERS = os.path.join(ROOT, "profiles", "mc_walk_staged_kernel_chunglu1m_query1pct_counters.json")


def kernel_source_sha(files=("saba_internal.hpp", "walks.hip")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2410_14056_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def estimator_traffic(walk_steps: int, launches: int, kernel: str):
    """Fabric bytes per launch of the walk-pair kernel from the committed counter runs, if they
    were taken on the current estimator source with the same kernel and query (same walk
    steps); else None.  The runs give bytes per walk step; a launch averages walk_steps /
    launches steps."""
    try:
        with open(EST_COUNTERS) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_sha") != kernel_source_sha(("saba_internal.hpp", "estimator.hpp",
                                                        "aesc.hip")):
        return None
    if c.get("kernel") != kernel:
        return None
    if c.get("walk_steps") != walk_steps or launches <= 0:
        return None
    return float(c["fabric_bytes_per_step"]) * walk_steps / launches


def measured_traffic(walks: int, steps: int, steps_per_launch: int):
    """Fabric bytes per launch of the walk kernel from committed rocprofv3 counter runs, if
    they were taken on the current kernel source with this workload; else None.  The runs give
    bytes per walk step (one line per step whatever the chunk size)."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_sha") != kernel_source_sha():
        return None
    if c.get("walks") != walks or c.get("length") != steps:
        return None
    return float(c["fabric_bytes_per_step"]) * steps_per_launch


def host_threads() -> int:
    """Threads for the oracle's CPU baselines: the host's CPU share as OMP_NUM_THREADS states
    it, else the visible cores."""
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return os.cpu_count() or 1


def walks_cpu_baseline(g, L, seed, target_s=12.0):
    """The oracle as it stands, on all host cores, on a slice of the walks."""
    import graphgen
    import oracle
    cores = host_threads()
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


def bench_walks(args, saba, torch, np):
    import graphgen
    g = graphgen.rmat(args.scale, 16, 0.57, 0.19, 0.19, 1)
    W, L, seed = 1 << args.walks_log2, args.length, 1
    src_np = graphgen.uniform_sources(g, W, 1)
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    src = torch.from_numpy(src_np).cuda()
    mode = saba.SABA_WALK_BOUQUET if args.mode == "bouquet" else saba.SABA_WALK_NAIVE
    ep = torch.empty(g.n, dtype=torch.int64, device="cuda")
    vi = torch.empty(g.n, dtype=torch.int64, device="cuda")

    tuned = None
    if mode == saba.SABA_WALK_BOUQUET:
        # one-time set-up outside the timed steps: pick the execution knobs on this workload
        tuned = saba.autotune_walks(sg, src, L, seed, group=args.group, spread=args.spread)

    def step():
        return saba.walks(sg, src, L, seed, group=args.group, spread=args.spread, mode=mode,
                          time_kernels=True, endpoint=ep, visits=vi)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kms, cms, tms = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        kms.append(r.stats["kernel_ms"])
        cms.append(r.stats["count_ms"])
        tms.append(r.stats["total_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert int(vi.sum().item()) == W * L and int(ep.sum().item()) == W
    # measured ceiling of dependent random 16-byte reads (one per walk step), outside the timing
    probe = saba.probe_random_reads(26, 256) if mode == saba.SABA_WALK_BOUQUET else None
    k_ms = float(np.mean(kms))
    call_ms = float(np.mean(tms))
    chunks = int(r.stats["batches"])  # walk-kernel launches per call (visit-log chunks)
    per_launch_steps = W * L // chunks
    bouquet = mode == saba.SABA_WALK_BOUQUET
    kbytes = WALK_KERNEL_BYTES_PER_STEP if bouquet else WALK_STEP_BYTES
    launch_s = k_ms / chunks * 1e-3
    achieved = kbytes * per_launch_steps / launch_s / 1e9
    line = WALK_KERNEL_BYTES_PER_STEP_LINE * per_launch_steps / launch_s / 1e9
    side = side_walks(args, saba, torch, np, sg, src, L, seed, ep, vi) if args.workload == "all" else None
    return g, {
        "value": W * L * args.steps / dt,
        "ms_per_step": dt * 1e3 / args.steps,
        "config": {
            "workload": f"rmat{args.scale}_ef16_walks_2^{args.walks_log2}x{L}",
            "graph": f"R-MAT scale {args.scale}, edge factor 16, a=0.57 b=0.19 c=0.19, seed 1, "
                     "symmetrised, deduplicated, int32 CSR",
            "n": g.n, "nnz": g.nnz, "walks": W, "length": L,
            "sources": "uniform non-isolated, seed 1",
            "mode": args.mode, "group": args.group, "spread": args.spread,
            "tuned": tuned,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(W, L, per_launch_steps) if bouquet else None,
            "traffic_basis": TRAFFIC_BASIS,
            "kernel": "walk_bouquet_log_kernel" if bouquet else "walk_naive_kernel",
            "kernel_ms_per_launch": k_ms / chunks,
            "launches_per_step": chunks,
            "bytes_per_step": kbytes,
            "bytes_basis": ("one random 64 B sector (the 16 B walk entry) + the 4 B coalesced "
                            "log store per step") if bouquet else
                           "vertex record, adjacency entry and counter update: 3 random 64 B sectors",
            "steps_per_launch": per_launch_steps,
            "line_pricing": {
                "bytes_per_step": WALK_KERNEL_BYTES_PER_STEP_LINE, "achieved": line,
                "frac": line / HBM_PEAK_GBS,
                "basis": "the 128 B L2 line a random read fetches on gfx950 (TCC_EA0_RDREQ_128B) "
                         "+ the 4 B log store"} if bouquet else None,
            "random_read_ceiling": None if probe is None else {
                "reads_per_s": probe["reads_per_s"],
                "kernel_steps_per_s": per_launch_steps / launch_s,
                "frac": per_launch_steps / launch_s / probe["reads_per_s"],
                "probe": "saba_probe_random_reads: 2^26 records of 16 B (1 GiB), 8192 x 256 lanes, "
                         "256 dependent reads each"},
            "call": {"ms": call_ms, "count_ms": float(np.mean(cms)),
                     "walk_ms": k_ms, "steps_per_s": W * L / (call_ms * 1e-3)},
        },
        "side_by_side": side,
    }


def side_walks(args, saba, torch, np, sg, src, L, seed, ep, vi):
    """The walk benchmark's other arrangements on the same starts: naive generation (one lane per
    walk in list order, CSR reads, atomic counters), the same list order on the bouquet kernel's
    data path (walk entries, visit log: the walk order alone differs from the headline), and
    the paper's grouped bouquets (G = 64 with S = 20 and S = 12: walks of a group share their
    path until their choices split, so a wavefront's reads coalesce; the walks are then
    correlated within a group, the more so the smaller S).  Both naive orders give the
    headline's histograms; G = 64 draws other walks.  G is not an execution knob: it changes
    which walks are drawn, so no autotuner may pick it."""
    W = int(src.numel())
    rows = []
    for name, mode, G, S, reps in (("naive G=1", saba.SABA_WALK_NAIVE, 1, 0, 3),
                                   ("naive order on walk entries + log G=1",
                                    saba.SABA_WALK_NAIVE_LOG, 1, 0, 5),
                                   ("bouquet G=64 S=20", saba.SABA_WALK_BOUQUET, 64, 20, 10),
                                   ("bouquet G=64 S=12", saba.SABA_WALK_BOUQUET, 64, 12, 10)):
        saba.walks(sg, src, L, seed, group=G, spread=S, mode=mode, endpoint=ep, visits=vi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = saba.walks(sg, src, L, seed, group=G, spread=S, mode=mode, endpoint=ep,
                           visits=vi, time_kernels=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert int(vi.sum().item()) == W * L and int(ep.sum().item()) == W
        rows.append({"arrangement": name, "ms_per_step": dt * 1e3,
                     "walk_steps_per_s": W * L / dt, "walk_kernel_ms": r.stats["kernel_ms"]})
        progress(f"walks {name}: {dt * 1e3:.2f} ms per call")
    return rows


def _hist_percentile(h, q):
    """Smallest k with at least a fraction q of the (vector, position) pairs at <= k distinct."""
    import numpy as np
    c = np.cumsum(h) / max(1, h.sum())
    return int(np.searchsorted(c, q - 1e-12))


def bench_ablation(args, saba, torch, np):
    """The paper's comparison of neighbour-choice functions and walk arrangements (the Table 7
    and Table 5 experiments) on the walk benchmark graph: each (execution mode, sampler, key
    grouping) runs the 2^24 x 64 workload for throughput, and a paper-shaped workload (4096
    uniform sources x 256 walks x 15 steps) for the branching statistics of 8-walk vectors."""
    import graphgen
    g = graphgen.rmat(args.scale, 16, 0.57, 0.19, 0.19, 1)
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    W, L = 1 << args.walks_log2, args.length
    src = torch.from_numpy(graphgen.uniform_sources(g, W, 1)).cuda()
    few = torch.from_numpy(np.repeat(graphgen.uniform_sources(g, 4096, 2), 256)).cuda()
    NV, BQ, NL = saba.SABA_WALK_NAIVE, saba.SABA_WALK_BOUQUET, saba.SABA_WALK_NAIVE_LOG
    rows_def = [
        ("naive, Eq. (3) per-walk stream, modulo", NV, 2, 1, 0),
        ("naive, Eq. (4) keyed hash, modulo", NV, 1, 1, 0),
        ("naive, Eq. (5) keyed hash, scaled", NV, 0, 1, 0),
        ("naive order on walk entries + log, Eq. (4) keyed hash, modulo", NL, 1, 1, 0),
        ("naive order on walk entries + log, Eq. (5) keyed hash, scaled", NL, 0, 1, 0),
        ("bouquet, Eq. (4) keyed hash, modulo", BQ, 1, 1, 0),
        ("bouquet, Eq. (5) keyed hash, scaled (headline)", BQ, 0, 1, 0),
        ("bouquet, Eq. (5) keyed, SABA groups G=64 S=20", BQ, 0, 64, 20),
        ("bouquet, Eq. (5) keyed, SABA groups G=64 S=12", BQ, 0, 64, 12),
        ("bouquet, Eq. (5) keyed, SABA groups G=256 S=4", BQ, 0, 256, 4),
        ("bouquet, Eq. (4) keyed modulo, groups G=64 S=20", BQ, 1, 64, 20),
        ("bouquet, Eq. (5) read literally (negative)", BQ, 3, 1, 0),
    ]
    ep = torch.empty(g.n, dtype=torch.int64, device="cuda")
    vi = torch.empty(g.n, dtype=torch.int64, device="cuda")
    rows = []
    for name, mode, sampler, G, S in rows_def:
        progress(f"ablation: {name}")
        saba.walks(sg, src, L, 1, group=G, spread=S, mode=mode, sampler=sampler, endpoint=ep,
                   visits=vi)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            saba.walks(sg, src, L, 1, group=G, spread=S, mode=mode, sampler=sampler,
                       endpoint=ep, visits=vi)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert int(vi.sum().item()) == W * L
        h = saba.walks(sg, few, 15, 1, group=G, spread=S, mode=mode, sampler=sampler,
                       distinct=True).distinct.cpu().numpy()
        rows.append({"name": name, "mode": {NV: "naive", BQ: "bouquet", NL: "naive_log"}[mode],
                     "sampler": sampler, "group": G, "spread": S, "ms_per_step": dt * 1e3,
                     "walk_steps_per_s": W * L / dt,
                     "distinct_mean": float((h * np.arange(9)).sum() / max(1, h.sum())),
                     "distinct_p1": _hist_percentile(h, 0.01),
                     "distinct_p10": _hist_percentile(h, 0.10),
                     "distinct_p25": _hist_percentile(h, 0.25),
                     "distinct_hist": h.tolist()})
    base = rows[0]["walk_steps_per_s"]
    for r in rows:
        r["speedup_vs_first"] = r["walk_steps_per_s"] / base
    # the grouped schedule an autotuner picks under a correlation budget (least mean distinct
    # vertices per 8-walk vector, measured on the same workload)
    tuned = []
    for budget in (() if args.no_tune else (7.5, 6.0, 4.0, 2.0, 1.0)):
        progress(f"ablation: bouquet autotuner at budget {budget}")
        b = saba.autotune_bouquet(sg, src, L, 1, budget)
        tuned.append({"min_distinct": budget, "group": b["group"], "spread": b["spread"],
                      "distinct_mean": b["distinct_mean"], "ms_per_step": b["ms"],
                      "walk_steps_per_s": W * L / (b["ms"] * 1e-3)})
    return {"workload": f"rmat{args.scale}_ef16_walks_2^{args.walks_log2}x{L}_samplers",
            "branching_workload": f"rmat{args.scale}: 4096 uniform sources x 256 walks x 15 steps",
            "rows": rows, "autotuned_schedules": tuned}


def bench_walks_paper(args, saba, torch, np):
    """The shape of the paper's walk-generation experiment (its Table 7): a fixed number of walks
    from every non-isolated vertex of the walk benchmark graph, 15 and 5 steps, naive order
    against bouquet order (G = 1) and grouped bouquets (G = 64).  The paper reports the speed-up
    of its SABA arrangement over naive generation; this is the same ratio on the GPU."""
    import graphgen
    g = graphgen.rmat(args.scale, 16, 0.57, 0.19, 0.19, 1)
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    pool = torch.from_numpy(np.flatnonzero(np.diff(g.row_ptr) > 0).astype(np.int32)).cuda()
    ep = torch.empty(g.n, dtype=torch.int64, device="cuda")
    vi = torch.empty(g.n, dtype=torch.int64, device="cuda")
    NV, BQ, NL = saba.SABA_WALK_NAIVE, saba.SABA_WALK_BOUQUET, saba.SABA_WALK_NAIVE_LOG
    # naive-log: the naive order on the bouquet kernel's data path (walk entries, visit log),
    # so that bouquet G=1 against it is the walk order alone
    arrangements = [("naive", NV, 1, 0), ("naive order, walk entries + log", NL, 1, 0),
                    ("bouquet G=1", BQ, 1, 0),
                    ("bouquet G=64 S=20", BQ, 64, 20), ("bouquet G=64 S=12", BQ, 64, 12)]
    rows = []
    for per_vertex, L in ((args.paper_walks, 15), (args.paper_walks, 5)):
        src = torch.repeat_interleave(pool, per_vertex)  # every start, in vertex order
        W = int(src.numel())
        for name, mode, G, S in arrangements:
            progress(f"walks_paper: {per_vertex} walks/vertex x {L} steps, {name}")
            saba.walks(sg, src, L, 1, group=G, spread=S, mode=mode, endpoint=ep, visits=vi)
            torch.cuda.synchronize()
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                saba.walks(sg, src, L, 1, group=G, spread=S, mode=mode, endpoint=ep, visits=vi)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            assert int(vi.sum().item()) == W * L and int(ep.sum().item()) == W
            rows.append({"walks_per_vertex": per_vertex, "steps": L, "walks": W,
                         "arrangement": name, "seconds": dt, "walk_steps_per_s": W * L / dt})
        del src
        torch.cuda.empty_cache()
    for r in rows:
        base = next(x for x in rows if x["steps"] == r["steps"] and x["arrangement"] == "naive")
        r["speedup_vs_naive"] = base["seconds"] / r["seconds"]
        nl = next(x for x in rows if x["steps"] == r["steps"]
                  and x["arrangement"] == "naive order, walk entries + log")
        r["speedup_vs_naive_order_same_data_path"] = nl["seconds"] / r["seconds"]
    return {"workload": f"rmat{args.scale}_ef16_every_vertex_x{args.paper_walks}_walks",
            "starts": int(pool.numel()), "rows": rows}


_CL1M = {}


def chung_lu_1e6():
    """The 10^6-vertex Chung-Lu graph (average degree 10, exponent 2.5, seed 1, largest
    component) and its lambda, built once per run."""
    if not _CL1M:
        import graphgen
        t0 = time.perf_counter()
        g = graphgen.largest_component(graphgen.chung_lu(1000000, 10, 2.5, 1))
        _CL1M.update(g=g, lam=graphgen.spectral_lambda(g), prep_s=time.perf_counter() - t0)
    return _CL1M["g"], _CL1M["lam"], _CL1M["prep_s"]


def bench_aesc(args, saba, torch, np):
    import graphgen
    g, lam, prep_s = chung_lu_1e6()
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    ce = graphgen.canonical_edges(g)
    perm = np.random.default_rng(7).permutation(g.m)
    k = max(1, int(round(args.aesc_frac * g.m)))
    q = np.ascontiguousarray(ce[np.sort(perm[:k])])
    qt = torch.from_numpy(q).cuda()
    warm = torch.from_numpy(np.ascontiguousarray(ce[np.sort(perm[k:k + 64])])).cuda()
    # execution knobs tuned on a sample of other edges (2% of the query's size); results do not
    # depend on them
    sample = torch.from_numpy(np.ascontiguousarray(ce[np.sort(perm[k + 64:k + 64 + k // 50])])).cuda()
    t0 = time.perf_counter()
    tuned = saba.autotune_aesc(sg, [{"graph": 0, "eps": args.aesc_eps, "lam": lam, "seed": 1,
                                     "edges": sample}],
                               mem_budget=int(args.aesc_mem_gib * (1 << 30)))
    tune_s = time.perf_counter() - t0
    mem = int(args.aesc_mem_gib * (1 << 30))
    # first the query with the other batch-stream setting (in order on one stream, or the
    # levels of batch k + 1 beside the walk pairs of batch k), its pools grown on the tuning
    # sample; then the timed query with the tuned knobs, last, so that its dispatches end a
    # profiled run.  The two give identical results.
    cfg = saba.get_config(sg)
    other = 2 if cfg["est_batch_streams"] == 1 else 1
    saba.set_config(sg, **{**cfg, "est_batch_streams": other})
    saba.aesc_query(sg, sample, args.aesc_eps, lam, 1, mem_budget=mem)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sc1, st1 = saba.aesc_query(sg, qt, args.aesc_eps, lam, 1, time_kernels=True, mem_budget=mem)
    torch.cuda.synchronize()
    d1 = time.perf_counter() - t1
    saba.set_config(sg, **cfg)
    saba.aesc_query(sg, sample, args.aesc_eps, lam, 1, mem_budget=mem)
    saba.aesc_query(sg, warm, args.aesc_eps, lam, 1, mem_budget=mem)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc, st = saba.aesc_query(sg, qt, args.aesc_eps, lam, 1, time_kernels=True, mem_budget=mem)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert bool(torch.isfinite(sc).all().item())
    assert torch.equal(sc, sc1), "results differ between the batch-stream settings"
    walk_s = st["kernel_ms"] * 1e-3
    # the walk-pair kernel of the tuned schedule (the staged one keeps the support bitmap in LDS)
    mc_kernel = "mc_walk_staged_kernel" if cfg["est_walk_queue"] == 2 else "mc_walk_kernel"
    achieved = AESC_STEP_BYTES * st["walk_steps"] / walk_s / 1e9 if walk_s > 0 else 0.0
    line = AESC_STEP_BYTES_LINE * st["walk_steps"] / walk_s / 1e9 if walk_s > 0 else 0.0
    out = {
        "value": k / dt,
        "unit": "edges/s",
        "seconds": dt,
        "edges": k,
        "eps": args.aesc_eps,
        "workload": "chung_lu_n1e6_k10_b2.5_lcc_eps0.1_query_1pct"
        if abs(args.aesc_frac - 0.01) < 1e-12 else f"chung_lu_n1e6_k10_b2.5_lcc_query_{args.aesc_frac}",
        "graph": {"n": g.n, "m": g.m, "lambda": lam, "prep_s": prep_s},
        "walk_steps": st["walk_steps"],
        "walk_steps_per_s": st["walk_steps"] / dt,
        "push_edge_visits": st["push_edge_visits"],
        "sources": st["sources"],
        "max_tau": st["max_tau"], "max_ttau": st["max_ttau"],
        "tuned": tuned, "autotune_s": tune_s, "batches": st["batches"],
        "other_batch_streams": {"est_batch_streams": other, "seconds": d1,
                                "edges_per_s": k / d1, "batches": st1["batches"],
                                "walk_kernel_ms": st1["kernel_ms"], "identical": True},
        "roofline": {"bound": "hbm", "kernel": mc_kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": estimator_traffic(st["walk_steps"], st["batches"], mc_kernel),
                     "traffic_basis": TRAFFIC_BASIS,
                     "kernel_ms": st["kernel_ms"], "launches": st["batches"],
                     "bytes_per_step": AESC_STEP_BYTES,
                     "bytes_basis": "one random 64 B sector (the 16 B walk entry) per step",
                     "line_pricing": {"bytes_per_step": AESC_STEP_BYTES_LINE, "achieved": line,
                                      "frac": line / HBM_PEAK_GBS,
                                      "basis": "the 128 B L2 line a random read fetches"}},
    }
    # the eigenpair form of the truncation (omega = 64) on the same query: the pairs are found
    # once per graph (timed separately) and cached; same eps guarantee
    if args.no_omega:
        return _aesc_cpu_baseline(args, g, lam, q, k, out)
    t1 = time.perf_counter()
    spec = saba.graph_spectrum(sg, 64, vectors=False)
    spec_s = time.perf_counter() - t1
    saba.aesc_query(sg, warm, args.aesc_eps, 0.0, 1, omega=64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st64 = saba.aesc_query(sg, qt, args.aesc_eps, 0.0, 1, omega=64)
    torch.cuda.synchronize()
    d64 = time.perf_counter() - t1
    out["omega64"] = {"edges_per_s": k / d64, "seconds": d64, "eigenpairs_s": spec_s,
                      "radius": spec["lambda_rest_bound"], "walk_steps": st64["walk_steps"],
                      "max_tau": st64["max_tau"]}
    return _aesc_cpu_baseline(args, g, lam, q, k, out)


def _aesc_cpu_baseline(args, g, lam, q, k, out):
    """The oracle on the host cores, on the first edges of the same query."""
    if not args.no_cpu_baseline:
        import oracle
        cores = host_threads()
        # double the sample until it takes more than 6 s of host work (the last one is kept)
        nq = 64
        while True:
            t1 = time.perf_counter()
            oracle.aesc(g, args.aesc_eps, lam, 1, query=q[:nq], nthreads=cores)
            dq = time.perf_counter() - t1
            if dq > 6.0 or nq >= k:
                break
            nq = min(k, 2 * nq)
        out["cpu_baseline"] = {"value": nq / dq, "unit": "edges/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"first {nq} edges of the same 1% sample ({dq:.1f} s wall, "
                                         "OpenMP over sources)"}
    return out


def bench_omega(args, saba, torch, np):
    """The eigenpair form of the truncation on the 1% query workload of the 10^6-vertex
    Chung-Lu graph: for each omega, the cost of the leading eigenpairs (a fresh Lanczos run),
    the radius tau is taken from, and the estimator's time and walk steps with the pairs
    cached.  omega = 0 is the plain series with the library's lambda.  Walk pairs on the staged
    schedule (support bitmaps in LDS; no knob changes a result)."""
    import graphgen
    g = graphgen.largest_component(graphgen.chung_lu(1000000, 10, 2.5, 1))
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    saba.set_config(sg, est_walk_queue=2)
    ce = graphgen.canonical_edges(g)
    perm = np.random.default_rng(7).permutation(g.m)
    k = max(1, int(round(args.aesc_frac * g.m)))
    qt = torch.from_numpy(np.ascontiguousarray(ce[np.sort(perm[:k])])).cuda()
    warm = torch.from_numpy(np.ascontiguousarray(ce[np.sort(perm[k:k + 64])])).cuda()
    lam = saba.graph_lambda(sg, max_iters=1000)
    rows = []
    base = None
    for omega in (0, 8, 32, 64):
        row = {"omega": omega}
        if omega > 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = saba.graph_spectrum(sg, omega, vectors=False)
            row["spectrum_s"] = time.perf_counter() - t0
            row.update({"radius": r["lambda_rest_bound"], "pairs": r["pairs"],
                        "iterations": r["iterations"], "max_residual": r["max_residual"],
                        "converged": r["converged"],
                        "smallest_kept_abs_theta": float(np.min(np.abs(r["values"])))})
        else:
            row["radius"] = lam["lambda_bound"]
        saba.aesc_query(sg, warm, args.aesc_eps, 0.0, 1, omega=omega)  # fills the pair cache
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc, st = saba.aesc_query(sg, qt, args.aesc_eps, 0.0, 1, omega=omega)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        row.update({"seconds": dt, "edges_per_s": k / dt, "walk_steps": st["walk_steps"],
                    "push_edge_visits": st["push_edge_visits"], "max_tau": st["max_tau"],
                    "sum_sc": float(sc.sum().item())})
        if base is None:
            base = sc
        else:
            row["max_abs_change_vs_omega0"] = float((sc - base).abs().max().item())
        rows.append(row)
        progress(f"omega {omega}: {dt:.2f} s, radius {row['radius']:.6f}")
    # the paper's grouping (SABA, G = 64, S = 20) on the same query: the walks of a group
    # share their path until their choices split, so a wavefront's reads coalesce; the eps
    # guarantee is then empirical
    grouped = []
    for omega in (0, 64):
        saba.aesc_query(sg, warm, args.aesc_eps, 0.0, 1, omega=omega, group=64, spread=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc, st = saba.aesc_query(sg, qt, args.aesc_eps, 0.0, 1, omega=omega, group=64, spread=20,
                                 time_kernels=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        grouped.append({"omega": omega, "group": 64, "spread": 20, "seconds": dt,
                        "edges_per_s": k / dt, "walk_steps": st["walk_steps"],
                        "walk_kernel_ms": st["kernel_ms"],
                        "max_abs_change_vs_omega0_G1": float((sc - base).abs().max().item()),
                        "mean_abs_change_vs_omega0_G1": float((sc - base).abs().mean().item())})
        progress(f"omega {omega}, G 64: {dt:.2f} s")
    return {"workload": "chung_lu_n1e6_k10_b2.5_lcc_eps0.1_query_1pct", "edges": k,
            "lambda": lam["lambda"], "rows": rows, "grouped": grouped}


def bench_aesc_full(args, saba, torch, np, tuned=None):
    """All edges of the 10^6-vertex Chung-Lu graph at eps = 0.1.  omega = 0: the sources in 100
    consecutive ranges (saba_aesc_sources, one progress line per range; each source's levels
    run once), then saba_aesc_combine, which gives saba_aesc's output bit for bit.  omega > 0
    (the eigenpair tail belongs to the undirected edge): the canonical edges in 40 query calls,
    each equal to the all-edges call's entries.  Execution knobs: those the 1% query leg tuned
    on this graph when given, else the staged walk-pair schedule (no knob changes a result)."""
    import graphgen
    g, lam1, _ = chung_lu_1e6()
    omega = args.omega
    # omega > 0: the radius of the rest of the spectrum comes from the library
    lam = lam1 if omega == 0 else 0.0
    sg = saba.SabaGraph.from_graph(g, trusted=True)
    knobs = dict(tuned) if tuned else {"est_walk_queue": 2}
    saba.set_config(sg, **knobs)
    ce = graphgen.canonical_edges(g)
    saba.aesc_query(sg, torch.from_numpy(np.ascontiguousarray(ce[:64])).cuda(), args.aesc_eps, lam, 1,
                    omega=omega)
    torch.cuda.synchronize()
    steps = 0
    t0 = time.perf_counter()
    if omega == 0:
        gd = torch.empty(g.nnz, dtype=torch.float64, device="cuda")
        nr = 100
        bounds = np.linspace(0, g.n, nr + 1).astype(int)
        for k in range(nr):
            st = saba.aesc_sources(sg, gd, int(bounds[k]), int(bounds[k + 1]), args.aesc_eps, lam, 1)
            torch.cuda.synchronize()
            steps += st["walk_steps"]
            progress(f"aesc full: {k + 1}/{nr} source ranges, {time.perf_counter() - t0:.1f} s")
        sc = saba.aesc_combine(sg, gd)
        torch.cuda.synchronize()
        sums = float(sc.sum().item())
        form = f"{nr} source ranges (saba_aesc_sources) and saba_aesc_combine"
    else:
        parts = np.array_split(np.arange(g.m), 40)
        sums = 0.0
        for k, idx in enumerate(parts):
            q = torch.from_numpy(np.ascontiguousarray(ce[idx])).cuda()
            sc, st = saba.aesc_query(sg, q, args.aesc_eps, lam, 1, omega=omega)
            torch.cuda.synchronize()
            steps += st["walk_steps"]
            sums += float(sc.sum().item())
            progress(f"aesc full: {k + 1}/{len(parts)} parts, {time.perf_counter() - t0:.1f} s")
        form = "40 query calls over the canonical edges"
    dt = time.perf_counter() - t0
    return {"workload": "chung_lu_n1e6_k10_b2.5_lcc_eps0.1_all_edges"
            + (f"_omega{omega}" if omega else ""), "edges": g.m, "n": g.n,
            "lambda": lam, "omega": omega, "seconds": dt, "edges_per_s": g.m / dt,
            "walk_steps": steps, "sum_sc": sums, "n_minus_1": g.n - 1, "form": form,
            "knobs": saba.get_config(sg)}


def _batch_graph(spec):
    """One graph of the batched workload: (kind, n, seed) -> (graph, lambda upper bound)."""
    import graphgen
    kind, n, seed = spec
    if kind == 0:
        g = graphgen.largest_component(graphgen.er_gnm(n, 4 * n, seed))
    elif kind == 1:
        g = graphgen.largest_component(graphgen.chung_lu(n, 8, 2.3, seed))
    else:
        side = max(2, int(round(n ** 0.5)))
        g = graphgen.largest_component(graphgen.grid_diagonals(side, side, 0.05, seed))
    # grids: lambda is left to the device (saba_graph_lambda on the batched handle); the CPU
    # eigensolver is slow to separate their eigenvalues near 1
    lam = None if kind == 2 else graphgen.spectral_lambda(g)
    return g.row_ptr, g.col_idx, lam


def _batch_graph_indexed(item):
    k, spec = item
    return k, _batch_graph(spec)


def progress(msg):
    print(json.dumps({"progress": msg}), file=sys.stderr, flush=True)


def parallel_build(fn, items, label):
    """Run fn over (index, spec) items in a spawn pool with one BLAS thread per worker (the
    pool supplies the parallelism); returns the results by index, printing progress."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    built = [None] * len(items)
    step = max(1, len(items) // 8)
    try:
        with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
            for done, (k, res) in enumerate(pool.imap_unordered(fn, list(enumerate(items))), 1):
                built[k] = res
                if done % step == 0 or done == len(items):
                    progress(f"{label}: {done}/{len(items)} graphs built "
                             f"({time.perf_counter() - t0:.0f} s)")
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return built


def batch_workload(G=256, edge_frac=0.01):
    """The batched workload's inputs: G graphs (kind k % 3, n uniform in [1e3, 2e5], seed
    1000 + k), lambda per graph (None for the grids: see device_lambdas), eps per graph from
    {0.1, 0.2, 0.3}, and a seeded fraction edge_frac of each graph's edges (at least one) as
    its query (int32 [q, 2])."""
    import graphgen
    import numpy as np
    rng = np.random.default_rng(4)
    specs = [(k % 3, int(rng.integers(1000, 200001)), 1000 + k) for k in range(G)]
    epss = [float(rng.choice([0.1, 0.2, 0.3])) for _ in range(G)]
    built = parallel_build(_batch_graph_indexed, specs, "batch workload")
    graphs = [graphgen.Graph(rp, ci) for rp, ci, _ in built]
    lams = [lam for _, _, lam in built]
    qs = []
    for g in graphs:
        ce = graphgen.canonical_edges(g)
        q = max(1, int(round(edge_frac * g.m)))
        pick = np.sort(rng.choice(g.m, min(g.m, q), replace=False))
        qs.append(np.ascontiguousarray(ce[pick]))
    return graphs, lams, epss, qs


def device_lambdas(saba, mg, lams):
    """lambda of the graphs the workload left to the device: the upper estimate
    saba_graph_lambda returns for graph k of the batched handle (below 1)."""
    out = list(lams)
    for k, lam in enumerate(lams):
        if lam is None:
            r = saba.graph_lambda(mg, index=k, max_iters=1000)
            out[k] = min(r["lambda_bound"], 1.0 - 1e-12)
    return out


def tuning_sample(reqs, every=16, edges=64):
    """The autotuner's sample of a request list: every 16th request, its first 64 edges."""
    return [{**r, "edges": r["edges"][:edges]} for r in reqs[::every]]


def truncation_bound(g, q, lam, eps, tau_cap):
    """Largest certified truncation error over the query edges q of graph g when tau is capped:
    (1/d_u + 1/d_v) lam^(tau + 1) / (1 - lam) at tau = min(CalculateTau, tau_cap), and whether
    every edge meets eps / 2 (Alg. 1's truncation budget)."""
    import math
    import numpy as np
    deg = np.diff(g.row_ptr).astype(np.float64)
    w = 1.0 / deg[q[:, 0]] + 1.0 / deg[q[:, 1]]
    # smallest tau with w lam^(tau+1) <= (eps/2)(1 - lam), from the log form
    need = np.ceil(np.log((eps / 2.0) * (1.0 - lam) / w) / math.log(lam) - 1.0)
    tau = np.minimum(np.maximum(need, 0.0), tau_cap)
    bound = w * lam ** (tau + 1.0) / (1.0 - lam)
    return float(bound.max()), bool(np.all(bound <= eps / 2.0 * (1.0 + 1e-9)))


def bench_batch(args, saba, torch, np):
    """Batched estimation: 256 graphs of uneven size (n uniform in [1e3, 2e5]; one third each
    Erdos-Renyi with average degree 8, Chung-Lu with exponent 2.3, square grids with 5% random
    diagonals), eps drawn from {0.1, 0.2, 0.3}, a seeded 1% of every graph's edges as its query,
    tau capped at 128.  One saba_aesc_batch call on a multi-graph handle against one
    saba_aesc_query call per graph; both must give identical results.  The grids mix so slowly
    (lambda within 1e-3 of 1) that the cap leaves a truncation error far above eps: their
    requests are reported apart as uncertified, and the certified throughput comes from a call
    over the other requests alone."""
    G = args.batch_graphs
    t0 = time.perf_counter()
    graphs, lams0, epss, qnp = batch_workload(G, args.batch_frac)
    prep_s = time.perf_counter() - t0
    qs = [torch.from_numpy(q).cuda() for q in qnp]
    nq = sum(int(q.shape[0]) for q in qs)
    mg = saba.SabaGraph.from_graphs(graphs, trusted=True)
    t0 = time.perf_counter()
    lams = device_lambdas(saba, mg, lams0)
    lam_s = time.perf_counter() - t0
    cert = [truncation_bound(g, q, l, e, 128) for g, q, l, e in zip(graphs, qnp, lams, epss)]
    certified = [k for k in range(G) if cert[k][1]]
    progress(f"batch workload: {nq} query edges, {len(certified)}/{G} requests certified at eps "
             f"with tau <= 128 (device lambda of the grids in {lam_s:.1f} s)")
    reqs = [{"graph": k, "eps": epss[k], "lam": lams[k], "seed": 1, "edges": qs[k], "tau_cap": 128}
            for k in range(G)]
    # the execution knobs (walk-pair and frontier-group grids, walk-pair schedule, batch
    # streams) tuned on every 16th request, its first 64 edges, on the multi-graph handle;
    # they do not change results, and the one-call-per-graph path below runs with them too
    progress("batch workload: autotuning the estimator grids")
    t0 = time.perf_counter()
    tuned = saba.autotune_aesc(mg, tuning_sample(reqs))
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    progress(f"batch workload: tuned {tuned} in {tune_s:.1f} s; one call per graph")
    # one call per graph: each graph in its own handle with the same knobs, uploaded and warmed
    # (its scratch sized by the same query) before its timed call, and freed afterwards, so the
    # handles' scratch does not pile up; the times of the calls alone are summed
    single, single_s = {}, {}
    t_wall = time.perf_counter()
    for k in range(G):
        h = saba.SabaGraph.from_graph(graphs[k], trusted=True)
        saba.set_config(h, **tuned)
        saba.aesc_query(h, qs[k], epss[k], lams[k], 1, tau_cap=128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        single[k] = saba.aesc_query(h, qs[k], epss[k], lams[k], 1, tau_cap=128)[0]
        torch.cuda.synchronize()
        single_s[k] = time.perf_counter() - t0
        h.close()
        if (k + 1) % 32 == 0:
            progress(f"batch workload: {k + 1}/{G} single calls ({sum(single_s.values()):.1f} s "
                     f"timed, {time.perf_counter() - t_wall:.0f} s wall)")
    t_single = sum(single_s.values())
    t_single_cert = sum(single_s[k] for k in certified)
    progress("batch workload: batched calls")

    def batched(rs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs, st = saba.aesc_batch(mg, rs, time_kernels=True)
        torch.cuda.synchronize()
        return outs, st, time.perf_counter() - t0

    batched(reqs)  # warm-up: the handle's pools grow to the workload, as the single calls' do
    outs, st, t_batch = batched(reqs)
    same = all(bool(torch.equal(single[k], outs[k])) for k in range(G))
    assert same, "batched results differ from single-graph results"
    outs_c, st_c, t_batch_cert = batched([reqs[k] for k in certified])
    assert all(bool(torch.equal(single[k], o)) for k, o in zip(certified, outs_c))
    # the three walk-pair schedules at the tuned grids
    sched = {}
    for wq, name in ((0, "static"), (1, "queue"), (2, "staged")):
        saba.set_config(mg, **{**tuned, "est_walk_queue": wq})
        _, st_q, t_q = batched(reqs)
        sched[name] = {"seconds": t_q, "walk_kernel_ms": st_q["kernel_ms"]}
        progress(f"batch workload: {name} schedule {t_q:.3f} s")
    saba.set_config(mg, **tuned)
    nq_cert = sum(int(qs[k].shape[0]) for k in certified)
    kinds = {0: "erdos_renyi", 1: "chung_lu", 2: "grid"}
    return {"workload": f"batch_{G}graphs_n1e3-2e5_er_cl_grid_q{args.batch_frac:g}",
            "graphs": G, "vertices": sum(g.n for g in graphs), "edges": sum(g.m for g in graphs),
            "query_edges": nq, "prep_s": prep_s, "device_lambda_s": lam_s,
            "single_calls_s": t_single, "single_edges_per_s": nq / t_single,
            "batched_s": t_batch, "batched_edges_per_s": nq / t_batch,
            "speedup": t_single / t_batch, "identical": same,
            "certified": {"requests": len(certified), "query_edges": nq_cert,
                          "kinds": sorted({kinds[k % 3] for k in certified}),
                          "single_calls_s": t_single_cert,
                          "batched_s": t_batch_cert, "batched_edges_per_s": nq_cert / t_batch_cert,
                          "speedup": t_single_cert / t_batch_cert,
                          "walk_steps": st_c["walk_steps"]},
            "uncertified": {"requests": G - len(certified),
                            "kinds": sorted({kinds[k % 3] for k in range(G) if not cert[k][1]}),
                            "max_truncation_bound": max((cert[k][0] for k in range(G)
                                                         if not cert[k][1]), default=0.0),
                            "lambda_range": [min((lams[k] for k in range(G) if not cert[k][1]),
                                                 default=0.0),
                                             max((lams[k] for k in range(G) if not cert[k][1]),
                                                 default=0.0)]},
            "schedules": sched,
            "walk_steps": st["walk_steps"], "sources": st["sources"], "batches": st["batches"],
            "walk_kernel_ms": st["kernel_ms"], "tau_capped": bool(st["warnings"] & 1),
            "tuned": tuned, "autotune_s": tune_s}


def _serve_graph_indexed(item):
    """One resident graph of the serving workload: the Chung-Lu generator of the 10^6-vertex
    estimator workload (average degree 10, exponent 2.5) at its own size and seed."""
    import graphgen
    k, (n, seed) = item
    g = graphgen.largest_component(graphgen.chung_lu(n, 10, 2.5, seed))
    return k, (g.row_ptr, g.col_idx, graphgen.spectral_lambda(g))


class _Collector:
    """Waits for served tickets on its own thread (the wait call releases the GIL) and keeps
    each request's outcome."""

    def __init__(self, srv):
        import queue
        import threading
        self.srv, self.q, self.done = srv, queue.Queue(), []
        self.th = threading.Thread(target=self._run, daemon=True)
        self.th.start()

    def _run(self):
        while True:
            item = self.q.get()
            if item is None:
                return
            ticket, q, keep = item
            sc, res = self.srv.wait(ticket)
            res["q"] = q
            res["t_done"] = time.perf_counter()
            if keep is not None:
                keep[ticket] = sc
            self.done.append(res)

    def finish(self):
        self.q.put(None)
        self.th.join()
        return self.done


def _latency_summary(done, t_start):
    import numpy as np
    if not done:
        return {"completed": 0}
    lat = np.array([d["latency_ms"] for d in done])
    edges = sum(d["q"] for d in done)
    t_end = max(d["t_done"] for d in done)
    return {"completed": len(done), "edges": edges,
            "edges_per_s": edges / (t_end - t_start), "requests_per_s": len(done) / (t_end - t_start),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "queue_p50_ms": float(np.percentile([d["queue_ms"] for d in done], 50)),
            "mean_batches_per_request": float(np.mean([d["batches"] for d in done]))}


def serve_workload():
    """The serving workload's resident graphs: Chung-Lu (average degree 10, exponent 2.5),
    n_i = round(10^(4 + 2i/15)) for i = 0..15, seeds 1..16, largest components; and lambda per
    graph."""
    import graphgen
    ns = [int(round(10 ** (4 + 2 * i / 15))) for i in range(16)]
    built = parallel_build(_serve_graph_indexed, [(n, i + 1) for i, n in enumerate(ns)],
                           "serve workload")
    return [graphgen.Graph(rp, ci) for rp, ci, _ in built], [lam for _, _, lam in built]


def bench_serve(args, saba, torch, np):
    """Serving: 16 resident Chung-Lu graphs (n_i = round(10^(4 + 2i/15)), i = 0..15, seeds
    1..16, largest components), SC query requests of 1-4096 uniformly chosen edges of one
    uniformly chosen graph at eps drawn from {0.1, 0.2, 0.3}.
      offered:   Poisson arrivals at --serve-rate requests/s for --serve-seconds, into a server
                 whose admission queue holds --serve-queue-edges edges (beyond it requests are
                 refused: backpressure); throughput and latency of what was served;
      sustained: Poisson arrivals at --serve-sustain-frac of the throughput measured above, for
                 --serve-sustain-seconds, with an unbounded queue: p50 / p99 latency;
      plain:     the same --serve-compare requests one saba_aesc_query call each (one graph per
                 launch) against all of them submitted to the server at once; the results must
                 be identical."""
    import graphgen
    t0 = time.perf_counter()
    graphs, lams = serve_workload()
    prep_s = time.perf_counter() - t0
    ces = [graphgen.canonical_edges(g) for g in graphs]
    mg = saba.SabaGraph.from_graphs(graphs, trusted=True)
    saba.set_config(mg, est_walk_queue=args.serve_walk_queue)
    budget = int(args.serve_mem_gib * (1 << 30))

    def server(**kw):
        return saba.SabaServer(mg, lanes=args.serve_lanes, mem_budget=budget,
                               max_batch_sources=args.serve_max_batch, **kw)

    def stream(seed, qmax=4096):
        rng = np.random.default_rng(seed)
        while True:
            k = int(rng.integers(len(graphs)))
            q = int(rng.integers(1, qmax + 1))
            m = ces[k].shape[0]
            pick = rng.choice(m, q, replace=False) if q < m else np.arange(m)
            yield k, np.ascontiguousarray(ces[k][pick]), float(rng.choice([0.1, 0.2, 0.3]))

    def submit(srv, req, omega=0):
        k, e, eps = req
        # omega > 0: the radius of the rest of the spectrum is left to the library
        return srv.submit(k, e, eps, 0.0 if omega else lams[k], 1, omega=omega)

    def open_loop(srv, rate, seconds, seed, label, omega=0):
        rng = np.random.default_rng(seed + 100)
        gen = stream(seed)
        col = _Collector(srv)
        offered = rejected = 0
        t_start = time.perf_counter()
        t_next = 0.0
        t_report = t_start + 10.0
        while t_next < seconds:
            now = time.perf_counter() - t_start
            if now < t_next:
                time.sleep(t_next - now)
            req = next(gen)
            offered += 1
            try:
                col.q.put((submit(srv, req, omega), len(req[1]), None))
            except saba.SabaError as e:
                if e.name != "SABA_E_BUSY":
                    raise
                rejected += 1
            t_next += float(rng.exponential(1.0 / rate))
            if time.perf_counter() > t_report:
                progress(f"serve {label}: {offered} offered, {rejected} refused, "
                         f"{len(col.done)} finished")
                t_report += 10.0
        t_arrivals = time.perf_counter() - t_start
        progress(f"serve {label}: arrivals over ({offered} offered, {rejected} refused); draining")
        done = col.finish()
        out = _latency_summary(done, t_start)
        out.update({"offered_rate": rate, "arrival_seconds": t_arrivals, "offered": offered,
                    "refused": rejected, "failed": sum(1 for d in done if d["status"] != 0)})
        return out

    def compare(gen, count, label):
        progress(f"serve workload: plain calls against the server ({label} requests)")
        reqs = [next(gen) for _ in range(count)]
        handles = [saba.SabaGraph.from_graph(g, trusted=True) for g in graphs]
        dev = [torch.from_numpy(e).cuda() for _, e, _ in reqs]
        # the plain path keeps each graph's scratch between calls: size it once, untimed, with a
        # request of the largest size on every graph (the server allocates its own at creation)
        for k, h in enumerate(handles):
            m = ces[k].shape[0]
            warm = torch.from_numpy(np.ascontiguousarray(ces[k][:min(m, 4096)])).cuda()
            saba.aesc_query(h, warm, 0.3, lams[k], 1, mem_budget=budget)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [saba.aesc_query(handles[k], d, eps, lams[k], 1, mem_budget=budget)[0]
                 for (k, _, eps), d in zip(reqs, dev)]
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        del handles
        keep = {}
        with server() as srv:
            col = _Collector(srv)
            t0 = time.perf_counter()
            tickets = []
            for r in reqs:
                tickets.append(submit(srv, r))
                col.q.put((tickets[-1], len(r[1]), keep))
            col.finish()
            t_served = time.perf_counter() - t0
        same = all(bool(torch.equal(p, keep[t])) for p, t in zip(plain, tickets))
        assert same, "served results differ from the plain per-request results"
        nedge = sum(len(e) for _, e, _ in reqs)
        return {"requests": len(reqs), "edges": nedge, "plain_s": t_plain,
                "plain_edges_per_s": nedge / t_plain, "served_s": t_served,
                "served_edges_per_s": nedge / t_served, "speedup": t_plain / t_served,
                "identical": same}

    if args.serve_short:
        # the default run's serving leg: the offered load with backpressure, then a sustained
        # load without refusals (its p50 / p99 are the headline latencies)
        with server() as srv:
            srv.wait(srv.submit(15, ces[15][:256], 0.1, lams[15], 1))
        torch.cuda.synchronize()
        res = {"workload": "serve_16_chung_lu_n1e4-1e6_k10_b2.5_q1-4096_eps0.1-0.3",
               "graphs": len(graphs), "vertices": sum(g.n for g in graphs),
               "edges": sum(g.m for g in graphs), "prep_s": prep_s, "lanes": args.serve_lanes,
               "mem_budget_gib": args.serve_mem_gib, "knobs": saba.get_config(mg)}
        with server(max_queued_edges=args.serve_queue_edges) as srv:
            res["offered"] = open_loop(srv, args.serve_rate, args.serve_seconds, 11, "offered")
            res["offered"]["queue_bound_edges"] = args.serve_queue_edges
        off = res["offered"]
        off["refused_frac"] = off["refused"] / max(1, off["offered"])
        cap = off.get("edges_per_s", 0.0) / 2048.5
        rate = max(0.2, args.serve_sustain_frac * cap)
        progress(f"serve workload: sustained load at {rate:.2f} requests/s")
        with server(max_queued_edges=1 << 40) as srv:
            res["sustained"] = open_loop(srv, rate, args.serve_sustain_seconds, 12, "sustained")
        res["sustained"]["refused_frac"] = res["sustained"]["refused"] / max(1, res["sustained"]["offered"])
        return res

    # warm the lanes' scratch on the largest graph
    with server() as srv:
        t = srv.submit(15, ces[15][:256], 0.1, lams[15], 1)
        srv.wait(t)
    torch.cuda.synchronize()

    res = {"workload": "serve_16_chung_lu_n1e4-1e6_k10_b2.5_q1-4096_eps0.1-0.3",
           "graphs": len(graphs), "vertices": sum(g.n for g in graphs),
           "edges": sum(g.m for g in graphs), "prep_s": prep_s, "lanes": args.serve_lanes,
           "mem_budget_gib": args.serve_mem_gib, "knobs": saba.get_config(mg)}
    progress("serve workload: offered load")
    with server(max_queued_edges=args.serve_queue_edges) as srv:
        res["offered"] = open_loop(srv, args.serve_rate, args.serve_seconds, 11, "offered")
        res["offered"]["queue_bound_edges"] = args.serve_queue_edges
        res["offered"]["server"] = srv.stats()
    # the refusals favour small requests, so the capacity in requests/s is taken from the
    # edge throughput and the mean request size (2048.5 edges)
    cap = res["offered"].get("edges_per_s", 0.0) / 2048.5
    rate = max(0.2, args.serve_sustain_frac * cap)
    progress(f"serve workload: sustained load at {rate:.2f} requests/s")
    with server(max_queued_edges=1 << 40) as srv:
        res["sustained"] = open_loop(srv, rate, args.serve_sustain_seconds, 12, "sustained")
        res["sustained"]["server"] = srv.stats()

    if args.serve_omega > 0:
        # the same offered load in the eigenpair form; each graph's pairs are found at its
        # first such request and cached in the handle, so they are computed beforehand
        with server(max_queued_edges=args.serve_queue_edges) as srv:
            t0 = time.perf_counter()
            for k in range(len(graphs)):
                srv.wait(submit(srv, (k, ces[k][:8], 0.1), args.serve_omega))
            res["omega_pairs_s"] = time.perf_counter() - t0
            progress(f"serve workload: offered load with omega {args.serve_omega} "
                     f"(pairs found in {res['omega_pairs_s']:.1f} s)")
            res["offered_omega"] = open_loop(srv, args.serve_rate, args.serve_seconds, 11,
                                             f"offered omega {args.serve_omega}",
                                             args.serve_omega)
            res["offered_omega"]["omega"] = args.serve_omega
            res["offered_omega"]["server"] = srv.stats()

    # plain one-request-per-call path against the server on the same requests: requests of
    # the workload's size, and small requests (1-64 edges), where per-call work dominates
    res["plain_vs_served"] = compare(stream(13), args.serve_compare, "workload-sized")
    res["plain_vs_served_small"] = compare(stream(14, qmax=64), 256, "small")
    return res


def bench_er2000(args, saba, torch, np):
    """All edges of ER n=2000, m=8000, seed 1 (largest component), eps=0.3, plain walks."""
    import graphgen
    g = graphgen.largest_component(graphgen.er_gnm(2000, 8000, 1))
    lam = graphgen.spectral_lambda(g)
    sg = saba.SabaGraph.from_graph(g)
    saba.aesc(sg, 0.3, lam, 1)
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        sc, st = saba.aesc(sg, 0.3, lam, 1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    out = {"workload": "er_n2000_m8000_s1_lcc_eps0.3_all_edges", "n": g.n, "m": g.m,
           "latency_ms_median": med * 1e3, "latency_ms_min": min(times) * 1e3,
           "edges_per_s": g.m / med, "walk_steps": st["walk_steps"],
           "push_edge_visits": st["push_edge_visits"],
           "sum_sc": float(sc.sum().item()), "n_minus_1": g.n - 1}
    if not args.no_cpu_baseline:
        import oracle
        cores = host_threads()
        t0 = time.perf_counter()
        oracle.aesc(g, 0.3, lam, 1, nthreads=1)
        d1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.aesc(g, 0.3, lam, 1, nthreads=cores)
        dn = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": g.m / dn, "unit": "edges/s", "cores": cores,
                               "kind": "oracle", "single_thread_edges_per_s": g.m / d1,
                               "sample": "all edges of the same graph"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload",
                    choices=["all", "walks", "aesc", "aesc_full", "er2000", "batch", "serve", "ablation",
                             "omega", "copy", "walks_paper"],
                    default="all")
    ap.add_argument("--batch-graphs", type=int, default=256)
    ap.add_argument("--paper-walks", type=int, default=2048,
                    help="walks per non-isolated vertex in --workload walks_paper")
    ap.add_argument("--batch-frac", type=float, default=0.01,
                    help="fraction of every graph's edges queried in --workload batch")
    ap.add_argument("--serve-lanes", type=int, default=2)
    ap.add_argument("--serve-walk-queue", type=int, default=0,
                    help="walk-pair schedule of the served handle (est_walk_queue: 0 stride, "
                         "1 work queues, 2 staged tiles)")
    ap.add_argument("--serve-mem-gib", type=float, default=32.0)
    ap.add_argument("--serve-max-batch", type=int, default=0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-queue-edges", type=int, default=1 << 15)
    ap.add_argument("--serve-sustain-frac", type=float, default=0.7)
    ap.add_argument("--serve-sustain-seconds", type=float, default=20.0)
    ap.add_argument("--serve-compare", type=int, default=48)
    ap.add_argument("--serve-omega", type=int, default=64,
                    help="eigenpairs of the serving run's extra offered phase (0: none)")
    ap.add_argument("--mode", choices=["bouquet", "naive"], default="bouquet")
    ap.add_argument("--group", type=int, default=1)
    ap.add_argument("--spread", type=int, default=0)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--walks-log2", type=int, default=24)
    ap.add_argument("--length", type=int, default=64)
    ap.add_argument("--aesc-frac", type=float, default=0.01)
    ap.add_argument("--aesc-eps", type=float, default=0.1)
    ap.add_argument("--aesc-mem-gib", type=float, default=0.0,
                    help="source scratch of the estimator (0: the library default)")
    ap.add_argument("--omega", type=int, default=0,
                    help="eigenpairs of the all-edges estimator run (aesc_full)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="ablation: skip the grouped-bouquet autotuner (counter runs)")
    ap.add_argument("--no-full", action="store_true",
                    help="skip the all-edges estimator pass of the default run")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving leg of the default run")
    ap.add_argument("--serve-short", action="store_true",
                    help="serving: only the offered and sustained phases (the default run's leg)")
    ap.add_argument("--no-omega", action="store_true",
                    help="skip the omega = 64 row of the estimator leg (counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the walk range would be split across GPUs and the histograms summed; "
              "see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2410_14056_amd as saba

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    saba.load()
    if args.workload == "copy":
        # counter calibration: one device-to-device copy of 1 GiB (reads and writes 1 GiB)
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y.copy_(x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"workload": "copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "seconds": dt}), flush=True)
        return
    out = {"metric": METRIC, "value": None, "unit": "walk-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic"}
    if args.workload in ("all", "walks"):
        g, w = bench_walks(args, saba, torch, np)
        out.update({"value": w["value"], "ms_per_step": w["ms_per_step"], "config": w["config"],
                    "roofline": w["roofline"]})
        if w.get("side_by_side"):
            out["walks_side_by_side"] = w["side_by_side"]
        print(json.dumps({"progress": "walks done", "value": w["value"]}), file=sys.stderr, flush=True)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = walks_cpu_baseline(g, args.length, 1)
        del g
    if args.workload == "batch":
        b = bench_batch(args, saba, torch, np)
        out.update({"value": b["batched_edges_per_s"], "unit": "edges/s", "dtype": "f64",
                    "ms_per_step": b["batched_s"] * 1e3, "config": {"workload": b["workload"]},
                    "batch": b})
        print(json.dumps(out), flush=True)
        return
    if args.workload == "aesc_full":
        a = bench_aesc_full(args, saba, torch, np)
        out.update({"value": a["edges_per_s"], "unit": "edges/s", "dtype": "f64",
                    "ms_per_step": a["seconds"] * 1e3, "config": {"workload": a["workload"]},
                    "aesc_full": a})
        print(json.dumps(out), flush=True)
        return
    if args.workload == "ablation":
        a = bench_ablation(args, saba, torch, np)
        head = next(r for r in a["rows"] if "headline" in r["name"])
        out.update({"value": head["walk_steps_per_s"], "ms_per_step": head["ms_per_step"],
                    "config": {"workload": a["workload"]}, "ablation": a})
        print(json.dumps(out), flush=True)
        return
    if args.workload == "walks_paper":
        a = bench_walks_paper(args, saba, torch, np)
        head = next(r for r in a["rows"] if r["steps"] == 15 and r["arrangement"] == "bouquet G=1")
        out.update({"value": head["walk_steps_per_s"], "ms_per_step": head["seconds"] * 1e3,
                    "config": {"workload": a["workload"]}, "walks_paper": a})
        print(json.dumps(out), flush=True)
        return
    if args.workload == "omega":
        a = bench_omega(args, saba, torch, np)
        best = max(a["rows"], key=lambda r: r["edges_per_s"])
        out.update({"value": best["edges_per_s"], "unit": "edges/s", "dtype": "f64",
                    "ms_per_step": best["seconds"] * 1e3, "config": {"workload": a["workload"]},
                    "omega": a})
        print(json.dumps(out), flush=True)
        return
    if args.workload == "serve":
        r = bench_serve(args, saba, torch, np)
        sus = r["sustained"]
        out.update({"metric": METRIC, "value": r["offered"]["edges_per_s"], "unit": "edges/s",
                    "dtype": "f64", "ms_per_step": None, "config": {"workload": r["workload"]},
                    "p50_ms": sus.get("p50_ms"), "p99_ms": sus.get("p99_ms"), "serve": r})
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("all", "er2000"):
        out["er2000"] = bench_er2000(args, saba, torch, np)
        if args.workload == "er2000":
            out.update({"value": out["er2000"]["edges_per_s"], "unit": "edges/s", "dtype": "f64",
                        "ms_per_step": out["er2000"]["latency_ms_median"],
                        "config": {"workload": out["er2000"]["workload"]}})
    if args.workload in ("all", "aesc"):
        a = bench_aesc(args, saba, torch, np)
        out["aesc"] = a
        progress(f"aesc 1% query done: {a['value']:.0f} edges/s")
        if args.workload == "aesc":
            out.update({"value": a["value"], "unit": "edges/s", "dtype": "f64",
                        "ms_per_step": a["seconds"] * 1e3,
                        "config": {"workload": a["workload"]}, "roofline": a["roofline"]})
            if "cpu_baseline" in a:
                out["cpu_baseline"] = a["cpu_baseline"]
    if args.workload == "all" and not args.no_full:
        f = bench_aesc_full(args, saba, torch, np, tuned=out.get("aesc", {}).get("tuned"))
        out["aesc_all_edges"] = f
        progress(f"aesc all edges done: {f['edges_per_s']:.0f} edges/s, sum {f['sum_sc']:.1f} "
                 f"(n - 1 = {f['n_minus_1']})")
    if args.workload == "all" and not args.no_serve:
        args.serve_short = True
        args.serve_sustain_seconds = min(args.serve_sustain_seconds, 10.0)
        r = bench_serve(args, saba, torch, np)
        sus = r["sustained"]
        out["serve"] = r
        out["p50_ms"], out["p99_ms"] = sus.get("p50_ms"), sus.get("p99_ms")
        out["latency_load"] = (f"sustained Poisson load at {sus['offered_rate']:.2f} req/s "
                               f"(70% of the served capacity), {sus['refused']} of "
                               f"{sus['offered']} refused")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
