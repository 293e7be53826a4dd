"""Benchmark: the cell-graph path on the long-vector workload.

One step = dedup (radix sort + unique) -> dictionary build -> distance-1
edges, over 4,613,734 packed rows of 1024 bits (262,144 random bases, each
with 15 one-bit neighbours, plus 10% duplicate rows), already resident in
HBM when the timed region starts.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "distance-1 edges/sec and cells/sec at ℓ=1024, n=4M; % HBM roofline; p99"
HBM_PEAK_GBS = 8000.0
# HBM bytes moved by one cg_edges call on this workload: rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs over one step, each counter scaled by what it
# reads for a plain 512 MiB device copy (FETCH x2, WRITE x1); the per-kernel
# table is in profiles/cg_edges_long_vectors_traffic.md.  It describes the
# kernels as measured: set it to None when the cg_edges kernels change and
# re-measure.
EDGES_TRAFFIC_BYTES = 898521265


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(rows: np.ndarray, n_cells: int, n_edges: int, dedup_rows: int, search_cells: int):
    """The oracle on a bounded sample of the long-vector workload, extrapolated
    to the whole job (a full run takes minutes on the host):

    * sort + unique (the oracle's qsort) of the first `dedup_rows` rows,
      scaled to all rows as n log n;
    * the oracle's Algorithm-4 search form of the edges (every 0 bit of every
      cell flipped and looked up by binary search) over the first
      `search_cells` cells of that sorted sample, scaled to all cells linearly and
      by log2(cells) for the depth of each binary search.
    """
    import oracle
    sub = np.ascontiguousarray(rows[:dedup_rows])
    t0 = time.perf_counter()
    cells_sub, _ = oracle.dedup(sub, 1024, 64)
    t_dedup = time.perf_counter() - t0
    # the sample's sorted cells (rows are shuffled, so these are spread over the whole cell set)
    pool = np.ascontiguousarray(cells_sub[:search_cells])
    t0 = time.perf_counter()
    oracle.edges_search(pool, 1024, 64)
    t_search = time.perf_counter() - t0
    n = rows.shape[0]
    m = pool.shape[0]
    full_dedup = t_dedup * (n * np.log2(n)) / (dedup_rows * np.log2(dedup_rows))
    full_search = t_search * (n_cells / m) * (np.log2(n_cells) / np.log2(m))
    full = full_dedup + full_search
    out = {
        "value": n_edges / full,
        "unit": "edges/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "extrapolated": True,
        "sample": (f"sort+unique of {dedup_rows} of {n} rows ({t_dedup:.2f} s, scaled as n log n) + "
                   f"Algorithm-4 search edges over {m} of {n_cells} sorted cells ({t_search:.2f} s, scaled "
                   f"linearly in cells and by log2 of the cell count); extrapolated whole job {full:.1f} s"),
        "cells_per_s": n_cells / full,
    }
    out.update(cpu_info())
    return out


def small_configs(steps: int, with_cpu: bool):
    """The two small workloads (32 lines in the unit square, 10,000 points;
    128 planes in [-1,1]^3, 10^6 points), whole path from sign bytes on the
    GPU (pack, dedup, dictionary, edges) against the oracle's full run on the
    host cores and on one core; results compared with the oracle's."""
    import torch
    import oracle
    from paper_1503_06029_amd import inputs, pipeline
    out = {}
    for name, gen, ell in (("lines_l32_n10k", inputs.line_arrangement, 32),
                           ("planes_l128_n1M", inputs.plane_arrangement, 128)):
        R = gen()
        n = R.shape[0]
        g = pipeline.CellGraph(n, ell, 32, edge_cap=max(4096, 2 * n))
        bits = torch.from_numpy(np.ascontiguousarray(R)).cuda()
        g.pack(bits)
        g.run_checked()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for k in range(steps):
            g.run_bits(bits)
            ev[k + 1].record()
        torch.cuda.synchronize()
        ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
        res = g.fetch()
        line = {"rows": n, "ell": ell, "cells": res["ncells"], "edges": res["nedges"],
                "gpu_ms_per_step": float(ms.mean()), "gpu_p99_ms": float(np.percentile(ms, 99)),
                "edges_per_s": res["nedges"] / (ms.mean() / 1e3), "cells_per_s": res["ncells"] / (ms.mean() / 1e3)}
        if with_cpu:
            threads = oracle.threads()
            timings = {}
            for th, mode in ((threads, "all-pairs"), (threads, "search"), (1, "search")):
                oracle.set_threads(th)
                t0 = time.perf_counter()
                rows = oracle.pack(R, 32)
                cells, r2c = oracle.dedup(rows, ell, 32)
                uv, bit, off = oracle.edges(cells, 32) if mode == "all-pairs" else oracle.edges_search(cells, ell, 32)
                timings[f"{mode}_{th}t_s"] = time.perf_counter() - t0
            oracle.set_threads(threads)
            line["correct"] = bool(np.array_equal(res["cells"], cells) and np.array_equal(res["row_to_cell"], r2c)
                                   and np.array_equal(res["uv"], uv) and np.array_equal(res["bit"], bit)
                                   and np.array_equal(res["offsets"], off))
            line["oracle"] = {k: round(v, 4) for k, v in timings.items()}
            line["oracle_cores"] = threads
        out[name] = line
        log(f"{name}: {line}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-dedup-rows", type=int, default=400_000)
    ap.add_argument("--cpu-search-cells", type=int, default=131072)
    ap.add_argument("--no-small-configs", action="store_true")
    ap.add_argument("--workload", choices=("long", "batched", "served", "search", "sample", "queries", "paths", "copy"),
                    default="long",
                    help="long: 1024-bit vectors (the headline); batched: 512 plane scenes in one graph; "
                         "served: Poisson stream of those scenes")
    ap.add_argument("--scenes", type=int, default=512)
    ap.add_argument("--no-tune", action="store_true", help="batched: skip the autotuner")
    ap.add_argument("--no-baseline", action="store_true", help="batched: skip the per-scene launch chains")
    ap.add_argument("--key-bits", type=int, default=None, choices=(0, 32, 64, 96),
                    help="long: sort-key width of the fused build (default: timed choice among 0, 32, 64, 96)")
    ap.add_argument("--seconds", type=float, default=5.0, help="served: trace length")
    ap.add_argument("--sampled", action="store_true",
                    help="served: scenes as descriptions sampled on the GPU (no sign bytes over PCIe)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "search":
        return bench_search(args)
    if args.workload == "sample":
        return bench_sample(args)
    if args.workload == "queries":
        return bench_queries(args)
    if args.workload == "paths":
        return bench_paths(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "copy":
        return bench_copy(args)

    import torch
    from paper_1503_06029_amd import binding as B, inputs, pipeline

    log("generating workload")
    rows = inputs.long_vectors()
    n = rows.shape[0]
    want_cells, want_E = inputs.long_vectors_expected()
    dev_rows = pipeline.to_device_words(rows)
    g = pipeline.CellGraph(n, 1024, 64, edge_cap=want_E + 1024, with_bits=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    # the sort-key width of the fused build (cg_dict_params.key_bits): every
    # width gives the same bytes; pick the fastest on this input, as the
    # autotuner does for batch classes
    key_ms = {}
    if args.key_bits is None:
        for kb in (0, 32, 64, 96):
            g.params = B.cg_dict_params_default(key_bits=kb)
            g.dedup_dict(dev_rows)
            t = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            t[0].record(stream)
            for j in range(3):
                g.dedup_dict(dev_rows)
                t[j + 1].record(stream)
            torch.cuda.synchronize()
            key_ms[kb] = min(t[j].elapsed_time(t[j + 1]) for j in range(3))
        key_bits = min(key_ms, key=key_ms.get)
        log(f"key width: {key_ms} ms -> {key_bits}")
    else:
        key_bits = args.key_bits
    g.params = B.cg_dict_params_default(key_bits=key_bits)

    # a step: the fused dedup + dictionary build (cg_dedup_dict: the same
    # cells and dictionary as cg_dedup then cg_dict_build), then cg_edges
    log("warmup")
    for _ in range(args.warmup):
        g.dedup_dict(dev_rows)
        g.edges()
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log("timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        e = ev[k]
        e[0].record(stream)
        g.dedup_dict(dev_rows)
        e[1].record(stream)
        g.edges()
        e[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([e[0].elapsed_time(e[2]) for e in ev])
    dd_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    edges_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])

    nc = int(g.ncells.item())
    E = int(g.nedges.item())
    status = int(g.status.item())
    ok = (nc == want_cells and E == want_E and status == 0)
    ms = float(wall * 1e3 / args.steps)

    # algorithmic bytes of distance-1 + edges: read every cell once, write and
    # read one 8-byte count/offset per cell, write every edge (u, v)
    alg_bytes = nc * 1024 // 8 + 8 * nc + 8 * E
    edges_avg_s = float(edges_ms.mean()) / 1e3
    achieved = alg_bytes / edges_avg_s / 1e9

    out = {
        "metric": METRIC,
        "value": E / (ms / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "long vectors: 4,613,734 packed rows of 1024 bits (262,144 uniform bases x "
                        "(1 + 15 one-bit neighbours), shuffled, +10% duplicate rows), 16 x u64 per row",
            "cells": nc,
            "edges": E,
            "path": "cg_dedup_dict (dedup + dictionary build, fused) then cg_edges",
            "key_bits": key_bits,
            "key_bits_ms": {str(k): v for k, v in key_ms.items()},
        },
        "cells_per_s": nc / (ms / 1e3),
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "step_ms": {"dedup_dict": float(dd_ms.mean()), "edges": float(edges_ms.mean())},
        "correct": ok,
        "roofline": {
            "bound": "hbm",
            "kernel": "cg_edges (distance-1 queries + edge emission)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": EDGES_TRAFFIC_BYTES,
            "alg_bytes": alg_bytes,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(rows, want_cells, want_E, args.cpu_dedup_rows, args.cpu_search_cells)
    if not args.no_small_configs:
        log("small workloads (GPU whole path, oracle in full)")
        out["small_workloads"] = small_configs(20, not args.no_cpu_baseline)
    print(json.dumps(out), flush=True)
    if not ok:
        log(f"WRONG RESULT: cells {nc} (want {want_cells}), edges {E} (want {want_E}), status {status}")
        sys.exit(1)


def scene_pool(k):
    from paper_1503_06029_amd import inputs
    return [inputs.batch_scene(i) for i in range(k)]


def bench_copy(args):
    """A plain 512 MiB device-to-device copy (three of them): the kernel
    whose FETCH_SIZE / WRITE_SIZE counter readings scale those of the
    cell-graph kernels to bytes moved, and a measured HBM copy rate."""
    import torch
    a = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print(json.dumps({"metric": "plain device copy (512 MiB read + 512 MiB written)", "value": 2 * (1 << 29) / ms / 1e6,
                      "unit": "GB/s", "n_gpus": 1, "steps": 3, "warmup": 0, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
                      "data": "synthetic", "config": {"workload": "copy of 536870912 bytes"}}), flush=True)


def bench_batched(args):
    """512 scenes (l uniform in 16..512 planes, log-uniform sample counts) as
    one captured graph, against plain per-scene launch chains."""
    import torch
    from paper_1503_06029_amd import batch, pipeline
    log("generating scenes")
    scenes = scene_pool(args.scenes)
    shapes = [(R.shape[0], R.shape[1]) for R in scenes]
    rows = sum(n for n, _ in shapes)
    runner = batch.BatchRunner(shapes)
    runner.upload(scenes)
    tuned = {}
    t_tune = 0.0
    if not args.no_tune:
        from paper_1503_06029_amd import tuner
        tn = tuner.Tuner(path=None)
        t0 = time.perf_counter()
        for ids, sb in runner.classes:
            best, ms = tn.tune_class(sb)
            tuned[f"w{sb.words}"] = dict(best, ms=round(ms, 3))
            log(f"class w{sb.words}: {best} {ms:.2f} ms")
        t_tune = time.perf_counter() - t0
    runner.run_checked()
    runner.capture()
    for _ in range(args.warmup):
        runner.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        runner.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    cells, edges = runner.totals()
    base_ms, base_edges = None, edges
    if not args.no_baseline:
        base_ms, base_edges = per_scene_baseline(scenes)
    ms = float(step_ms.mean())
    out = {
        "metric": "batched scenes: cell-graph edges/s, one captured graph vs per-scene launches",
        "value": edges / (ms / 1e3), "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{len(scenes)} scenes, l uniform 16..512 planes in R^3, log-uniform 1e3..2e5 "
                               f"points ({rows} rows)", "cells": cells, "edges": edges,
                   "tuned": tuned, "tune_s": round(t_tune, 2)},
        "rows_per_s": rows / (ms / 1e3),
        "p50_ms": float(np.percentile(step_ms, 50)), "p99_ms": float(np.percentile(step_ms, 99)),
        "per_scene_ms": base_ms, "speedup_vs_per_scene": None if base_ms is None else base_ms / ms,
        "correct": base_edges == edges,
    }
    print(json.dumps(out), flush=True)


def per_scene_baseline(scenes):
    """The same scenes as plain per-scene launch chains: (ms, edges)."""
    import torch
    from paper_1503_06029_amd import pipeline
    log("per-scene baseline")
    graphs = []
    for R in scenes:
        g = pipeline.CellGraph(R.shape[0], R.shape[1], 32, edge_cap=max(4096, 4 * R.shape[0]))
        bits = torch.from_numpy(np.ascontiguousarray(R)).cuda()
        graphs.append((g, bits))
    for g, bits in graphs:  # warm up, size buffers
        if bits.shape[0]:
            g.pack(bits)
        g.run_checked()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, bits in graphs:
        if bits.shape[0]:
            g.pack(bits)
        g.run()
    torch.cuda.synchronize()
    base_ms = (time.perf_counter() - t0) * 1e3
    return base_ms, sum(int(g.nedges.item()) for g, _ in graphs)


def bench_served_sampled(args):
    """The served trace with every pool scene given as a description (its
    planes, point count and generator key) and sampled on the GPU inside the
    batch: a request moves a few bytes of scene table, not its sign bytes."""
    from paper_1503_06029_amd import inputs, serve
    log("scene descriptions")
    descs = [inputs.batch_scene_desc(i) for i in range(args.scenes)]
    t, sc = inputs.served_trace(seconds=args.seconds)
    t = np.asarray(t)
    srv = serve.SampledServer(descs, inputs.SAMPLE_BOX)
    srv.serve(np.zeros(8), sc[:8])
    lat, _, wall = srv.serve(t, sc)
    rows = sum(descs[int(i)][1] for i in sc)
    out = {
        "metric": "served scenes sampled on the GPU: requests/s and p50/p99 latency, continuous batching",
        "value": len(t) / wall, "unit": "requests/s", "n_gpus": 1, "steps": len(t), "warmup": 8,
        "ms_per_step": wall * 1e3 / len(t), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+u32", "data": "synthetic",
        "config": {"workload": f"Poisson 2000/s for {args.seconds} s over {len(descs)} scene descriptions "
                               "(l 16..512 planes, 1e3..2e5 points drawn on the GPU)", "requests": int(len(t)),
                   "rows": int(rows)},
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
    }
    print(json.dumps(out), flush=True)


def bench_served(args):
    """Poisson arrivals at 2,000 scenes/s over the scene pool: continuous
    batching against serial per-scene launches; p50/p99 latency."""
    if args.sampled:
        return bench_served_sampled(args)
    import torch
    from paper_1503_06029_amd import inputs, serve
    log("generating scene pool")
    pool = scene_pool(args.scenes)
    t, sc = inputs.served_trace(seconds=args.seconds)
    t = np.asarray(t)
    log(f"{len(t)} requests over {args.seconds} s")
    # without resident dictionaries: every request packs, deduplicates and builds in a batch
    srv = serve.Server(pool, resident_budget=0)
    srv.serve(np.zeros(8), sc[:8])
    lat0, _, wall0 = srv.serve(t, sc)
    del srv
    torch.cuda.empty_cache()
    log("with resident dictionaries")
    srv = serve.Server(pool)
    # warm-up: a short burst
    srv.serve(np.zeros(8), sc[:8])
    lat, _, wall = srv.serve(t, sc)
    pool_stats = {"budget_bytes": srv.pool.budget, "resident_scenes": len(srv.pool.scenes),
                  "resident_bytes": srv.pool.used, "hits": srv.pool.hits, "misses": srv.pool.misses,
                  "evictions": srv.pool.evictions}
    del srv
    torch.cuda.empty_cache()
    log("per-scene baseline")
    base = serve.PerSceneBaseline(pool)
    base.serve(np.zeros(4), sc[:4])
    blat, _, bwall = base.serve(t, sc)
    rows = sum(pool[int(i)].shape[0] for i in sc)
    out = {
        "metric": "served scenes: requests/s and p50/p99 latency, continuous batching vs per-scene launches",
        "value": len(t) / wall, "unit": "requests/s", "n_gpus": 1, "steps": len(t), "warmup": 8,
        "ms_per_step": wall * 1e3 / len(t), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"Poisson 2000/s for {args.seconds} s over {len(pool)} scenes "
                               "(l 16..512, 1e3..2e5 points)", "requests": int(len(t)), "rows": int(rows)},
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        # past the first second: every scene has been seen (resident dictionaries built)
        "p99_after_1s_ms": float(np.percentile(lat[t >= 1.0], 99) * 1e3),
        "resident": pool_stats,
        "no_resident": {"requests_per_s": len(t) / wall0, "p50_ms": float(np.percentile(lat0, 50) * 1e3),
                        "p99_ms": float(np.percentile(lat0, 99) * 1e3),
                        "p99_after_1s_ms": float(np.percentile(lat0[t >= 1.0], 99) * 1e3)},
        "baseline": {"requests_per_s": len(t) / bwall, "p50_ms": float(np.percentile(blat, 50) * 1e3),
                     "p99_ms": float(np.percentile(blat, 99) * 1e3)},
    }
    print(json.dumps(out), flush=True)


def bench_search(args):
    """Search on the cell graph of the plane arrangement (10^6 points, 128
    planes): undirected CSR from the edge list, then a breadth-first search
    from cell 0 over all levels (at most l + 1: in an arrangement the hop
    count equals the number of separating planes), captured as one graph."""
    import torch
    from paper_1503_06029_amd import inputs, pipeline
    log("generating the plane-arrangement scene")
    R = inputs.plane_arrangement()
    ell = R.shape[1]
    g = pipeline.CellGraph(R.shape[0], ell, 32, edge_cap=1_100_000)
    g.pack(torch.from_numpy(np.ascontiguousarray(R)).cuda())
    g.run_checked()
    nc, E = int(g.ncells.item()), int(g.nedges.item())
    S = pipeline.GraphSearch(g)
    levels = ell + 2
    S.build()
    S.bfs(0, levels)
    torch.cuda.synchronize()
    eager = S.fetch()
    S.capture(0, levels)
    for _ in range(args.warmup):
        S.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        S.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    got = S.fetch()
    # the search alone (levels only), eager, timed on the stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bfs_ms = []
    for _ in range(5):
        e0.record()
        S.bfs(0, levels)
        e1.record()
        torch.cuda.synchronize()
        bfs_ms.append(e0.elapsed_time(e1))
    reached = got["dist"] != 0xFFFFFFFF
    traversed = int(np.diff(got["adj_off"])[reached].sum())
    ok = (got["status"] == 0 and np.array_equal(got["dist"], eager["dist"]) and
          np.array_equal(got["parent"], eager["parent"]))
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        uv = g.uv[:E].cpu().numpy().view(np.uint32)
        t0 = time.perf_counter()
        dist, parent, far = oracle.bfs(nc, uv, 0)
        cpu_s = time.perf_counter() - t0
        ok = ok and np.array_equal(dist, got["dist"]) and np.array_equal(parent, got["parent"])
        cpu = {"value": traversed / cpu_s, "unit": "traversed edges/s", "cores": 1, "kind": "oracle",
               "sample": f"whole search: adjacency lists + BFS from cell 0 ({cpu_s:.3f} s)"}
    ms = float(step_ms.mean())
    # algorithmic bytes of the search: adjacency lists and offsets read once,
    # one 4-byte distance read per list entry, distance, parent and frontier
    # entries written once per reached cell
    alg = 4 * traversed + 8 * (nc + 1) + 4 * traversed + 16 * int(reached.sum())
    bms = float(np.median(bfs_ms))
    out = {
        "metric": "cell-graph search: BFS traversed edges/s (CSR build + full search, one captured graph)",
        "value": traversed / (ms / 1e3), "unit": "traversed edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"plane arrangement: {R.shape[0]} points in [-1,1]^3, {ell} planes, {nc} cells, "
                               f"{E} edges; BFS from cell 0", "cells": nc, "edges": E, "levels": got["levels"],
                   "launched_levels": levels},
        "bfs_only_ms": bms, "csr_plus_bfs_ms": ms,
        "roofline": {"bound": "hbm", "kernel": "k_bfs_level (all levels of one search)", "achieved": alg / (bms / 1e3) / 1e9,
                     "peak": 8000.0, "unit": "GB/s", "frac": alg / (bms / 1e3) / 8e12, "traffic": None,
                     "alg_bytes": alg},
        "cpu_baseline": cpu,
        "correct": bool(ok),
    }
    print(json.dumps(out), flush=True)


def bench_sample(args):
    """Sampling fused with packing at the plane-arrangement shape (10^6 points in
    [-1, 1]^3, 128 planes): points drawn and signs evaluated on the GPU and
    written as packed rows, against the host route (sign bytes made on the
    host, copied from pinned memory, then packed on the GPU)."""
    import torch
    from paper_1503_06029_amd import binding as B, pipeline
    n, ell, seed, scene = 1_000_000, 128, 150306029, 1
    rng = np.random.default_rng(seed)
    gnorm = rng.standard_normal((ell, 3))
    planes = np.concatenate([gnorm / np.linalg.norm(gnorm, axis=1, keepdims=True),
                             rng.uniform(-0.5, 0.5, ell)[:, None]], axis=1)
    box = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    d_planes = torch.from_numpy(planes).cuda()
    g = pipeline.CellGraph(n, ell, 32, edge_cap=1_100_000)
    for _ in range(args.warmup):
        g.sample(d_planes, seed, scene, box)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        g.sample(d_planes, seed, scene, box)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]))
    # the whole path from the sampler: sample + dedup + dictionary + edges
    g.sample(d_planes, seed, scene, box)
    g.run_checked()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    path_ms = []
    for _ in range(5):
        e0.record()
        g.sample(d_planes, seed, scene, box)
        g.run()
        e1.record()
        torch.cuda.synchronize()
        path_ms.append(e0.elapsed_time(e1))
    nc, E = int(g.ncells.item()), int(g.nedges.item())
    # host route: the same signs as bytes, pinned, copied and packed
    import oracle
    t0 = time.perf_counter()
    sample_rows = 200_000
    oracle.sample_signs(planes, sample_rows, seed, scene, box)
    cpu_s = time.perf_counter() - t0
    bits = oracle.sample_signs(planes, n, seed, scene, box)
    want = oracle.pack(bits[:20000], 32)
    ok = np.array_equal(g.packed[:20000].cpu().numpy().view(np.uint32), want)
    pinned = torch.from_numpy(bits).pin_memory()
    dev_bits = torch.empty_like(pinned, device="cuda")
    host_ms = []
    for _ in range(5):
        e0.record()
        dev_bits.copy_(pinned, non_blocking=True)
        g.pack(dev_bits)
        e1.record()
        torch.cuda.synchronize()
        host_ms.append(e0.elapsed_time(e1))
    ops = 7 * ell * n  # per plane: three products, two sums, the offset, the comparison (float64)
    peak_ops = 256 * 64 * 2.4e9
    out = {
        "metric": "sampled rows/s: points drawn, signs evaluated and packed on the GPU (no sign bytes)",
        "value": n / (ms / 1e3), "unit": "rows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n} points uniform in [-1,1]^3 (Philox4x64-10), {ell} planes, packed 4 x u32",
                   "cells": nc, "edges": E},
        "path_from_sampler_ms": float(np.median(path_ms)),
        "host_route_ms": float(np.median(host_ms)),
        "host_route": "128 MB of sign bytes copied from pinned host memory, then cg_pack",
        "roofline": {"bound": "alu", "kernel": "k_sample_pack", "achieved": ops / (ms / 1e3) / 1e12,
                     "peak": peak_ops / 1e12, "unit": "Tops/s (float64, unfused)", "frac": ops / (ms / 1e3) / peak_ops,
                     "traffic": None},
        "cpu_baseline": {"value": sample_rows / cpu_s, "unit": "rows/s", "cores": int(oracle.threads()),
                         "kind": "oracle", "sample": f"{sample_rows} of {n} points ({cpu_s:.3f} s)"},
        "correct": bool(ok),
    }
    print(json.dumps(out), flush=True)


def bench_queries(args):
    """Resident dictionary over the long-vector cells (4,194,304 cells of
    1,024 bits): batches of membership + distance-1 queries (half cells,
    half one-position flips of cells), a served trace of query requests with
    continuous batching, and an insert-by-rebuild of 1 % new rows."""
    import torch
    from paper_1503_06029_amd import inputs, pipeline, service
    log("generating workload")
    rows = inputs.long_vectors()
    n, W = rows.shape
    ell = 1024
    svc = service.DictService(ell, 64, capacity=n + n // 100 + 1024)
    svc.build(pipeline.to_device_words(rows))
    nc = svc.n
    cells = svc.cells[:nc]
    rng = np.random.default_rng(7)
    m = 1 << 16

    def make_queries(k):
        idx = torch.from_numpy(rng.integers(0, nc, k)).cuda()
        q = cells[idx].clone()
        f = torch.from_numpy(rng.integers(0, ell, k // 2)).cuda()
        rows_ = torch.arange(k // 2, device="cuda")
        bit = (torch.ones(k // 2, dtype=torch.int64, device="cuda") << (63 - f % 64))
        q[rows_, f // 64] ^= bit
        return q

    q = make_queries(m)
    me = torch.empty(m, dtype=torch.int32, device="cuda")
    cnt = torch.empty(m, dtype=torch.int32, device="cuda")
    mask = torch.empty((m, W), dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        svc.query(q, me, cnt, mask)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        svc.query(q, me, cnt, mask)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]))
    # probe bytes of the timed batch: per query its row, its own bucket's
    # directory entries and every cell row of that bucket, and the directory
    # entries of the p flips inside the directory bits; per query out: mask,
    # id and count
    pbits = int(svc.dict.params.dir_bits)
    dir_h = svc.dict_mem[:4 * ((1 << pbits) + 1)].cpu().numpy().view(np.uint32)
    heads = q[:, 0].cpu().numpy().view(np.uint64)
    g = (heads >> np.uint64(64 - pbits)).astype(np.int64) if pbits else np.zeros(m, np.int64)
    bucket = (dir_h[g + 1].astype(np.int64) - dir_h[g].astype(np.int64))
    probe_bytes = int(m * (8 * W + 8 + 8 * pbits) + 8 * W * bucket.sum())
    out_bytes = m * (8 * W + 8)
    # check a sample against the oracle
    import oracle
    hs = 2000
    hq = q[:hs].cpu().numpy().view(np.uint64)
    hcells = cells.cpu().numpy().view(np.uint64)
    t0 = time.perf_counter()
    want_cnt, want_self, want_mask = oracle.d1_queries(hcells, hq, 64)
    cpu_s = time.perf_counter() - t0
    ok = (np.array_equal(me[:hs].cpu().numpy().view(np.uint32), want_self) and
          np.array_equal(cnt[:hs].cpu().numpy().view(np.uint32), want_cnt) and
          np.array_equal(mask[:hs].cpu().numpy().view(np.uint64), want_mask))
    # served trace: requests of 64 queries, Poisson arrivals
    rate, secs, k_req = 20000.0, 2.0, 64
    arr = np.cumsum(rng.exponential(1.0 / rate, int(rate * secs)))
    pool = make_queries(1 << 14).cpu().numpy().view(np.uint64)
    reqs = [pool[(i * k_req) % pool.shape[0]:(i * k_req) % pool.shape[0] + k_req] for i in range(len(arr))]
    srv = service.QueryServer(svc, max_batch=1 << 16)
    srv.serve(arr[:50] - arr[0], reqs[:50])
    lat, _, wall = srv.serve(arr, reqs)
    # insert-by-rebuild of 1 % new rows (fresh random vectors)
    new = torch.from_numpy(rng.integers(0, 2 ** 63, (n // 100, W), dtype=np.int64)).cuda()
    t0 = time.perf_counter()
    svc.insert(new)
    ins_s = time.perf_counter() - t0
    alg = probe_bytes + out_bytes
    out = {
        "metric": "resident-dictionary queries/s (membership + all one-position flips per query)",
        "value": m / (ms / 1e3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"dictionary over {nc} cells of {ell} bits (long-vector workload); batches of {m} "
                               "queries, half cells and half one-position flips of cells", "cells": nc},
        "flips_per_s": m * ell / (ms / 1e3),
        "served": {"requests_per_s": len(arr) / wall, "offered_per_s": rate, "queries_per_request": k_req,
                   "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)},
        "insert_rebuild_s": ins_s, "inserted_rows": int(n // 100), "cells_after_insert": svc.n,
        "roofline": {"bound": "hbm", "kernel": "k_d1_bucket", "achieved": alg / (ms / 1e3) / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": alg / (ms / 1e3) / 8e12, "traffic": None, "alg_bytes": alg,
                     "mean_bucket_cells": float(bucket.mean()),
                     "note": "query rows, directory entries (own bucket and the p prefix flips) and every cell "
                             "row of the query's bucket read; masks, ids and counts written"},
        "cpu_baseline": {"value": hs / cpu_s, "unit": "queries/s", "cores": int(oracle.threads()),
                         "kind": "oracle", "sample": f"{hs} queries by full scan of the cells ({cpu_s:.2f} s)"},
        "correct": bool(ok),
    }
    print(json.dumps(out), flush=True)


# integer lane-op peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit op per lane per cycle
INT_LANE_OPS_PEAK = 256 * 64 * 2.4e9


def bench_paths(args):
    """The three edge paths on one dictionary (the plane arrangement: 10^6
    points, 128 planes -> 85,032 cells): flip-and-look-up, the (*)-pruned
    all-pairs scan of Section 3.1 (h = 0 and 4 references) and the O(n l)
    additive-hash probes.  The all-pairs scan is bound by the integer ALUs:
    its line counts pair tests per second and the filter's lane operations
    (3 per reference per pair: subtract, compare, and) against the integer
    lane-op peak; the exact test of the few surviving pairs is not counted."""
    import torch
    from paper_1503_06029_amd import binding as B, inputs, pipeline
    log("generating the plane-arrangement scene")
    R = inputs.plane_arrangement()
    ell = R.shape[1]
    bits = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    out = {}
    ref = None
    for name, kw in (("lookup", dict()), ("allpairs_h0", dict(path=B.CG_PATH_ALLPAIRS, n_refs=0)),
                     ("allpairs_h4", dict(path=B.CG_PATH_ALLPAIRS, n_refs=4)), ("hash", dict(path=B.CG_PATH_HASH))):
        g = pipeline.CellGraph(R.shape[0], ell, 32, params=B.cg_dict_params_default(**kw), edge_cap=1_100_000)
        g.pack(bits)
        g.run_checked()
        nc, E = int(g.ncells.item()), int(g.nedges.item())
        uv = g.uv[:E].cpu().numpy()
        same = ref is None or np.array_equal(uv, ref)
        ref = uv if ref is None else ref
        steps = max(3, args.steps // (20 if name.startswith("allpairs") else 1))
        for _ in range(2):
            g.edges()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            g.edges()
            ev[k + 1].record()
        torch.cuda.synchronize()
        ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
        rec = {"edges_ms": ms, "cells": nc, "edges": E, "same_bytes_as_lookup": bool(same)}
        if name.startswith("allpairs"):
            h = kw["n_refs"]
            pairs = nc * (nc - 1) / 2
            rec["pair_tests_per_s"] = pairs / (ms / 1e3)
            if h:
                ops = 3 * h * pairs / (ms / 1e3)
                rec["filter_lane_ops_per_s"] = ops
                rec["roofline"] = {"bound": "alu", "achieved": ops / 1e12, "peak": INT_LANE_OPS_PEAK / 1e12,
                                   "unit": "Tops/s", "frac": ops / INT_LANE_OPS_PEAK}
        if name == "hash":
            rec["probes_per_s"] = nc * ell / 2 / (ms / 1e3)
        out[name] = rec
        log(f"{name}: {ms:.3f} ms, {E} edges, same bytes {same}")
        del g
        torch.cuda.empty_cache()
    line = {"metric": "edge paths on one dictionary: lookup, (*)-pruned all-pairs, O(n l) hash probes",
            "value": out["allpairs_h4"]["pair_tests_per_s"], "unit": "pair tests/s (all-pairs, h = 4)",
            "n_gpus": 1, "steps": args.steps, "warmup": 2, "ms_per_step": out["allpairs_h4"]["edges_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "plane arrangement: 10^6 points, 128 planes in [-1, 1]^3",
                       "cells": out["lookup"]["cells"], "edges": out["lookup"]["edges"]},
            "roofline": out["allpairs_h4"].get("roofline"), "paths": out,
            "correct": all(v["same_bytes_as_lookup"] for v in out.values())}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
