#!/usr/bin/env python3
"""Throughput benchmark of the batched K-Best GED search on one MI355X.

A step is one batched search (every level of every pair: expand and
evaluate, select the best K, update the beam, complete and pick the best
leaf) over the whole synthetic batch, already resident in HBM, followed by a
stream synchronize.  Default workload: 4096 pairs of Erdos-Renyi graphs,
n ~ U{10..30}, p ~ U[0.1, 0.3], 5 vertex labels, unit costs, K = 64.

Prints one JSON line: batched pairs/s (`value`), the per-pair-launch
baseline at the same K, the roofline of the search kernel, the CPU oracle's
throughput on the host cores, and whether every GPU result matched the
oracle bit for bit.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GED pairs/sec at K=64 batched vs per-pair on 1 GPU; serving p50/p99 latency"

# The serving measurement runs SERVE_STREAMS streams per size class.  Streams
# that share one of the process's hardware queues run one after another (a
# long large-query launch then blocks the small queries behind it), and HIP's
# default is 4 queues per process, so the bench asks for enough queues before
# the runtime starts.
SERVE_STREAMS = 4
# four size classes x 4 streams (the large class twice that) need queues of their
# own, and the process holds other streams as well (torch's, the runtime's): with
# exactly 17 queues a mid-size stream still shared a queue with a large-query
# stream (mid p99 55-58 ms at half load).  With 32 queues and the server's batch
# formation and residency caps, the mid class's p99 stays near 1.4 ms at 0.8 of
# saturation; the large class, whose launches last tens of milliseconds, sets the
# overall p99 there
HW_QUEUES = 32
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < HW_QUEUES:
    os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)
# int32 VALU peak of MI355X: 256 CUs x 64 lanes x 2.4 GHz, one op per lane per clock
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12


def ops_per_candidate(w: int, planes: int) -> int:
    """Algorithmic int32 operations per evaluated child (bitset formulation).

    Two AND+popcount per target-row word (edges kept, edges into the image),
    with edge labels one XOR/OR per plane word plus one AND+popcount per word,
    10 for the vertex-label test and cost combination, 6 for selection
    (threshold compare, tie rank, compaction).
    """
    lab = 2 * w * (planes + 1) if planes > 0 else 0
    return 4 * w + lab + 16


# the files each kernel is compiled from (names in csrc/, or paths from the repository root)
KERNEL_SOURCES = {"kb_wave_kernel": ("kb_wave.hip", "wave_common.h", "ged_types.h"),
                  "kb_wave2_kernel": ("kb_wave2.h", "kb_wave2.hip", "kb_wave2_k128.hip", "kb_wave2_src128.hip",
                                      "wave_common.h", "ged_types.h", "ged_internal.h", "include/ged.h"),
                  "kb_block_kernel": ("kb_block.hip", "ged_internal.h", "ged_types.h", "include/ged.h")}


def kernel_source_hash(kernel: str) -> str:
    """sha256 over the sources the kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        path = os.path.join(ROOT, f) if "/" in f else os.path.join(ROOT, "paper_2605_00830_amd", "csrc", f)
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter runs (profiles/traffic.json),
    or None when there are none for this kernel and workload or the kernel's
    sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    with open(path) as fh:
        entries = json.load(fh)
    for e in entries:
        if e["kernel"] == kernel and e["workload"] == workload and e["source_sha256"] == kernel_source_hash(kernel):
            return e
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def oracle_mod():
    import oracle
    return oracle


def cpu_oracle(graphs, pairs, costs, K, threads: int, last_complete: bool = False, directed: bool = False):
    """Run the CPU oracle over `pairs` with `threads` threads (ctypes releases the GIL)."""
    import oracle
    oracle._load()
    shards = [np.arange(t, len(pairs), threads) for t in range(threads)]
    results = [None] * threads

    def work(t):
        results[t] = oracle.kbest_pairs(graphs, pairs[shards[t]], costs, K, last_complete=last_complete,
                                        directed=directed)

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    wall = time.perf_counter() - t0
    dist = np.zeros(len(pairs), np.int64)
    n_src = np.asarray(graphs.n, np.int64)[pairs[:, 0]]
    off = np.zeros(len(pairs), np.int64)
    if len(pairs) > 1:
        np.cumsum(n_src[:-1], out=off[1:])
    maps = np.zeros(int(n_src.sum()), np.int32)
    for t in range(threads):
        d, m, o = results[t]
        dist[shards[t]] = d
        for k, p in enumerate(shards[t]):
            maps[off[p]:off[p] + n_src[p]] = m[o[k]:o[k] + n_src[p]]
    return wall, dist, maps


def serve_measure(ged, w, n_queries: int, fracs=(0.8,), perpair_queries: int = 2000, seed: int = 7,
                  streams: int = 1, method: int = 0):
    """Serving on the mix workload: saturated throughput (closed loop), then
    Poisson arrivals at fractions of it; latency = completion - scheduled
    arrival.  The same loop with one launch per query is the per-pair path.
    method 1 serves the bipartite method, on the queries whose pair has
    n1 + n2 <= 256 (its limit)."""
    ndb = w.meta["ndb"]
    directed = bool(w.meta.get("directed", False))
    nq = min(n_queries, len(w.pairs))
    db = ged.Database(w.graphs.slice(0, ndb), directed=directed)
    qgs = w.graphs.slice(ndb, ndb + nq)
    recs, keep = ged.pack_queries(qgs)
    targets = np.ascontiguousarray(w.pairs[:nq, 1])

    def run(srv, idx, arrivals=None):
        """Submit queries idx (at arrivals, monotonic ns, or as fast as possible).

        One producer thread submits; the server numbers accepted queries
        consecutively, so query k of this run has ticket base + k."""
        n = len(idx)
        t_sub = np.zeros(n, np.int64)
        t_done = np.zeros(n, np.int64)
        base = []
        err = []

        def producer():
            try:
                k = 0
                while k < n:
                    hi = n
                    if arrivals is not None:
                        now = time.monotonic_ns()
                        hi = int(np.searchsorted(arrivals, now, side="right"))
                        if hi <= k:
                            time.sleep(max(0.0, min(2e-4, (arrivals[k] - now) * 1e-9)))
                            continue
                    hi = min(hi, k + 4096)
                    tk = srv.submit_batch(recs[idx[k:hi]], targets[idx[k:hi]])
                    if len(tk) and not base:
                        base.append(int(tk[0]) - k)
                    k += len(tk)
                    if len(tk) == 0:
                        time.sleep(1e-4)
            except Exception as e:  # reported by the caller
                err.append(e)

        th = threading.Thread(target=producer)
        th.start()
        got = 0
        while got < n and not err:
            r = srv.collect(max_count=8192, timeout_us=200_000)
            if r is None:
                continue
            tk, d, times, _ = r
            while not base:            # collected before the producer recorded the first ticket
                time.sleep(1e-5)
            i = tk.astype(np.int64) - base[0]
            t_sub[i] = times[:, 0]
            t_done[i] = times[:, 1]
            got += len(tk)
        th.join()
        if err:
            raise err[0]
        return t_sub, t_done

    # the server's size classes: small (both orders <= 32) and mid (<= 64) for K <= 64,
    # medium (<= 128), large; bipartite: n1 + n2 <= 64, 128, 192, 256
    n_q = np.asarray(qgs.n, np.int64)
    n_t = np.asarray(w.graphs.n, np.int64)[targets]
    n_max = np.maximum(n_q, n_t)
    wave = w.K <= 64
    if method == 1:
        cls = (n_q + n_t + 63) // 64 - 1
        sel = np.nonzero(n_q + n_t <= 256)[0]
        class_names = ("le64", "le128", "le192", "le256")
    elif directed:
        # directed: pairs of up to 32 vertices on the two-word kernel (class 1), then
        # up to 128, then up to 256 (the directed limit)
        cls = np.where(wave & (n_max <= 32), 1, np.where(n_max <= 128, 2, 3))
        sel = np.nonzero(n_max <= 256)[0]
        class_names = ("none", "small", "medium", "large")
    else:
        cls = np.where(wave & (n_max <= 32), 0, np.where(wave & (n_max <= 64), 1, np.where(n_max <= 128, 2, 3)))
        sel = np.arange(nq)
        class_names = ("small", "mid", "medium", "large")

    def latency_stats(t_done, arrivals, idx=None):
        lat = (t_done - arrivals) / 1e6
        c = cls[idx] if idx is not None else cls[:len(lat)]
        skip = len(lat) // 100               # first 1% is warm-up
        lat, c = lat[skip:], c[skip:]
        out = {"p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
               "p999_ms": round(float(np.percentile(lat, 99.9)), 4), "mean_ms": round(float(lat.mean()), 4)}
        per = {}
        for k, name in enumerate(class_names):
            x = lat[c == k]
            if len(x):
                per[name] = {"queries": int(len(x)), "p50_ms": round(float(np.percentile(x, 50)), 4),
                             "p99_ms": round(float(np.percentile(x, 99)), 4)}
        out["by_class"] = per
        return out

    out = {"config": {"workload": w.name, "database_graphs": ndb, "queries": int(len(sel)), "K": w.K,
                      "costs": list(w.costs), "streams_per_class": streams,
                      "method": "bipartite" if method == 1 else "tree", "directed": directed,
                      "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")}}
    srv = ged.Server(db, w.K, w.costs, hbm_budget=8 << 30, streams=streams, max_batch=2048, max_inflight=8192,
                     method=method)
    warm = sel[:min(2000, len(sel))]
    run(srv, warm)
    idx = sel
    nq = len(idx)
    ts, td = run(srv, idx)
    qps_sat = nq / ((td.max() - ts.min()) / 1e9)
    out["saturated_qps"] = round(qps_sat, 1)
    log(f"serving: saturated {qps_sat:.0f} queries/s over {nq} queries")
    rng = np.random.default_rng(seed)
    out["open_loop"] = []
    for f in fracs:
        lam = f * qps_sat
        gaps = rng.exponential(1.0 / lam, nq)
        t0 = time.monotonic_ns() + 20_000_000
        arrivals = t0 + np.cumsum(gaps * 1e9).astype(np.int64)
        ts, td = run(srv, idx, arrivals)
        achieved = nq / ((td.max() - arrivals[0]) / 1e9)
        entry = {"load": f, "offered_qps": round(lam, 1), "achieved_qps": round(achieved, 1)}
        entry.update(latency_stats(td, arrivals, idx))
        out["open_loop"].append(entry)
        log(f"serving at {f:.2f} x saturated: {entry}")
    out["server_stats"] = srv.stats()
    srv.close()
    # per-pair path: one launch per query, same loop
    pp = ged.Server(db, w.K, w.costs, hbm_budget=4 << 30, streams=1, max_batch=1, max_inflight=1, method=method)
    pidx = sel[:min(perpair_queries, nq)]
    ts, td = run(pp, pidx)
    qps_pp = len(pidx) / ((td.max() - ts.min()) / 1e9)
    lam = fracs[0] * qps_sat
    entry = {"saturated_qps": round(qps_pp, 1), "queries": int(len(pidx)), "offered_qps": round(lam, 1)}
    if qps_pp < lam:
        entry["saturated_at_offered_load"] = True
    else:
        gaps = rng.exponential(1.0 / lam, len(pidx))
        t0 = time.monotonic_ns() + 20_000_000
        arrivals = t0 + np.cumsum(gaps * 1e9).astype(np.int64)
        ts, td = run(pp, pidx, arrivals)
        entry.update(latency_stats(td, arrivals, pidx))
    out["perpair"] = entry
    log(f"serving per-pair path: {entry}")
    pp.close()
    db.close()
    return out


# The paper's single-pair runtimes on an A100 (other hardware: context only):
# runtime versus K for two 20-vertex graphs, and K = 5000 at 500 vertices.
LARGE_K_RUNS = [(20, 6, 1000, 35.0), (20, 6, 100_000, 120.0), (20, 6, 700_000, 473.0),
                (20, 6, 1_200_000, 780.0), (500, 7, 5000, 428.0), (950, 8, 5000, 1000.0)]
# the oracle's results on these pairs, written by tests/golden/make_digests.py --large-k
LARGE_K_ORACLE = os.path.join(ROOT, "tests", "golden", "large_k.json")
# CPU baseline of the single-pair search: the oracle on one of the shapes above
LARGE_K_CPU = (20, 6, 100_000)


def large_k_measure(ged, reps: int = 5, cpu: bool = True):
    """Single-pair large-K search (ged_wide_*) on the paper's runtime shapes: median of
    `reps` timed runs (HIP events on the launch stream) after one warm-up run; parity
    with the oracle's stored result where there is one; the roofline of a run: its
    children at ops_per_candidate(target words, planes) each over its duration against
    the int32 VALU peak, and its candidate-matrix bytes (each child's PED written once
    and read back by the count and compaction passes, 12 B) against HBM bandwidth."""
    import torch
    from paper_2605_00830_amd import synth
    stored = json.load(open(LARGE_K_ORACLE)) if os.path.exists(LARGE_K_ORACLE) else {}
    out = []
    for n, seed, K, paper_ms in LARGE_K_RUNS:
        w = synth.pair_er_large_k(n, seed)
        db = ged.Database(w.graphs)
        wide = ged.Wide(db, 0, 1, K)
        dist, maps, cand = wide.outputs()
        s = torch.cuda.current_stream()
        wide.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            wide.run(w.costs, dist, maps, cand, stream=s)
            e1.record(s)
            s.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        ce = int(cand.item())
        d_gpu = int(dist.item())
        m_gpu = maps[:n].cpu().numpy()
        words = (n + 31) // 32
        ops = float(ce) * ops_per_candidate(words, 0)
        ach = ops / (ms / 1e3) / 1e12
        entry = {"workload": w.name, "n": n, "K": K, "costs": list(w.costs), "ms": round(ms, 3),
                 "dist": d_gpu, "children_evaluated": ce, "ce_per_s": round(ce / (ms / 1e3), 1),
                 "workspace_bytes": wide.bytes, "paper_a100_ms": paper_ms,
                 "ratio_to_paper_a100": round(paper_ms / ms, 1),
                 "roofline": {"bound": "alu", "achieved": round(ach, 4), "peak": round(PEAK_INT32_TOPS, 2),
                              "unit": "Tops/s", "frac": round(ach / PEAK_INT32_TOPS, 5),
                              "ops_per_child": ops_per_candidate(words, 0),
                              "candidate_bytes_gbps": round(12.0 * ce / (ms / 1e3) / 1e9, 1),
                              "candidate_bytes_frac_of_hbm": round(12.0 * ce / (ms / 1e3) / 8.0e12, 5)}}
        ref = stored.get(f"{w.name}@K{K}")
        if ref is not None:
            entry["parity"] = {"oracle": "tests/golden/large_k.json",
                               "bit_exact": bool(ref["dist"] == d_gpu and ref["children"] == ce and
                                                 np.array_equal(np.asarray(ref["map"], np.int32), m_gpu))}
        else:
            entry["parity"] = "parity unpinned: no stored oracle result for this shape"
        out.append(entry)
        log(f"large K: n={n} K={K}: {ms:.3f} ms, {ce / (ms / 1e3):.3e} children/s, parity {entry['parity']}")
        wide.close()
        db.close()
    if cpu:
        # the oracle (one thread: it is one pair) on one of the shapes
        import oracle
        n, seed, K = LARGE_K_CPU
        w = synth.pair_er_large_k(n, seed)
        t0 = time.perf_counter()
        d, m, _, c = oracle.kbest_pairs(w.graphs, w.pairs, w.costs, K, with_cand=True)
        sec = time.perf_counter() - t0
        cb = {"value": round(1.0 / sec, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
              "sample": f"{w.name} at K={K}: {int(c[0])} children in {sec:.2f} s",
              "children_per_s": round(int(c[0]) / sec, 1)}
    else:
        cb = None
    return {"runs": out, "cpu_baseline": cb}


# int32 operations per column relaxation of the bipartite method's solver
# step: the reduced cost (two subtractions), the tentative-distance compare and
# two selects (distance, predecessor), the open-column term of the minimum,
# and the potential or distance update (two)
BIP_OPS_PER_RELAX = 8


def cpu_oracle_bip(graphs, pairs, costs, K, threads: int):
    """The bipartite oracle over `pairs` with `threads` threads: (wall, dist, maps, solves, steps)."""
    import oracle
    oracle._load()
    shards = [np.arange(t, len(pairs), threads) for t in range(threads)]
    results = [None] * threads

    def work(t):
        results[t] = oracle.bipartite_pairs(graphs, pairs[shards[t]], costs, K, with_steps=True)

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    wall = time.perf_counter() - t0
    n_src = np.asarray(graphs.n, np.int64)[pairs[:, 0]]
    off = np.zeros(len(pairs), np.int64)
    if len(pairs) > 1:
        np.cumsum(n_src[:-1], out=off[1:])
    dist = np.zeros(len(pairs), np.int64)
    solves = np.zeros(len(pairs), np.int64)
    steps = np.zeros(len(pairs), np.int64)
    maps = np.zeros(int(n_src.sum()), np.int32)
    for t in range(threads):
        d, m, o, sv, st = results[t]
        dist[shards[t]] = d
        solves[shards[t]] = sv
        steps[shards[t]] = st
        for k, p in enumerate(shards[t]):
            maps[off[p]:off[p] + n_src[p]] = m[o[k]:o[k] + n_src[p]]
    return wall, dist, maps, solves, steps


def bipartite_measure(ged, db, w, steps: int, warmup: int, tune: bool, tune_cache):
    """The same batch by the bipartite K-best-assignment method: pairs/s and
    kernel time of its plan; parity and the roofline come from the oracle leg."""
    import torch
    P = len(w.pairs)
    plan = ged.Plan(db, w.pairs, w.K, method=ged.METHOD_BIPARTITE)
    dist, maps, cand = plan.outputs(with_cand=True)
    s = torch.cuda.current_stream()
    plan.set_timing(True)
    if tune:
        plan.tune(w.costs, dist, maps, stream=s, cache_path=tune_cache)
        s.synchronize()
    for _ in range(warmup):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
    ks = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
        ks.append(plan.kernel_ms())
    wall = time.perf_counter() - t0
    out = {"value": round(P * steps / wall, 2), "unit": "pairs/s", "ms_per_step": round(wall * 1e3 / steps, 4),
           "kernel_ms": round(float(np.mean(ks)), 4), "bins": plan.bins(), "K": w.K,
           "assignment_solves": int(cand[:P].sum().item())}
    log(f"bipartite: kernel {out['kernel_ms']} ms, {out['value']:.0f} pairs/s")
    d = dist[:P].cpu().numpy().astype(np.int64)
    m = maps[:plan.map_size].cpu().numpy()
    c = cand[:P].cpu().numpy()
    plan.close()
    return out, d, m, c


def complete_measure(ged, db, w, steps: int, warmup: int, literal_dist, tune: bool, tune_cache):
    """The batch with the complete-then-minimum last level (Sec. 4.4.1 applied to
    every child of the last level): kernel time of the same plan shape, and how
    often and by how much the distance falls below the default search's."""
    import torch
    P = len(w.pairs)
    plan = ged.Plan(db, w.pairs, w.K, last_level=ged.LAST_COMPLETE)
    dist, maps, cand = plan.outputs(with_cand=True)
    s = torch.cuda.current_stream()
    plan.set_timing(True)
    if tune:
        plan.tune(w.costs, dist, maps, stream=s, cache_path=tune_cache)
        s.synchronize()
    for _ in range(warmup):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
    ks = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
        ks.append(plan.kernel_ms())
    wall = time.perf_counter() - t0
    d = dist[:P].cpu().numpy().astype(np.int64)
    lit = np.asarray(literal_dist, np.int64)
    gain = (lit - d)[lit > 0] / lit[lit > 0]
    out = {"value": round(P * steps / wall, 2), "unit": "pairs/s", "ms_per_step": round(wall * 1e3 / steps, 4),
           "kernel_ms": round(float(np.mean(ks)), 4), "bins": plan.bins(),
           "never_above_default": bool((d <= lit).all()),
           "pairs_below_default": int((d < lit).sum()),
           "mean_relative_reduction": round(float(gain.mean()) if gain.size else 0.0, 5)}
    log(f"complete-then-min: kernel {out['kernel_ms']} ms, {out['pairs_below_default']} of {P} pairs below default")
    maps_np = maps[:plan.map_size].cpu().numpy()
    plan.close()
    return out, d, maps_np


def directed_measure(ged, steps: int, warmup: int, tune: bool, tune_cache, threads: int, check_every: int = 1):
    """Directed graphs: the 4096-pair directed batch (n 10..30, arcs with p 0.05..0.15,
    K = 64, unit costs; pairs of up to 32 vertices take the two-word wavefront kernel's
    directed instantiation); kernel time, throughput, roofline, parity on every
    `check_every`-th pair (all of them by default), and the oracle's rate on those pairs."""
    import torch
    from paper_2605_00830_amd import synth
    w = synth.batch_directed_10_30(4096)
    P = len(w.pairs)
    db = ged.Database(w.graphs, directed=True)
    plan = ged.Plan(db, w.pairs, w.K)
    dist, maps, cand = plan.outputs(with_cand=True)
    s = torch.cuda.current_stream()
    plan.set_timing(True)
    if tune:
        plan.tune(w.costs, dist, maps, stream=s, cache_path=tune_cache)
        s.synchronize()
    for _ in range(warmup):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
    ks = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
        ks.append(plan.kernel_ms())
    wall = time.perf_counter() - t0
    d = dist[:P].cpu().numpy()
    m = maps[:plan.map_size].cpu().numpy()
    # algorithmic work: a directed vertex's row is an out-row and an in-row, so
    # twice the words of an undirected row of the same order
    ce = cand[:P].cpu().numpy().astype(np.int64)
    n2 = np.asarray(w.graphs.n, np.int64)[w.pairs[:, 1]]
    words = 2 * np.maximum((n2 + 31) // 32, 1)
    ops = float(sum(ops_per_candidate(int(x), 0) * int(c) for x, c in zip(words, ce)))
    kms = float(np.mean(ks))
    achieved = ops / (kms / 1e3) / 1e12
    # algorithmic HBM bytes: as for the undirected batch, with each graph's rows
    # twice (out-arc and in-arc blocks)
    gn = np.asarray(w.graphs.n, np.int64)
    gbytes = 2 * gn * np.maximum((gn + 31) // 32, 1) * 4 + gn * 4 + 32
    n1 = gn[w.pairs[:, 0]]
    alg_bytes = float(gbytes[w.pairs[:, 0]].sum() + gbytes[w.pairs[:, 1]].sum() + 24 * P + (4 + 4 * n1 + 8).sum())
    bins = plan.bins()
    tr = measured_traffic(bins[0][0], w.name) if len(bins) == 1 else None
    out = {"config": {"workload": w.name, "pairs": P, "K": w.K, "costs": list(w.costs),
                      "mean_order": round(float(w.graphs.n.mean()), 2), "mean_arcs": round(float(w.graphs.m.mean()), 2)},
           "value": round(P * steps / wall, 2), "unit": "pairs/s", "ms_per_step": round(wall * 1e3 / steps, 4),
           "kernel_ms": round(kms, 4), "bins": plan.bins(),
           "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_INT32_TOPS, 2),
                        "unit": "Tops/s", "frac": round(achieved / PEAK_INT32_TOPS, 5),
                        "traffic": None if tr is None else tr["bytes_per_launch"],
                        "kernel": bins[0][0] if len(bins) == 1 else None,
                        "hbm": {"algorithmic_bytes": alg_bytes,
                                "algorithmic_gbps": round(alg_bytes / (kms / 1e3) / 1e9, 2),
                                "measured_gbps": None if tr is None else
                                round(tr["bytes_per_launch"] / (kms / 1e3) / 1e9, 2)},
                        "candidates_per_launch": int(ce.sum()), "ops_per_launch": ops}}
    plan.close()
    db.close()
    idx = np.arange(0, P, check_every)
    cw, cd, cm = cpu_oracle(w.graphs, w.pairs[idx], w.costs, w.K, threads, directed=True)
    n_src = np.asarray(w.graphs.n, np.int64)[w.pairs[:, 0]]
    moff = np.concatenate([[0], np.cumsum(n_src)])
    coff = np.concatenate([[0], np.cumsum(n_src[idx])])
    maps_ok = all(np.array_equal(m[moff[q]:moff[q + 1]], cm[coff[k]:coff[k + 1]]) for k, q in enumerate(idx))
    out["parity"] = {"pairs_checked": int(len(idx)), "dist_equal": bool(np.array_equal(d[idx], cd)),
                     "maps_equal": bool(maps_ok)}
    out["cpu_baseline"] = {"value": round(len(idx) / cw, 2), "unit": "pairs/s", "cores": threads, "kind": "oracle",
                           "sample": f"{len(idx)} of {P} pairs, {threads} threads, {cw:.2f} s wall"}
    log(f"directed: kernel {out['kernel_ms']} ms, {out['value']:.0f} pairs/s, parity {out['parity']}")
    return out


def alu_roofline(w, ce: np.ndarray, kms: float, bins, kernel: str) -> dict:
    """Roofline of one batched launch: algorithmic int32 operations (ops_per_candidate per
    evaluated child, from each pair's target words and the database's label planes) over
    the launch's duration, against the int32 VALU peak; and its algorithmic HBM bytes
    (both graphs' packed rows and labels, work item in; distance, mapping, count out)."""
    P = len(w.pairs)
    n2 = np.asarray(w.graphs.n, np.int64)[w.pairs[:, 1]]
    words = np.maximum((n2 + 31) // 32, 1)
    planes = 0
    if w.graphs.elabel is not None:
        nl = len(np.unique(w.graphs.elabel))
        while (1 << planes) < nl:
            planes += 1
    ops = float(sum(ops_per_candidate(int(x), planes) * int(c) for x, c in zip(words, ce)))
    achieved = ops / (kms / 1e3) / 1e12
    gn = np.asarray(w.graphs.n, np.int64)
    gw = np.maximum((gn + 31) // 32, 1)
    gbytes = gn * gw * 4 * (1 + planes) + gn * 4 + 32
    n1 = gn[w.pairs[:, 0]]
    alg_bytes = float(gbytes[w.pairs[:, 0]].sum() + gbytes[w.pairs[:, 1]].sum() + 24 * P + (4 + 4 * n1 + 8).sum())
    hbm_peak = 8.0e12
    hbm = {"algorithmic_bytes": alg_bytes,
           "algorithmic_gbps": round(alg_bytes / (kms / 1e3) / 1e9, 2),
           "algorithmic_frac": round(alg_bytes / (kms / 1e3) / hbm_peak, 6),
           "peak_gbps": hbm_peak / 1e9}
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_INT32_TOPS, 2),
            "unit": "Tops/s", "frac": round(achieved / PEAK_INT32_TOPS, 5), "traffic": None,
            "ce_per_s": round(float(ce.sum()) / (kms / 1e3), 1), "hbm": hbm,
            "kernel": kernel, "kernel_ms": round(kms, 4), "bins": bins,
            "candidates_per_launch": int(ce.sum()), "ops_per_launch": ops}


def config_measure(ged, name: str, steps: int, warmup: int, tune: bool, tune_cache, threads: int,
                   cpu: bool = True) -> dict:
    """One more of the batched workloads (the molecule query batch, the large-pair
    stress batch): pairs/s over timed steps, the roofline of its launch (all of its
    bins), the oracle on the workload's bounded sample with the same threads (its
    CPU baseline) and a bit-exact comparison of that sample with the GPU results."""
    import torch
    w, sample_n = workload(name)
    P = len(w.pairs)
    db = ged.Database(w.graphs)
    plan = ged.Plan(db, w.pairs, w.K)
    dist, maps, cand = plan.outputs(with_cand=True)
    s = torch.cuda.current_stream()
    plan.set_timing(True)
    if tune:
        plan.tune(w.costs, dist, maps, stream=s, cache_path=tune_cache)
        s.synchronize()
    for _ in range(warmup):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
    ks = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(w.costs, dist, maps, cand, stream=s)
        s.synchronize()
        ks.append(plan.kernel_ms())
    wall = time.perf_counter() - t0
    kms = float(np.mean(ks))
    bins = plan.bins()
    ce = cand[:P].cpu().numpy().astype(np.int64)
    gpu_dist = dist[:P].cpu().numpy()
    gpu_maps = maps[:plan.map_size].cpu().numpy()
    dominant = max(bins, key=lambda b: b[1])[0] if bins else "none"
    out = {"config": {"workload": w.name, "pairs": P, "K": w.K, "costs": list(w.costs)},
           "value": round(P * steps / wall, 2), "unit": "pairs/s", "ms_per_step": round(wall * 1e3 / steps, 4),
           "roofline": alu_roofline(w, ce, kms, bins, dominant)}
    log(f"{w.name}: {out['ms_per_step']} ms/step, kernel {kms:.3f} ms, {out['value']:.0f} pairs/s, "
        f"{out['roofline']['frac']:.4f} of the int32 peak")
    if cpu:
        sample = np.arange(min(sample_n, P))
        cw, cd, cm = cpu_oracle(w.graphs, w.pairs[sample], w.costs, w.K, min(threads, len(sample)))
        used = min(threads, len(sample))
        out["cpu_baseline"] = {"value": round(len(sample) / cw, 3), "unit": "pairs/s", "cores": used,
                               "kind": "oracle",
                               "sample": f"first {len(sample)} of {P} pairs, {used} threads, {cw:.2f} s wall"}
        n_src = np.asarray(w.graphs.n, np.int64)[w.pairs[:, 0]]
        moff = np.concatenate([[0], np.cumsum(n_src)])
        g_sel = np.concatenate([gpu_maps[moff[p]:moff[p + 1]] for p in sample])
        out["parity"] = {"pairs_checked": int(len(sample)),
                         "bit_exact": bool(np.array_equal(gpu_dist[sample], cd) and np.array_equal(g_sel, cm))}
        log(f"{w.name}: oracle {out['cpu_baseline']['value']} pairs/s, parity {out['parity']}")
    plan.close()
    db.close()
    return out


def workload(name: str):
    from paper_2605_00830_amd import synth
    if name == "batch":
        return synth.batch_er_10_30(4096), None
    if name == "pair":
        return synth.pair_er_8x9(), None
    if name == "query":
        return synth.query_molecule_10_70(10000), 500
    if name == "stress":
        return synth.stress_er_100_500(256), 4
    if name == "molecule":
        return synth.batch_molecule_k64(10000), 1000
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "pair", "query", "stress", "molecule", "serve"])
    ap.add_argument("--serve-queries", type=int, default=100000,
                    help="queries of the serving measurement (the serving mix has 100,000)")
    ap.add_argument("--serve-db", type=int, default=100000, help="database graphs of the serving measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-large-k", action="store_true", help="skip the single-pair large-K measurement")
    ap.add_argument("--large-k-only", action="store_true",
                    help="run only the single-pair large-K measurement and print its JSON")
    ap.add_argument("--serve-streams", type=int, default=SERVE_STREAMS, help="server streams per size class")
    ap.add_argument("--serve-method", choices=["tree", "bipartite"], default="tree",
                    help="method the serving measurement runs (--workload serve)")
    ap.add_argument("--serve-directed", action="store_true",
                    help="serve the directed mix (--workload serve, tree method)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0 = min(16, cores))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-perpair", action="store_true")
    ap.add_argument("--no-complete", action="store_true",
                    help="skip the complete-then-minimum last-level measurement")
    ap.add_argument("--no-bipartite", action="store_true",
                    help="skip the bipartite K-best-assignment measurement")
    ap.add_argument("--no-directed", action="store_true", help="skip the directed-graph measurement")
    ap.add_argument("--eager", action="store_true",
                    help="time eager plan runs instead of replays of the plan's captured HIP graph")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the molecule query and large-pair stress batches of the default run")
    ap.add_argument("--no-tune", action="store_true", help="keep the plan's default schedule (no autotuning)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: reuse its choices, append new ones (default: tune afresh)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); pairs are independent, "
              "so a multi-GPU run would shard the batch over GPUs; sharding is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")

    import torch
    from paper_2605_00830_amd import ged

    torch.cuda.set_device(0)
    if args.large_k_only:
        print(json.dumps({"large_k": large_k_measure(ged, cpu=not args.no_cpu_baseline)}), flush=True)
        return
    if args.workload == "serve":
        from paper_2605_00830_amd import synth
        t0 = time.perf_counter()
        sw = (synth.serve_mix_directed if args.serve_directed else synth.serve_mix)(args.serve_db, args.serve_queries)
        log(f"serving workload generated in {time.perf_counter() - t0:.1f} s")
        res = serve_measure(ged, sw, args.serve_queries, fracs=(0.5, 0.8, 0.95), streams=args.serve_streams,
                            method=1 if args.serve_method == "bipartite" else 0)
        head = res["open_loop"][1]
        print(json.dumps({
            "metric": METRIC, "value": res["saturated_qps"], "unit": "pairs/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int32", "data": "synthetic", "config": res["config"],
            "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "serving": res}), flush=True)
        return
    w, cpu_sample = workload(args.workload)
    P = len(w.pairs)
    log(f"workload {w.name}: {P} pairs, K={w.K}, costs={w.costs}")
    db = ged.Database(w.graphs)
    plan = ged.Plan(db, w.pairs, w.K)
    dist, maps, cand = plan.outputs(with_cand=True)
    stream = torch.cuda.current_stream()
    plan.set_timing(True)
    if not args.no_tune:
        timed = plan.tune(w.costs, dist, maps, stream=stream, cache_path=args.tune_cache)
        stream.synchronize()
        log(f"autotuner timed {timed} bin(s)")

    bins = plan.bins()
    dominant = max(bins, key=lambda b: b[1])[0] if bins else "none"
    log(f"bins: {bins}")
    if args.copy_calibration_mib > 0:
        # the source is the first quarter of a buffer four times its size, filled
        # front to back, so it has left the last-level cache when it is copied
        nbytes = args.copy_calibration_mib << 20
        big = torch.ones(nbytes, dtype=torch.int32, device="cuda")
        dst = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        dst.copy_(big[:nbytes // 4])
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written once")
        del big, dst

    for _ in range(args.warmup):
        plan.run(w.costs, dist, maps, cand, stream=stream)
        stream.synchronize()
    torch.cuda.synchronize()
    # the search kernels' duration: the plan's HIP events around them, eager runs
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(w.costs, dist, maps, cand, stream=stream)
        stream.synchronize()
        kernel_ms.append(plan.kernel_ms())
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kms = float(np.mean(kernel_ms))
    launch = "eager"
    synced_ms = eager_ms
    if args.eager:
        ms_per_step = eager_ms
    else:
        # the timed steps: the plan's run captured once as a HIP graph (kernel nodes
        # only) and replayed on a stream of its own, the K steps enqueued back to
        # back (each a full pass over the batch) and the stream synchronized
        # after the last; the same with a synchronize after every step is
        # reported beside it
        gstream = torch.cuda.Stream()
        plan.capture(w.costs, dist, maps, cand, stream=gstream)
        for _ in range(args.warmup):
            plan.replay(stream=gstream)
            gstream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.replay(stream=gstream)
            gstream.synchronize()
        torch.cuda.synchronize()
        synced_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.replay(stream=gstream)
        gstream.synchronize()
        torch.cuda.synchronize()
        ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
        launch = "hip_graph, steps back to back"
    value = P / (ms_per_step / 1e3)
    log(f"batched ({launch}): {ms_per_step:.3f} ms/step (eager {eager_ms:.3f}, synchronized "
        f"{synced_ms:.3f}), kernel {kms:.3f} ms, {value:.0f} pairs/s")

    gpu_dist = dist[:P].cpu().numpy()
    gpu_maps = maps[:plan.map_size].cpu().numpy()
    ce = cand[:P].cpu().numpy().astype(np.int64)

    # algorithmic work of one launch of the search kernel
    n2 = np.asarray(w.graphs.n, np.int64)[w.pairs[:, 1]]
    words = np.maximum((n2 + 31) // 32, 1)
    planes = 0
    if w.graphs.elabel is not None:
        nl = len(np.unique(w.graphs.elabel))
        while (1 << planes) < nl:
            planes += 1
    ops = float(sum(ops_per_candidate(int(x), planes) * int(c) for x, c in zip(words, ce)))
    achieved = ops / (kms / 1e3) / 1e12
    tr = measured_traffic(dominant, w.name) if len(bins) == 1 else None
    # algorithmic HBM bytes of a launch: both graphs' rows (and label planes)
    # and vertex labels, two records and a work item per pair in; distance,
    # mapping and candidate count per pair out
    gn = np.asarray(w.graphs.n, np.int64)
    gw = np.maximum((gn + 31) // 32, 1)
    gbytes = gn * gw * 4 * (1 + planes) + gn * 4 + 32
    n1 = gn[w.pairs[:, 0]]
    alg_bytes = float(gbytes[w.pairs[:, 0]].sum() + gbytes[w.pairs[:, 1]].sum() + 24 * P +
                      (4 + 4 * n1 + 8).sum())
    hbm_peak = 8.0e12
    hbm = {"algorithmic_bytes": alg_bytes,
           "algorithmic_gbps": round(alg_bytes / (kms / 1e3) / 1e9, 2),
           "algorithmic_frac": round(alg_bytes / (kms / 1e3) / hbm_peak, 6),
           "peak_gbps": hbm_peak / 1e9}
    if tr is not None:
        hbm["measured_gbps"] = round(tr["bytes_per_launch"] / (kms / 1e3) / 1e9, 2)
        hbm["measured_frac"] = round(tr["bytes_per_launch"] / (kms / 1e3) / hbm_peak, 6)
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_INT32_TOPS, 2),
                "unit": "Tops/s", "frac": round(achieved / PEAK_INT32_TOPS, 5),
                "traffic": None if tr is None else tr["bytes_per_launch"],
                "ce_per_s": round(float(ce.sum()) / (kms / 1e3), 1), "hbm": hbm,
                "kernel": dominant, "kernel_ms": round(kms, 4), "bins": bins,
                "candidates_per_launch": int(ce.sum()), "ops_per_launch": ops}

    perpair = None
    if not args.no_perpair:
        plan.run(w.costs, dist, maps, cand, stream=stream, perpair=True)
        stream.synchronize()
        t0 = time.perf_counter()
        plan.run(w.costs, dist, maps, cand, stream=stream, perpair=True)
        stream.synchronize()
        pw = time.perf_counter() - t0
        pk = plan.kernel_ms()
        same = bool(np.array_equal(dist[:P].cpu().numpy(), gpu_dist) and
                    np.array_equal(maps[:plan.map_size].cpu().numpy(), gpu_maps))
        perpair = {"value": round(P / pw, 2), "unit": "pairs/s", "ms_per_step": round(pw * 1e3, 3),
                   "launches": plan.kernel_launches(), "kernel_span_ms": round(pk, 3),
                   "same_results_as_batched": same}
        log(f"per-pair: {pw * 1e3:.1f} ms for {P} launches, {P / pw:.0f} pairs/s")

    # edit-path output of the batch's mappings (one synchronous library call:
    # work-list staging, the kernel, the per-pair counts read back)
    epath = None
    if args.workload == "batch":
        e_ops, e_off, e_cnt = ged.edit_path(db, w.pairs, w.costs, maps)
        eps = []
        for _ in range(5):
            t1 = time.perf_counter()
            e_ops, e_off, e_cnt = ged.edit_path(db, w.pairs, w.costs, maps)
            eps.append(time.perf_counter() - t1)
        # pair p's operations are the first e_cnt[p] of its slots from e_off[p]
        # (its capacity, n1 + n2 + m1 + m2, may leave unwritten slots after them)
        e_sum = np.array([int(e_ops[e_off[p]:e_off[p] + e_cnt[p], 5].sum()) for p in range(P)], dtype=np.int64)
        epath = {"ms_per_call": round(float(np.median(eps)) * 1e3, 3), "operations": int(e_cnt.sum()),
                 "costs_sum_to_distance": bool(np.array_equal(e_sum, gpu_dist.astype(np.int64)))}
        log(f"edit paths: {epath}")

    complete = None
    if not args.no_complete and args.workload == "batch":
        complete, c_dist, c_maps = complete_measure(ged, db, w, args.steps, args.warmup, gpu_dist,
                                                       not args.no_tune, args.tune_cache)
        # the same per-child operation count as the default search (the last
        # level's completion adds a few operations per child, not counted)
        ach_c = ops / (complete["kernel_ms"] / 1e3) / 1e12
        complete["roofline"] = {"bound": "alu", "achieved": round(ach_c, 4), "peak": round(PEAK_INT32_TOPS, 2),
                                "unit": "Tops/s", "frac": round(ach_c / PEAK_INT32_TOPS, 5)}

    bip = None
    if not args.no_bipartite and args.workload in ("batch", "query"):
        bip, b_dist, b_maps, b_cand = bipartite_measure(ged, db, w, args.steps, args.warmup, not args.no_tune,
                                                        args.tune_cache)

    directed = None
    if not args.no_directed and args.workload == "batch":
        directed = directed_measure(ged, args.steps, args.warmup, not args.no_tune, args.tune_cache,
                                    args.cpu_threads or min(16, os.cpu_count() or 1))

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        sample = np.arange(P) if cpu_sample is None else np.arange(min(cpu_sample, P))
        log(f"cpu oracle on {len(sample)} pairs with {threads} threads ...")
        cw, cd, cm = cpu_oracle(w.graphs, w.pairs[sample], w.costs, w.K, threads)
        # one core on a tenth of the sample (the oracle is single-threaded per pair)
        one = sample[:max(1, len(sample) // 10)]
        c1, _, _ = cpu_oracle(w.graphs, w.pairs[one], w.costs, w.K, 1)
        cpu = {"value": round(len(sample) / cw, 2), "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(sample)} of {P} pairs of the same workload, {threads} threads, "
                         f"{cw:.2f} s wall",
               "single_core": {"value": round(len(one) / c1, 2), "unit": "pairs/s", "pairs": int(len(one))},
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        n_src = np.asarray(w.graphs.n, np.int64)[w.pairs[:, 0]]
        moff = np.concatenate([[0], np.cumsum(n_src)])
        g_maps = np.concatenate([gpu_maps[moff[p]:moff[p + 1]] for p in sample]) if len(sample) else gpu_maps[:0]
        ok = bool(np.array_equal(gpu_dist[sample], cd) and np.array_equal(g_maps, cm))
        parity = {"pairs_checked": int(len(sample)), "bit_exact": ok}
        log(f"cpu oracle: {len(sample) / cw:.1f} pairs/s; GPU parity on sample: {ok}")
        if complete is not None:
            # the same bounded sample through the oracle's complete-then-minimum mode
            _, kd, km = cpu_oracle(w.graphs, w.pairs[sample], w.costs, w.K, threads, last_complete=True)
            c_sel = np.concatenate([c_maps[moff[p]:moff[p + 1]] for p in sample]) if len(sample) else c_maps[:0]
            complete["parity"] = {"pairs_checked": int(len(sample)),
                                  "bit_exact": bool(np.array_equal(c_dist[sample], kd) and np.array_equal(c_sel, km))}
        if epath is not None:
            # the oracle's expansion of the same mappings, first 256 pairs
            ok_ep = True
            for q in range(min(256, P)):
                a_, b_ = int(w.pairs[q, 0]), int(w.pairs[q, 1])
                ref = oracle_mod().edit_path(w.graphs.graph(a_), w.graphs.graph(b_), w.costs, gpu_maps[moff[q]:moff[q + 1]])
                got = e_ops[e_off[q]:e_off[q] + e_cnt[q]]
                ok_ep = ok_ep and e_cnt[q] == len(ref) and np.array_equal(got, np.asarray(ref, np.int32).reshape(-1, 6))
            epath["parity"] = {"pairs_checked": min(256, P), "equal_to_oracle": bool(ok_ep)}
        if bip is not None:
            # the bipartite oracle on the same sample: parity, its own CPU
            # baseline, and the solver steps that price the kernel's work
            bw, bd, bm, bsv, bst = cpu_oracle_bip(w.graphs, w.pairs[sample], w.costs, w.K, threads)
            b_sel = np.concatenate([b_maps[moff[p]:moff[p + 1]] for p in sample]) if len(sample) else b_maps[:0]
            bip["parity"] = {"pairs_checked": int(len(sample)),
                             "bit_exact": bool(np.array_equal(b_dist[sample], bd) and np.array_equal(b_sel, bm) and
                                               np.array_equal(b_cand[sample], bsv))}
            bip["cpu_baseline"] = {"value": round(len(sample) / bw, 2), "unit": "pairs/s", "cores": threads,
                                   "kind": "oracle", "sample": f"{len(sample)} of {P} pairs, {threads} threads, "
                                                               f"{bw:.2f} s wall"}
            if len(sample) == P:
                order = np.asarray(w.graphs.n, np.int64)[w.pairs].sum(1)
                relax = int((bst * order).sum())
                ops = float(relax) * BIP_OPS_PER_RELAX
                ach = ops / (bip["kernel_ms"] / 1e3) / 1e12
                bip["roofline"] = {"bound": "alu", "achieved": round(ach, 4), "peak": round(PEAK_INT32_TOPS, 2),
                                   "unit": "Tops/s", "frac": round(ach / PEAK_INT32_TOPS, 5),
                                   "solver_steps": int(bst.sum()), "column_relaxations": relax,
                                   "ops_per_relaxation": BIP_OPS_PER_RELAX, "ops_per_launch": ops}
            log(f"bipartite oracle: {len(sample) / bw:.1f} pairs/s; parity {bip['parity']['bit_exact']}")

    configs = None
    if not args.no_configs and args.workload == "batch":
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        configs = {nm: config_measure(ged, nm, max(3, args.steps // 4), 1, not args.no_tune, args.tune_cache,
                                      threads, cpu=not args.no_cpu_baseline)
                   for nm in ("query", "stress")}

    large_k = None
    if not args.no_large_k and args.workload == "batch":
        large_k = large_k_measure(ged, cpu=not args.no_cpu_baseline)

    serving = None
    if not args.no_serve and args.workload == "batch":
        from paper_2605_00830_amd import synth
        t0 = time.perf_counter()
        sw = synth.serve_mix(args.serve_db, args.serve_queries)
        log(f"serving workload generated in {time.perf_counter() - t0:.1f} s")
        serving = serve_measure(ged, sw, args.serve_queries, fracs=(0.5, 0.8, 0.95), streams=args.serve_streams)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "pairs": P, "K": w.K, "costs": list(w.costs), "launch": launch},
        "eager_ms_per_step": round(eager_ms, 4),
        "synchronized_ms_per_step": round(synced_ms, 4),
        "perpair": perpair,
        "speedup_vs_perpair": None if perpair is None else round(value / perpair["value"], 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "edit_path": epath,
        "complete_then_min": complete,
        "bipartite": bip,
        "directed": directed,
        "configs": configs,
        "large_k": large_k,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    plan.close()
    db.close()


if __name__ == "__main__":
    main()
