#!/usr/bin/env python
"""GED-Walk benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints ONE JSON line.  `value` is whole-step walk-count throughput in GTEPS:
arcs x columns traversed by every walk-count step kernel of the timed steps,
divided by the wall time of those steps (inputs resident in HBM, graph CSR
uploaded before timing).  `roofline` reports the dominant step kernel's
algorithmic bytes per launch over its average HIP-event duration, against the
8 TB/s HBM peak; `cpu_baseline` times the CPU oracle on a bounded sample of the
same workload.

Workloads (a "step" is one pass of the hot path over one batch of input):
  rmat22  (default) R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05),
          symmetrized: per step the per-graph precompute (t-levels, ell*),
          16 single-group scores (|S|=5) and greedy k=100.
  ba1m    Barabasi-Albert n=1,000,000, m=5: precompute, 16 scores (|S|=5),
          greedy k=10 and a batched scoring of 256 groups (|S| ~ U[1,200]).
  er1k    Erdos-Renyi n=1,000, average degree 10: precompute, score |S|=5,
          greedy k=5.
  batch   Barabasi-Albert n=2,000,000, m=8: 4,096 groups (|S| ~ U[1,200])
          scored batched vs 4,096 sequential single-group calls.
  serve   request stream over 8 resident graphs (see paper_1910_13874_amd/serve.py).
  variants  directed graphs, arc weights, the spectral bound and the stochastic
          greedy on ~10^5-vertex graphs; the CPU baseline leg runs the oracle on
          the same calls.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-count SpMV GTEPS (%HBM roofline); greedy k=100 s; p50/p99 score ms"
HBM_PEAK_GBS = 8000.0
EPS = 1e-4
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ged_kernels.hip", "ged_internal.h"):
        with open(os.path.join(ROOT, "paper_1910_13874_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None
    if there is none or the step kernels changed since it was taken."""
    p = os.path.join(PROFILES, f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def host_cpu():
    """CPU model and logical CPU count of this host."""
    model = "?"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(g, alpha, groups, budget_s=6.0, max_threads=16):
    """The oracle's single-group score, timed on this host: first on one
    core, then on up to max_threads threads scoring independent groups at once
    (the oracle is single-threaded C; its calls release the interpreter lock),
    each for about budget_s seconds of wall time."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    def run(offset, stop_at):
        done, edges = 0, 0.0
        while time.perf_counter() < stop_at:
            S = groups[(offset + done) % len(groups)]
            ell = oracle.score(g, S, alpha, EPS)[1]
            edges += ell * g.nnz
            done += 1
        return done, edges

    t0 = time.perf_counter()
    one_done, one_edges = run(0, t0 + budget_s)
    one_dt = time.perf_counter() - t0
    threads = max(1, min(max_threads, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda i: run(i, t0 + budget_s), range(threads)))
    dt = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    edges = sum(r[1] for r in res)
    return {"value": edges / dt / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{done} single-group scores (|S|={len(groups[0])}) of the same graph by "
                      f"the single-threaded FP64 oracle on {threads} threads at once, {dt:.1f} s; "
                      f"one core: {one_done} scores in {one_dt:.1f} s",
            "one_core_value": one_edges / one_dt / 1e9,
            "seconds_per_score_one_core": one_dt / one_done,
            "host": host_cpu()}


def step_bytes(n, nnz, C, weighted=False):
    """Algorithmic bytes of one masked walk-count step over C FP64 columns:
    row_ptr 4(n+1), col_idx 4 nnz (+ 8 nnz weights), one read of the input
    columns 8nC, one write of the output columns 8nC, the group bitmap n/8."""
    return 4.0 * (n + 1) + 4.0 * nnz + 16.0 * n * C + n / 8.0 + (8.0 * nnz if weighted else 0.0)


def oracle_greedy_context(g, name, k, rg):
    """The oracle's greedy trace for this graph and k, when one is stored with
    the tests (written once by tests/golden/make_golden.py): its wall time on
    one core and whether the GPU's picks and walk lengths equal it."""
    p = os.path.join(ROOT, "tests", "golden", f"{name}_k{k}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f)
    if rec.get("fingerprint") != g.fingerprint():
        return None
    m = len(rec["group"])
    return {"picks_stored": m, "oracle_s": rec.get("oracle_s"),
            "oracle_s_note": "one core, single-threaded FP64 oracle, run in segments of "
                             f"{rec.get('segment')} picks (forced-prefix replay)",
            "same_picks": [int(x) for x in rg["group"][:m]] == rec["group"],
            "same_ells": [int(x) for x in rg["ell"][:m]] == rec["ell"]}


def roofline(prof, ged, workload, n, nnz, weighted=False):
    """Dominant step kernel: step_bytes() for its column count over its
    average launch duration (HIP events on the launch stream), against the
    HBM peak.  The bytes the kernel's own operands occupy (32-bit counts,
    column masks, combining inputs) are reported beside it."""
    ms = prof["dominant_ms"] / max(1, prof["dominant_launches"])
    C = prof["dominant_columns"]
    bytes_per = step_bytes(n, nnz, C, weighted)
    operand_per = prof["dominant_bytes"] / max(1, prof["dominant_launches"])
    achieved = bytes_per / (ms * 1e-3) / 1e9
    kname = ged.kernel_name(C, prof["dominant_kind"])
    tr = traffic_for(workload, kname)
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "kernel": kname, "columns": C,
           "avg_launch_us": ms * 1e3, "algorithmic_bytes_per_launch": bytes_per,
           "launches": prof["dominant_launches"],
           "operand_bytes_per_launch": operand_per,
           "operand_frac": operand_per / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if tr:
        # measured L2-miss bytes per launch over the same event-timed duration
        out["traffic_gbs"] = tr / (ms * 1e-3) / 1e9
        out["traffic_frac"] = out["traffic_gbs"] / HBM_PEAK_GBS
    return out


def run_steps(step, K, W, gg, torch):
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    gg.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        step()
        log(f"step {i + 1}/{K} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = gg.profile_read()
    gg.profile_enable(False)
    return dt, prof


def score_latency(gg, groups, alpha, torch, reps=200):
    lat = []
    for j in range(reps):
        S = groups[j % len(groups)]
        t = time.perf_counter()
        gg.score(S, alpha, EPS)
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def bench_graph_workload(args, torch, ged, inputs):
    name = args.workload
    spec = {
        "ba1m": dict(graph="ba1m", k=10, n_scores=16, batch=256,
                     desc="Barabasi-Albert n=1,000,000 m=5, CSR int32, FP64, alpha=1/(maxdeg+1), "
                          "eps=1e-4: precompute + 16 scores |S|=5 + greedy k=10 + batch of 256 "
                          "groups |S|~U[1,200]"),
        "rmat22": dict(graph="rmat22", k=100, n_scores=16, batch=0,
                       desc="R-MAT scale 22 edge factor 16 (0.57,0.19,0.19,0.05) symmetrized, "
                            "FP64, alpha=1/(maxdeg+1), eps=1e-4: precompute + 16 scores |S|=5 + "
                            "greedy k=100"),
        "er1k": dict(graph="er1k", k=5, n_scores=1, batch=0,
                     desc="Erdos-Renyi n=1,000 avg degree 10, FP64, alpha=1/(maxdeg+1), "
                          "eps=1e-4: precompute + score |S|=5 + greedy k=5"),
    }[name]
    t_gen = time.perf_counter()
    g = inputs.workload_graph(spec["graph"])
    log(f"graph {name}: n={g.n} nnz={g.nnz} dmax={g.max_degree} "
        f"({time.perf_counter() - t_gen:.1f}s)")
    torch.cuda.synchronize()  # device context up before the upload is timed
    t_up = time.perf_counter()
    gg = ged.GedGraph.from_graph(g, keep_order=args.order == "input")
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t_up  # host CSR to the device, relabelling
    if args.buckets is not None:
        gg.set_source_buckets(args.buckets)
    stream = torch.cuda.Stream()
    gg.set_stream(stream)
    if args.greedy_width:
        gg.set_greedy_width(args.greedy_width)
    if args.tile:
        gg.set_batch_tile(args.tile)
    alpha = gg.default_alpha()
    groups = [inputs.group(g.n, 5, 1000 + j) for j in range(max(spec["n_scores"], 16))]
    if spec["batch"]:
        off, mem = inputs.groups(g.n, spec["batch"], 1, 200, 104)
    info = {}

    def step():
        gg.invalidate()
        info["ell"] = gg.prepare(alpha, EPS)[0]
        for S in groups[:spec["n_scores"]]:
            gg.score(S, alpha, EPS)
        t = time.perf_counter()
        r = gg.greedy(spec["k"], alpha, EPS)
        info["greedy_s"] = time.perf_counter() - t
        info["greedy"] = r
        if spec["batch"]:
            gg.score_batch(off, mem, alpha, EPS)

    dt, prof = run_steps(step, args.steps, args.warmup, gg, torch)
    p50, p99 = score_latency(gg, groups, alpha, torch)
    # greedy alone, untimed by the profiler (its own wall clock)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rg = gg.greedy(spec["k"], alpha, EPS)
    greedy_s = time.perf_counter() - t
    out = {
        "metric": METRIC, "value": prof["edges"] / dt / 1e9, "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": spec["desc"], "graph": spec["graph"], "n": g.n, "nnz": g.nnz,
                   "max_degree": g.max_degree, "alpha": alpha, "eps": EPS, "ell_star": info["ell"],
                   "greedy_k": spec["k"], "score_groups": spec["n_scores"],
                   "batch_groups": spec["batch"], "parallelism": "single GPU"},
        "roofline": roofline(prof, ged, name, g.n, g.nnz),
        "greedy_s": greedy_s,
        "greedy_ells": [int(x) for x in rg["ell"]],
        "greedy_evals": int(rg["evals"][-1]),
        "score_ms_p50": p50, "score_ms_p99": p99,
        "step_kernels_ms": prof["total_ms"] / args.steps,
        "step_kernels_frac_of_step": prof["total_ms"] / (dt * 1e3),
        "batch_tile": gg.batch_tile() if spec["batch"] else None,
        "greedy_width": gg.greedy_width(),
        # the graph is handed over as host CSR arrays once, outside the timed
        # steps: its creation time, and the rate of a one-step job including it
        "graph_create_s": create_s,
        "value_incl_graph_upload": prof["edges"] / args.steps / (dt / args.steps + create_s) / 1e9,
    }
    ctx = oracle_greedy_context(g, spec["graph"], spec["k"], rg)
    if ctx:
        out["oracle_greedy"] = ctx
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, alpha, groups)
    gg.close()
    if name == "rmat22" and not args.no_batch:
        log("batched-scoring context: BA n=2e6, 4096 groups")
        out["batched"] = batch_ratio(torch, ged, inputs)
    return out


def batch_ratio(torch, ged, inputs, groups=4096, steps=2):
    """Batched scoring of `groups` groups (|S| ~ U[1,200], seed 104) on BA
    n=2,000,000, m=8 against the same groups scored one call at a time on the
    same GPU: queries/s of each and their ratio (context keys of the default
    line; --workload batch is the full measurement)."""
    g = inputs.workload_graph("ba2m")
    gg = ged.GedGraph.from_graph(g)
    gg.set_stream(torch.cuda.Stream())
    alpha = gg.default_alpha()
    off, mem = inputs.groups(g.n, groups, 1, 200, 104)
    gg.prepare(alpha, EPS)
    gg.score_batch(off, mem, alpha, EPS)  # autotune, capture
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        b = gg.score_batch(off, mem, alpha, EPS)
    torch.cuda.synchronize()
    bq = groups * steps / (time.perf_counter() - t)
    seq = np.zeros(groups)
    t = time.perf_counter()
    for j in range(groups):
        seq[j] = gg.score(mem[off[j]:off[j + 1]], alpha, EPS)
    torch.cuda.synchronize()
    pq = groups / (time.perf_counter() - t)
    out = {"workload": f"BA n=2,000,000 m=8, {groups} groups |S|~U[1,200]",
           "batch_queries_per_s": bq, "plain_queries_per_s": pq, "batch_speedup": bq / pq,
           "tile": gg.batch_tile(), "row_cut_div": gg.batch_row_cut(),
           "max_rel_batch_vs_plain": float(np.max(np.abs(b - seq) / np.maximum(np.abs(seq), 1e-300)))}
    gg.close()
    return out


def bench_batch(args, torch, ged, inputs):
    """Batched scoring of 4,096 groups vs 4,096 sequential single-group calls."""
    g = inputs.workload_graph("ba2m")
    log(f"graph ba2m: n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g, keep_order=args.order == "input")
    if args.buckets is not None:
        gg.set_source_buckets(args.buckets)
    stream = torch.cuda.Stream()
    gg.set_stream(stream)
    alpha = gg.default_alpha()
    G = args.groups
    off, mem = inputs.groups(g.n, G, 1, 200, 104)
    gg.prepare(alpha, EPS)
    if args.tile:
        gg.set_batch_tile(args.tile)

    def step():
        gg.score_batch(off, mem, alpha, EPS)

    dt, prof = run_steps(step, args.steps, args.warmup, gg, torch)
    batch_qps = G * args.steps / dt
    # sequential plain calls on the same GPU (the one-at-a-time baseline)
    n_seq = min(G, args.seq_sample)
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq = np.zeros(n_seq)
    for j in range(n_seq):
        seq[j] = gg.score(mem[off[j]:off[j + 1]], alpha, EPS)
    torch.cuda.synchronize()
    seq_dt = time.perf_counter() - t
    plain_qps = n_seq / seq_dt
    b = gg.score_batch(off, mem, alpha, EPS)
    maxrel = float(np.max(np.abs(b[:n_seq] - seq) / np.maximum(np.abs(seq), 1e-300)))
    out = {
        "metric": METRIC, "value": prof["edges"] / dt / 1e9, "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched scoring: {G} groups |S|~U[1,200] on Barabasi-Albert "
                               "n=2,000,000 m=8, FP64, eps=1e-4", "n": g.n, "nnz": g.nnz,
                   "groups": G, "tile": gg.batch_tile(), "parallelism": "single GPU"},
        "roofline": roofline(prof, ged, "batch", g.n, g.nnz),
        "batch_queries_per_s": batch_qps, "plain_queries_per_s": plain_qps,
        "batch_speedup": batch_qps / plain_qps, "plain_sample": n_seq,
        "batch_vs_plain_max_rel": maxrel,
    }
    if not args.no_cpu:
        groups = [mem[off[j]:off[j + 1]] for j in range(8)]
        out["cpu_baseline"] = cpu_baseline(g, alpha, groups)
    gg.close()
    return out


def bench_variants(args, torch, ged, inputs, k=10, n_scores=16):
    """The paper's variants beside the undirected unweighted path -- directed
    graphs, arc weights, the spectral tail bound, the stochastic greedy --
    each on a graph of about 10^5 vertices: 16 scores (|S| = 5) and a greedy
    (k = 10) timed on the GPU with the dominant step kernel's roofline.  The
    CPU baseline leg (skipped with --no-cpu) times the oracle on the same calls
    (two of the scores, the whole greedy) and reports its agreement."""

    def directed_rmat():
        u = inputs.rmat(17, 8, seed=21)
        src = np.repeat(np.arange(u.n, dtype=np.int64), np.diff(u.row_ptr))
        dst = u.col_idx.astype(np.int64)
        # one orientation per undirected edge, chosen by a hash of the pair
        lo, hi = np.minimum(src, dst), np.maximum(src, dst)
        flip = ((lo * 2654435761 + hi * 40503) >> 7) & 1
        keep = src == np.where(flip == 1, lo, hi)
        return inputs.from_edges(u.n, src[keep], dst[keep], symmetrize=False, name="rmat17_dir")

    ba = inputs.barabasi_albert(100000, 5, 33)
    deg = np.diff(ba.row_ptr).astype(np.float64)
    rows = np.repeat(np.arange(ba.n), np.diff(ba.row_ptr))
    w = 1.0 / np.sqrt(deg[rows] * deg[ba.col_idx])
    gd = directed_rmat()
    cases = {"directed": (gd, None, "combinatorial"), "weighted": (ba, w, "combinatorial"),
             "spectral": (ba, None, "spectral"), "stochastic": (ba, None, "combinatorial")}
    res, runs, edges, wall = {}, {}, 0.0, 0.0
    for name, (g, wt, bound) in cases.items():
        log(f"variant {name}: n={g.n} nnz={g.nnz}")
        gg = ged.GedGraph.from_graph(g, weights=wt)
        stream = torch.cuda.Stream()
        gg.set_stream(stream)
        sigma = None
        if bound == "spectral":
            gg.set_tail_bound("spectral")
            sigma = gg.sigma_max()
            alpha = 0.5 / sigma
        elif wt is not None:
            # half the inverse of the largest weighted out-degree (the sum of
            # the weights of the arcs leaving a vertex), beyond 1/(max + 1)
            alpha = 0.5 / float(np.bincount(g.col_idx, weights=wt, minlength=g.n).max())
        else:
            alpha = gg.default_alpha()
        groups = [inputs.group(g.n, 5, 2000 + j) for j in range(n_scores)]
        if name == "stochastic":
            run_greedy = lambda: gg.greedy_stochastic(k, alpha, EPS, eta=0.1, seed=1)
        else:
            run_greedy = lambda: gg.greedy(k, alpha, EPS)
        gg.score(groups[0], alpha, EPS)  # warm-up: precompute, tables, kernels
        run_greedy()
        torch.cuda.synchronize()
        gg.profile_enable(True)
        t0 = time.perf_counter()
        scores = [gg.score(S, alpha, EPS) for S in groups]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rg = run_greedy()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        prof = gg.profile_read()
        gg.profile_enable(False)
        edges += prof["edges"]
        wall += t2 - t0
        res[name] = {
            "graph": g.name, "n": g.n, "nnz": g.nnz, "alpha": alpha,
            "score_ms": (t1 - t0) / n_scores * 1e3, "greedy_ms": (t2 - t1) * 1e3,
            "greedy_ells": [int(x) for x in rg["ell"]],
            "roofline": roofline(prof, ged, "variants", g.n, g.nnz, weighted=wt is not None),
        }
        runs[name] = dict(g=g, wt=wt, sigma=sigma, alpha=alpha, groups=groups[:2],
                          scores=scores[:2], group=list(rg["group"]))
        log(f"variant {name}: score {res[name]['score_ms']:.3f} ms, greedy "
            f"{res[name]['greedy_ms']:.1f} ms")
        gg.close()
    out = {
        "metric": METRIC, "value": edges / wall / 1e9, "unit": "GTEPS", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper variants: directed R-MAT s17 ef8, weighted BA n=1e5 "
                               "m=5 (D^-1/2 A D^-1/2), spectral bound and stochastic greedy "
                               "(eta=0.1) on BA n=1e5 m=5; 16 scores |S|=5 + greedy k=10 each",
                   "parallelism": "single GPU"},
        "variants": res, "host": host_cpu(),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = variants_cpu_baseline(runs, k, inputs)
    return out


def variants_cpu_baseline(runs, k, inputs):
    """The oracle on the variants' calls, one at a time on one core: two of
    each variant's scores and its whole greedy, with their agreement with the
    GPU's results (scores' largest relative difference, identical groups)."""
    import oracle
    per, edges, dt = {}, 0.0, 0.0
    for name, r in runs.items():
        g, wt, sigma, alpha = r["g"], r["wt"], r["sigma"], r["alpha"]
        t = time.perf_counter()
        osc = [oracle.score(g, S, alpha, EPS, w=wt, sigma=sigma) for S in r["groups"]]
        o_score = (time.perf_counter() - t) / len(r["groups"])
        dt += o_score * len(r["groups"])
        edges += sum(x[1] for x in osc) * g.nnz
        t = time.perf_counter()
        if name == "stochastic":
            ro = oracle.greedy(g, k, alpha, EPS, stochastic=True, eta=0.1, seed=1)
        else:
            rev = inputs.reverse(g) if g.directed else None
            ro = oracle.greedy(g, k, alpha, EPS, rev=rev, w=wt, w_rev=wt, sigma=sigma)
        o_greedy = time.perf_counter() - t
        rel = max(abs(a - b[0]) / max(abs(a), abs(b[0]), 1e-300)
                  for a, b in zip(r["scores"], osc))
        per[name] = {"oracle_score_s": o_score, "oracle_greedy_s": o_greedy,
                     "scores_max_rel_vs_oracle": rel,
                     "greedy_same_as_oracle": r["group"] == list(ro["group"])}
        log(f"variant {name}: oracle {o_score:.2f} s / {o_greedy:.1f} s")
    return {"value": edges / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "two single-group scores (|S|=5) per variant by the single-threaded FP64 "
                      "oracle, one at a time; and each variant's greedy k=10 (per_variant)",
            "per_variant": per, "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22",
                    choices=["ba1m", "rmat22", "er1k", "batch", "serve", "variants"])
    ap.add_argument("--groups", type=int, default=4096)
    ap.add_argument("--tile", type=int, default=0,
                    help="batch, ba1m: fix the batched tile width (0 = autotune)")
    ap.add_argument("--buckets", type=int, default=None,
                    help="source-bucket bytes of the long rows (0 = library's choice, "
                         "-1 = off)")
    ap.add_argument("--greedy-width", type=int, default=0,
                    help="candidates per gain SpMM of the greedy (0 = the library's choice)")
    ap.add_argument("--seq-sample", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true",
                    help="rmat22: skip the batched-scoring context keys")
    ap.add_argument("--order", choices=("degree", "input"), default="degree",
                    help="internal vertex order: degree-descending relabel (default) or the "
                         "generator's order")
    ap.add_argument("--requests", type=int, default=1000, help="serve: requests in the stream")
    ap.add_argument("--qps", type=float, default=2000.0, help="serve: arrival rate")
    ap.add_argument("--greedy-frac", type=float, default=0.1,
                    help="serve: fraction of greedy requests in the stream")
    ap.add_argument("--serve-small", action="store_true", help="serve: only the 3 small graphs")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the walk-count hot path runs on one GPU; multi-GPU runs are not "
              "supported (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    from paper_1910_13874_amd import ged, inputs
    if args.copy_calib:
        a = torch.empty(256 * 2 ** 20 // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batch":
        out = bench_batch(args, torch, ged, inputs)
    elif args.workload == "variants":
        out = bench_variants(args, torch, ged, inputs)
    elif args.workload == "serve":
        from paper_1910_13874_amd import serve
        out = serve.bench(args, torch, ged, inputs, METRIC)
    else:
        out = bench_graph_workload(args, torch, ged, inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
