"""Serving workload: a Poisson request stream over resident graphs.

The server itself is native (C ABI ``ged_server_*``); this module generates
the seeded request stream, feeds it at its arrival times, collects latencies,
and replays the same stream through a one-at-a-time loop of plain
``ged_score`` / ``ged_greedy`` calls for comparison.
"""
from __future__ import annotations

import time

import numpy as np

SERVE_GRAPHS = ["er10k", "er100k", "ba100k", "ba1m_m8", "ba2m_m16", "rmat17", "rmat20", "rmat22"]
GREEDY_KS = (5, 20, 100)


def make_requests(ns, n_req, qps, seed, greedy_frac=0.1, smax=100):
    """Seeded stream: exponential inter-arrival gaps at rate qps, graph uniform,
    a fraction greedy_frac of greedy requests with k uniform over GREEDY_KS, the
    rest scores with |S| ~ U[1, smax]."""
    from . import inputs
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    gid = rng.integers(0, len(ns), size=n_req)
    kind = (rng.random(n_req) < greedy_frac).astype(int)
    reqs = []
    for j in range(n_req):
        n = ns[gid[j]]
        if kind[j] == 0:
            size = int(rng.integers(1, smax + 1))
            S = inputs.group(n, min(size, n), seed * 1000003 + j)
            reqs.append({"t": float(t[j]), "g": int(gid[j]), "kind": 0, "S": S})
        else:
            k = int(GREEDY_KS[rng.integers(0, len(GREEDY_KS))])
            reqs.append({"t": float(t[j]), "g": int(gid[j]), "kind": 1, "k": min(k, n)})
    return reqs


def run_server(server, gids, reqs):
    """Submit at the arrival times, collect every result.  Returns
    {request index: (kind, status, score, latency_s, group or None)}."""
    by_id = {}
    out = {}
    t0 = time.perf_counter()
    pending = 0

    def drain(timeout_us=0):
        nonlocal pending
        for r in server.poll(4096, timeout_us):
            j = by_id.pop(r.id)
            grp = server.group(r.id, r.k) if (r.kind == 1 and r.status == 0) else None
            out[j] = (r.kind, r.status, r.score, (r.t_done_us - r.t_submit_us) * 1e-6, grp)
            pending -= 1

    for j, q in enumerate(reqs):
        while time.perf_counter() - t0 < q["t"]:
            drain(0)
        if q["kind"] == 0:
            rid = server.submit_score(gids[q["g"]], q["S"])
        else:
            rid = server.submit_greedy(gids[q["g"]], q["k"])
        by_id[rid] = j
        pending += 1
    while pending:
        drain(100000)
    wall = time.perf_counter() - t0
    return out, wall


def run_plain(graphs, alphas, reqs, eps):
    """One request at a time, FIFO, plain calls; latency counts queueing from
    the request's arrival time on a simulated clock fed by measured service times."""
    lat = {}
    clock = 0.0
    results = {}
    busy = 0.0
    for j, q in enumerate(reqs):
        start = max(clock, q["t"])
        t = time.perf_counter()
        gg = graphs[q["g"]]
        if q["kind"] == 0:
            res = gg.score(q["S"], alphas[q["g"]], eps)
        else:
            res = gg.greedy(q["k"], alphas[q["g"]], eps)
        dt = time.perf_counter() - t
        busy += dt
        clock = start + dt
        lat[j] = clock - q["t"]
        results[j] = res
    return lat, results, clock, busy


def _pct(x, p):
    return float(np.percentile(np.asarray(x), p)) if len(x) else None


def bench(args, torch, ged, inputs, metric):
    eps = 1e-4
    names = SERVE_GRAPHS if not getattr(args, "serve_small", False) else SERVE_GRAPHS[:3]
    graphs, alphas, ns = [], [], []
    t = time.perf_counter()
    for nm in names:
        g = inputs.workload_graph(nm)
        gg = ged.GedGraph.from_graph(g)
        graphs.append(gg)
        alphas.append(gg.default_alpha())
        ns.append(g.n)
    setup_s = time.perf_counter() - t
    # three greedy workers: greedy requests on one graph run one at a time (they
    # share its handle), those on different graphs overlap; more workers crowd
    # the device and delay the score tiles
    server = ged.Server(hbm_budget_bytes=200 << 30, greedy_workers=min(3, len(graphs)))
    gids = [server.add_graph(gg, a, eps) for gg, a in zip(graphs, alphas)]
    n_req = getattr(args, "requests", 1000)
    qps = getattr(args, "qps", 2000.0)
    gfrac = getattr(args, "greedy_frac", 0.1)
    reqs = make_requests(ns, n_req, qps, seed=105, greedy_frac=gfrac)
    # warm the pools and the greedy path once
    warm = make_requests(ns, 16, 1e6, seed=7, greedy_frac=0.0)
    run_server(server, gids, warm)
    out, wall = run_server(server, gids, reqs)
    stats = server.stats()
    server.close()
    lat_s = [out[j][3] for j in out if out[j][0] == 0]
    lat_g = [out[j][3] for j in out if out[j][0] == 1]
    n_score = len(lat_s)
    # the same stream through the one-at-a-time loop
    lat_plain, res_plain, plain_clock, plain_busy = run_plain(graphs, alphas, reqs, eps)
    pl_s = [lat_plain[j] for j in lat_plain if reqs[j]["kind"] == 0]
    pl_g = [lat_plain[j] for j in lat_plain if reqs[j]["kind"] == 1]
    maxrel = 0.0
    same_groups = True
    for j, q in enumerate(reqs):
        if q["kind"] == 0:
            a, b = out[j][2], res_plain[j]
            if a != b:
                maxrel = max(maxrel, abs(a - b) / max(abs(a), abs(b)))
        else:
            same_groups = same_groups and list(out[j][4]) == list(res_plain[j]["group"])
    for gg in graphs:
        gg.close()
    span = max(q["t"] for q in reqs)
    return {
        "metric": metric, "value": n_req / wall, "unit": "queries/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson stream of {n_req} requests at {qps:g} req/s "
                               f"over {len(names)} resident graphs ({', '.join(names)}); "
                               f"{100 * (1 - gfrac):g}% score |S|~U[1,100], {100 * gfrac:g}% "
                               "greedy k in {5,20,100}, eps=1e-4, FP64",
                   "requests": n_req, "qps": qps, "greedy_frac": gfrac, "graphs": names, "parallelism": "single GPU"},
        "served_queries_per_s": n_req / wall,
        "plain_queries_per_s": n_req / plain_clock,
        "served_vs_plain": (n_req / wall) / (n_req / plain_clock),
        "score_ms_p50": _pct(lat_s, 50) * 1e3, "score_ms_p99": _pct(lat_s, 99) * 1e3,
        "greedy_ms_p50": _pct(lat_g, 50) * 1e3 if lat_g else None,
        "greedy_ms_p99": _pct(lat_g, 99) * 1e3 if lat_g else None,
        "plain_score_ms_p50": _pct(pl_s, 50) * 1e3, "plain_score_ms_p99": _pct(pl_s, 99) * 1e3,
        "plain_greedy_ms_p50": _pct(pl_g, 50) * 1e3 if pl_g else None,
        "plain_greedy_ms_p99": _pct(pl_g, 99) * 1e3 if pl_g else None,
        "score_requests": n_score, "greedy_requests": len(lat_g),
        "arrival_span_s": span, "served_wall_s": wall, "plain_wall_s": plain_clock,
        "plain_busy_s": plain_busy, "server_stats": stats,
        "served_vs_plain_score_max_rel": maxrel, "served_vs_plain_greedy_identical": same_groups,
        "setup_s": setup_s,
    }
