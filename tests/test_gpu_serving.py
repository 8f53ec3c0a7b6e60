"""Serving (continuous batching): every result equals the same request run
alone (scores to 1e-12, groups identical) and the CPU oracle on the same
graph, alpha and eps (scores to 1e-9 relative; greedy groups identical, with
the group's final score to 1e-9)."""
import numpy as np
import pytest

import oracle
from paper_1910_13874_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 1e-4
REL = 1e-9


def rel(a, b):
    return 0.0 if a == b else abs(a - b) / max(abs(a), abs(b))


class OracleCheck:
    """Checks served results against the oracle on the same graph, alpha and
    eps (directed graphs need the reverse graph for the greedy's backward
    chain; weighted graphs their arc weights)."""

    def __init__(self, g, alpha, w=None):
        self.g, self.alpha, self.w = g, alpha, w
        self.rev = inputs.reverse(g) if g.directed else None
        self.greedy_cache = {}

    def score(self, S, served, tag):
        c, ell, B, _ = oracle.score(self.g, S, self.alpha, EPS, w=self.w)
        assert rel(served, c) <= REL, (tag, served, c)

    def greedy(self, k, grp, served_score, tag):
        if k not in self.greedy_cache:
            self.greedy_cache[k] = oracle.greedy(self.g, k, self.alpha, EPS, rev=self.rev,
                                                 w=self.w, w_rev=self.w)
        ro = self.greedy_cache[k]
        assert [int(x) for x in grp] == [int(x) for x in ro["group"]], (tag, grp, ro["group"])
        assert rel(served_score, ro["score"]) <= REL, (tag, served_score, ro["score"])


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_13874_amd import ged as mod
    return mod


def test_mix_equals_alone(ged):
    from paper_1910_13874_amd import serve
    gs = [inputs.erdos_renyi(20000, 100000, 21), inputs.barabasi_albert(50000, 5, 22)]
    ggs = [ged.GedGraph.from_graph(g) for g in gs]
    alphas = [gg.default_alpha() for gg in ggs]
    print("[serving mix] graphs", [g.n for g in gs], flush=True)
    srv = ged.Server(hbm_budget_bytes=8 << 30, score_slots=16, greedy_workers=2)
    gids = [srv.add_graph(gg, a, EPS) for gg, a in zip(ggs, alphas)]
    reqs = serve.make_requests([g.n for g in gs], 300, 5e4, seed=9, greedy_frac=0.03)
    reqs += [{"t": 0.0, "g": 0, "kind": 0, "S": np.zeros(0, dtype=np.int32)}]  # empty group
    out, wall = serve.run_server(srv, gids, reqs)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["peak_columns"] > 1
    orc = [OracleCheck(g, a) for g, a in zip(gs, alphas)]
    for j, q in enumerate(reqs):
        kind, status, score, lat, grp = out[j]
        assert status == 0
        if q["kind"] == 0:
            alone = ggs[q["g"]].score(q["S"], alphas[q["g"]], EPS)
            assert abs(score - alone) <= 1e-12 * max(abs(alone), 1e-300), (j, score, alone)
            orc[q["g"]].score(q["S"], score, j)
        else:
            alone = ggs[q["g"]].greedy(q["k"], alphas[q["g"]], EPS)
            assert list(grp) == list(alone["group"])
            assert abs(score - alone["score"]) <= 1e-12 * abs(alone["score"])
            orc[q["g"]].greedy(q["k"], grp, score, j)
    print(f"[serving mix] {len(reqs)} results checked against the oracle", flush=True)
    srv.close()
    for gg in ggs:
        gg.close()


def test_burst_fills_wide_tiles(ged):
    """Default lane width (64 columns for this size): a burst of scores runs
    as tiles of many widths, each result equal to the request alone."""
    from paper_1910_13874_amd import serve
    g = inputs.barabasi_albert(30000, 4, 23)
    gg = ged.GedGraph.from_graph(g)
    alpha = gg.default_alpha()
    print("[serving burst] n", g.n, flush=True)
    srv = ged.Server(hbm_budget_bytes=8 << 30, greedy_workers=1)
    gid = srv.add_graph(gg, alpha, EPS)
    reqs = serve.make_requests([g.n], 200, 1e7, seed=31, greedy_frac=0.0)
    out, wall = serve.run_server(srv, [gid], reqs)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["peak_columns"] > 32, st
    orc = OracleCheck(g, alpha)
    for j, q in enumerate(reqs):
        kind, status, score, lat, grp = out[j]
        assert status == 0
        alone = gg.score(q["S"], alpha, EPS)
        assert abs(score - alone) <= 1e-12 * max(abs(alone), 1e-300), (j, score, alone)
        orc.score(q["S"], score, j)
    srv.close()
    gg.close()


def test_admission_and_queue_limits(ged):
    g = inputs.barabasi_albert(200000, 4, 23)
    gg = ged.GedGraph.from_graph(g)
    # a budget that holds the score pool but no greedy working memory
    srv = ged.Server(hbm_budget_bytes=60 << 20, score_slots=8, max_queue=4, greedy_workers=1)
    gid = srv.add_graph(gg, None, EPS)
    with pytest.raises(ged.GedError) as e:
        srv.submit_greedy(gid, 5)
    assert e.value.code == -6
    with pytest.raises(ged.GedError) as e:
        srv.submit_score(gid, [g.n])
    assert e.value.code == -2
    assert srv.stats()["rejected"] == 1
    srv.close()
    srv2 = ged.Server(hbm_budget_bytes=4 << 30, score_slots=8, max_queue=2, greedy_workers=1)
    gid = srv2.add_graph(gg, None, EPS)
    busy = 0
    for j in range(64):
        try:
            srv2.submit_score(gid, [j])
        except ged.GedError as err:
            assert err.code == -8
            busy += 1
    assert busy > 0
    got = 0
    while got < 64 - busy:
        got += len(srv2.poll(64, 200000))
    srv2.close()
    gg.close()


@pytest.mark.parametrize("name", ["ba", "rmat", "directed", "weighted"])
def test_greedy_footprint_bounds_allocations(ged, name):
    """The greedy's memory estimate (what serving admission charges) bounds
    what a run leaves allocated, from a fresh handle, for several k; the
    workspace is kept for the next call, so a repeated run adds nothing."""
    if name == "ba":
        g, w = inputs.barabasi_albert(30000, 4, 41), None
    elif name == "rmat":
        g, w = inputs.rmat(15, 16, seed=42), None
    elif name == "directed":
        r = inputs.uniform_ints(2 * 60000, 8000, 43)
        g, w = inputs.from_edges(8000, r[0::2], r[1::2], symmetrize=False, name="dir8k"), None
    else:
        g = inputs.barabasi_albert(20000, 4, 44)
        deg = g.degrees.astype(np.float64)
        rows = np.repeat(np.arange(g.n), g.degrees)
        w = 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])
    gg = ged.GedGraph.from_graph(g, weights=w)
    alpha = gg.default_alpha()
    for k in (5, 40):
        est, held0 = gg.greedy_footprint(k, alpha, EPS)
        gg.greedy(k, alpha, EPS)
        _, held1 = gg.greedy_footprint(k, alpha, EPS)
        print(f"[footprint] {name} k={k}: estimate {est} held {held0} -> {held1}", flush=True)
        assert held1 <= est, (name, k, held1, est)
        gg.greedy(k, alpha, EPS)
        assert gg.greedy_footprint(k, alpha, EPS)[1] == held1
    gg.close()


def test_cancel_and_deadline(ged):
    """A greedy cancelled right after submission and one given a deadline 1 ms
    away both complete with their stop status (whether they were still
    waiting or already running: a running greedy stops before its next
    round), a later request on the same graph is still correct, and the
    server's counters add up."""
    import time
    g = inputs.barabasi_albert(200000, 4, 45)
    gg = ged.GedGraph.from_graph(g)
    alpha = gg.default_alpha()
    srv = ged.Server(hbm_budget_bytes=16 << 30, score_slots=8, greedy_workers=1)
    gid = srv.add_graph(gg, alpha, EPS)
    r1 = srv.submit_greedy(gid, 100)
    assert srv.cancel(r1) == 0
    r2 = srv.submit_greedy(gid, 100)
    # the server's clock is the steady clock (CLOCK_MONOTONIC), in microseconds
    assert srv.set_deadline(r2, time.monotonic() * 1e6 + 1000.0) == 0
    S = inputs.group(g.n, 20, 7)
    r3 = srv.submit_score(gid, S)
    r4 = srv.submit_greedy(gid, 5)
    got = {}
    t0 = time.time()
    while len(got) < 4 and time.time() - t0 < 60:
        for r in srv.poll(16, 100000):
            got[r.id] = (r.status, r.score)
    assert got[r1][0] == -10, got[r1]
    assert got[r2][0] == -11, got[r2]
    assert got[r3][0] == 0 and got[r4][0] == 0
    assert srv.cancel(r1) == -1  # finished
    c, _, _, _ = oracle.score(g, S, alpha, EPS)
    assert rel(got[r3][1], c) <= REL
    ro = oracle.greedy(g, 5, alpha, EPS)
    assert list(srv.group(r4, 5)) == [int(x) for x in ro["group"]]
    st = srv.stats()
    assert st["admitted"] == 4 and st["completed"] == 4
    srv.close()
    gg.prepare(alpha * 0.5, EPS)  # the handle is free again after destroy
    srv2, srv3 = ged.Server(), ged.Server()
    srv2.add_graph(gg, alpha, EPS)
    with pytest.raises(ged.GedError) as e:
        srv3.add_graph(gg, alpha, EPS)  # a handle serves one server at a time
    assert e.value.code == -8
    srv3.close()
    srv2.close()
    gg.close()


def test_served_handle_refuses_other_alpha(ged):
    """A registered handle keeps its (alpha, eps) until the server is gone."""
    g = inputs.barabasi_albert(20000, 4, 46)
    gg = ged.GedGraph.from_graph(g)
    alpha = gg.default_alpha()
    srv = ged.Server(hbm_budget_bytes=8 << 30)
    srv.add_graph(gg, alpha, EPS)
    assert gg.score([1, 2], alpha, EPS) > 0  # same alpha, eps: fine
    for call in (lambda: gg.score([1, 2], alpha * 0.5, EPS), gg.invalidate,
                 lambda: gg.set_tail_bound("spectral")):
        with pytest.raises(ged.GedError) as e:
            call()
        assert e.value.code == -8
    srv.close()
    assert gg.score([1, 2], alpha * 0.5, EPS) > 0
    gg.close()


def test_directed_and_weighted_lanes(ged):
    """A directed graph (level-by-level column pool) and a weighted undirected one
    (split tiles without integer levels) served side by side: every result equals
    the same request alone."""
    from paper_1910_13874_amd import serve
    r = inputs.uniform_ints(2 * 60000, 8000, 24)
    gd = inputs.from_edges(8000, r[0::2], r[1::2], symmetrize=False, name="dir8k")
    gw = inputs.barabasi_albert(30000, 4, 25)
    deg = gw.degrees.astype(np.float64)
    rows = np.repeat(np.arange(gw.n), gw.degrees)
    w = 1.0 / np.sqrt(deg[rows] * deg[gw.col_idx])
    ggs = [ged.GedGraph.from_graph(gd), ged.GedGraph.from_graph(gw, weights=w)]
    alphas = [gg.default_alpha() for gg in ggs]
    print("[serving directed+weighted]", [gd.n, gw.n], flush=True)
    srv = ged.Server(hbm_budget_bytes=8 << 30, score_slots=8, greedy_workers=2)
    gids = [srv.add_graph(gg, a, EPS) for gg, a in zip(ggs, alphas)]
    reqs = serve.make_requests([gd.n, gw.n], 160, 4e4, seed=11, greedy_frac=0.05)
    out, wall = serve.run_server(srv, gids, reqs)
    assert srv.stats()["completed"] == len(reqs)
    orc = [OracleCheck(gd, alphas[0]), OracleCheck(gw, alphas[1], w=w)]
    for j, q in enumerate(reqs):
        kind, status, score, lat, grp = out[j]
        assert status == 0
        if q["kind"] == 0:
            alone = ggs[q["g"]].score(q["S"], alphas[q["g"]], EPS)
            assert abs(score - alone) <= 1e-12 * max(abs(alone), 1e-300), (j, q["g"], score, alone)
            orc[q["g"]].score(q["S"], score, (j, q["g"]))
        else:
            alone = ggs[q["g"]].greedy(q["k"], alphas[q["g"]], EPS)
            assert list(grp) == list(alone["group"])
            orc[q["g"]].greedy(q["k"], grp, score, (j, q["g"]))
    srv.close()
    for gg in ggs:
        gg.close()
