"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (from the method's FP64 requirement): scores within 1e-9 relative and the
same ell*; greedy picks and walk lengths identical (ties within 1e-12 excepted).
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1910_13874_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4
REL = 1e-9
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_13874_amd import ged as mod
    return mod


def rel(a, b):
    if a == b:
        return 0.0
    return abs(a - b) / max(abs(a), abs(b))


def check_score(gg, g, S, alpha, eps=EPS, tag=""):
    s, ell, B = gg.score(S, alpha, eps, with_info=True)
    c, ell_o, B_o, _ = oracle.score(g, S, alpha, eps)
    assert ell == ell_o, (tag, ell, ell_o)
    assert rel(s, c) <= REL, (tag, s, c, rel(s, c))
    assert rel(B, B_o) <= 1e-9
    return s


GRAPHS = {
    "er1k": lambda: inputs.erdos_renyi(1000, 5000, 1),
    "ba20k": lambda: inputs.barabasi_albert(20000, 5, 2),
    "rmat16": lambda: inputs.rmat(16, 16, seed=18),
    "er_sparse": lambda: inputs.erdos_renyi(3000, 2000, 7),  # many isolated vertices
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_score_parity(ged, name):
    g = GRAPHS[name]()
    say(f"[score parity] {name} n={g.n} nnz={g.nnz} dmax={g.max_degree}")
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    for seed, size in [(101, 5), (7, 1), (8, 37), (9, 200), (10, min(g.n, 1000))]:
        check_score(gg, g, inputs.group(g.n, size, seed), alpha, tag=(name, seed, size))
    # empty group, full vertex set, duplicates
    assert gg.score([], alpha, EPS) == 0.0
    full = gg.score(np.arange(g.n), alpha, EPS)
    c_full = oracle.score(g, np.arange(g.n), alpha, EPS)[0]
    assert rel(full, c_full) <= REL
    S = inputs.group(g.n, 10, 3)
    dup = np.concatenate([S, S[:4]])
    assert gg.score(dup, alpha, EPS) == gg.score(S, alpha, EPS)
    # a different eps re-prepares ell*
    check_score(gg, g, S, alpha, eps=1e-8, tag=(name, "eps1e-8"))
    check_score(gg, g, S, alpha, eps=EPS, tag=(name, "eps back"))
    gg.close()


def test_scores_across_streams(ged):
    """Scores issued back to back on one stream, then on another stream after
    ged_set_stream, then on the handle's own stream again: each call leaves its
    clean-up running on the stream it used, and every score still equals the
    oracle's (the switch waits for the old stream)."""
    import torch
    g = GRAPHS["ba20k"]()
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    groups = [inputs.group(g.n, size, 300 + size) for size in (1, 5, 40, 400)]
    ref = [oracle.score(g, S, alpha, EPS)[0] for S in groups]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for st in (None, s1, s2, None, s1):
        gg.set_stream(st)
        for S, c in zip(groups, ref):
            assert rel(gg.score(S, alpha, EPS), c) <= REL
        for S, c in zip(reversed(groups), reversed(ref)):
            assert rel(gg.score(S, alpha, EPS), c) <= REL
    gg.close()


def test_score_deterministic_and_alpha_change(ged):
    g = GRAPHS["rmat16"]()
    gg = ged.GedGraph.from_graph(g)
    S = inputs.group(g.n, 20, 44)
    a1 = g.default_alpha()
    x = [gg.score(S, a1, EPS) for _ in range(3)]
    assert x[0] == x[1] == x[2]
    check_score(gg, g, S, a1 / 3, tag="alpha/3")
    assert gg.score(S, a1, EPS) == x[0]
    gg.close()


def directed_graph():
    """Directed G(n, M)-like graph: 2,000 vertices, 9,000 uniform arcs, seed 61."""
    n = 2000
    r = inputs.uniform_ints(2 * 9000, n, 61)
    return inputs.from_edges(n, r[0::2], r[1::2], symmetrize=False, name="dir2k")


def test_directed_score_and_greedy(ged):
    g = directed_graph()
    n = g.n
    rev = inputs.reverse(g)
    say(f"[directed] n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g)
    alpha = oracle.default_alpha(g)
    assert abs(gg.default_alpha() - alpha) == 0.0
    for seed, size in [(1, 3), (2, 40)]:
        S = inputs.group(n, size, seed)
        check_score(gg, g, S, alpha, tag=("dir", seed))
        s, ell, B = gg.score(S, alpha, EPS, with_info=True)
        check_by_complement(g, S, alpha, ell, s, ("dir", seed))
    rg = gg.greedy(5, alpha, EPS)
    ro = oracle.greedy(g, 5, alpha, EPS, rev=rev)
    assert list(rg["group"]) == list(ro["group"])
    assert list(rg["ell"]) == list(ro["ell"])
    gg.close()


def test_edgeless_and_tiny(ged):
    g = inputs.from_edges(5, [], [], symmetrize=True)
    gg = ged.GedGraph.from_graph(g)
    assert gg.score([0, 3], 0.5, EPS) == 0.0
    r = gg.greedy(2, 0.5, EPS)
    assert list(r["group"]) == [0, 1]
    gg.close()
    k2 = inputs.from_edges(2, [0], [1])
    gk = ged.GedGraph.from_graph(k2)
    s = gk.score([0], 0.4, 1e-12)
    assert abs(s - 2 * 0.4 / 0.6) <= 1e-11  # 2 walks of every length touch vertex 0
    gk.close()


def test_errors(ged):
    g = GRAPHS["er1k"]()
    gg = ged.GedGraph.from_graph(g)
    with pytest.raises(ged.GedError) as e:
        gg.score([g.n], g.default_alpha(), EPS)
    assert e.value.code == -2
    with pytest.raises(ged.GedError) as e:
        gg.score([1], 1.0 / g.max_degree, EPS)
    assert e.value.code == -3
    with pytest.raises(ged.GedError) as e:
        gg.score([1], g.default_alpha(), 0.0)
    assert e.value.code == -4
    with pytest.raises(ged.GedError) as e:
        gg.greedy(g.n + 1, g.default_alpha(), EPS)
    assert e.value.code == -1
    # still usable after errors
    check_score(gg, g, [1, 2, 3], g.default_alpha())
    gg.close()
    # malformed CSR
    with pytest.raises(ged.GedError) as e:
        ged.GedGraph(3, np.array([0, 1, 2, 3]), np.array([1, 2, 2]))  # self-loop at 2
    assert e.value.code == -5
    with pytest.raises(ged.GedError) as e:
        ged.GedGraph(3, np.array([0, 1, 1, 1]), np.array([1]))  # not symmetric
    assert e.value.code == -5


def compare_greedy(rg, ro, tag):
    assert list(rg["group"]) == list(ro["group"]), (tag, rg["group"], ro["group"])
    assert list(rg["ell"]) == list(ro["ell"]), (tag, rg["ell"], ro["ell"])
    for j in range(len(rg["group"])):
        assert rel(rg["L1"][j], ro["L1"][j]) <= REL, (tag, j, rg["L1"][j], ro["L1"][j])
        if not np.isnan(ro["U2"][j]):
            assert rel(rg["U2"][j], ro["U2"][j]) <= REL
    assert rel(rg["score"], ro["score"]) <= REL
    assert rg["score_ell"] == ro["score_ell"]


# ba20k: the first candidate batches (hubs) take the dense second gain level,
# later ones the pushed one, so k = 20 moves between the two many times
# rmat15: from pick 2 on ell = 16 and omega_4 > 2^32, so the candidate batches
# run FP64 gain levels carrying speculative miss columns, and most picks take
# their miss levels from the winner's column
@pytest.mark.parametrize("name,k", [("er1k", 5), ("ba20k", 10), ("ba20k", 20), ("rmat16", 8),
                                    ("er_sparse", 6), ("rmat15", 8)])
def test_greedy_parity(ged, name, k):
    g = GRAPHS[name]() if name in GRAPHS else inputs.rmat(15, 16, seed=42)
    say(f"[greedy parity] {name} k={k}")
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    rg = gg.greedy(k, alpha, EPS)
    ro = oracle.greedy(g, k, alpha, EPS)
    compare_greedy(rg, ro, name)
    gg.close()


@pytest.mark.parametrize("width", [0, 2, 4, 8, 16])
def test_greedy_width_parity(ged, width):
    """The candidate batch width changes how many gains one SpMM evaluates,
    not the decisions: every fixed width, and the default that widens a
    round's batches 2, 4, 8, 16 (width 0; the double star's exact ties need
    several batches in one round), gives the oracle's picks, walk lengths and
    gains, on graphs whose batches take the 32-bit count levels (ER), the
    pushed and dense second gain levels (BA), FP64 levels (R-MAT), and the
    level-by-level chains of a directed graph."""
    cases = [("ba20k", GRAPHS["ba20k"](), 10), ("rmat16", GRAPHS["rmat16"](), 8),
             ("er_sparse", inputs.erdos_renyi(3000, 4500, 57), 6)]
    for name, g, k in cases:
        say(f"[greedy width {width}] {name} k={k}")
        gg = ged.GedGraph.from_graph(g)
        gg.set_greedy_width(width)
        assert gg.greedy_width() == (width or (8 if g.nnz <= 1 << 20 else 2))
        alpha = g.default_alpha()
        compare_greedy(gg.greedy(k, alpha, EPS), oracle.greedy(g, k, alpha, EPS),
                       f"{name} width {width}")
        gg.close()
    if width == 0:
        # above 2^20 arcs (a cycle of 600,000 vertices) three identical stars
        # K_{1,50}: their centres tie exactly, so a round's first batch of 2
        # cannot settle the runner-up and the round widens
        nc_ = 600_000
        src = list(range(nc_))
        dst = [(v + 1) % nc_ for v in range(nc_)]
        for c in range(3):
            ctr = nc_ + 51 * c
            src += [ctr] * 50
            dst += list(range(ctr + 1, ctr + 51))
        tied = inputs.from_edges(nc_ + 153, np.array(src, np.int32), np.array(dst, np.int32),
                                 name="cycle+3stars")
        assert tied.nnz > 1 << 20
        gg = ged.GedGraph.from_graph(tied)
        assert gg.greedy_width() == 2
        alpha = tied.default_alpha()
        r = gg.greedy(2, alpha, EPS)
        say(f"[greedy widening] picks {list(r['group'])} evals {list(r['evals'])} "
            f"rounds {r['rounds']}")
        compare_greedy(r, oracle.greedy(tied, 2, alpha, EPS), "tied stars, widening")
        assert r["evals"][-1] > 2 * r["rounds"], (r["evals"], r["rounds"])
        gg.close()
    gd = directed_graph()
    rev = inputs.reverse(gd)
    say(f"[greedy width {width}] directed n={gd.n}")
    gg = ged.GedGraph.from_graph(gd)
    gg.set_greedy_width(width)
    alpha = oracle.default_alpha(gd, None)
    compare_greedy(gg.greedy(6, alpha, EPS), oracle.greedy(gd, 6, alpha, EPS, rev=rev),
                   f"directed width {width}")
    gg.close()


def ba_multigraph():
    """BA(3000, 3) with 200 of its edges listed twice (both directions)."""
    g0 = inputs.barabasi_albert(3000, 3, 58)
    rows = [list(g0.col_idx[g0.row_ptr[v]:g0.row_ptr[v + 1]]) for v in range(g0.n)]
    rng = np.random.default_rng(58)
    for v in rng.choice(g0.n, 200, replace=False):
        u = rows[v][0]  # double the arc v-u in both directions
        rows[v].append(u)
        rows[u].append(int(v))
    rows = [sorted(r) for r in rows]
    rp = np.zeros(g0.n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.fromiter((u for r in rows for u in r), dtype=np.int32, count=int(rp[-1]))
    return inputs.Graph(n=g0.n, row_ptr=rp, col_idx=ci, name="ba_multi")


def test_greedy_multigraph(ged):
    """A graph with doubled arcs: the first gain level cannot be a push of
    single walks, so the greedy keeps the dense one-hot step; picks, walk
    lengths and gains still match the oracle (which counts every listed arc)."""
    g = ba_multigraph()
    say(f"[greedy multigraph] n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g)
    alpha = oracle.default_alpha(g, None)
    rg = gg.greedy(6, alpha, EPS)
    ro = oracle.greedy(g, 6, alpha, EPS)
    compare_greedy(rg, ro, "multigraph")
    gg.close()


def test_greedy_gain_layout(ged):
    """The greedy's gain and miss levels as 32-bit counts: on a sparse
    Erdos-Renyi graph (max degree 11, omega_13 < 2^32) every walk length the
    greedy reaches keeps its gain levels (up to ceil(ell/2) - 1) and miss
    levels (up to ceil(ell/2)) below 2^32, so the profiled dominant step
    kernel is one of the 32-bit gain, gain-combination or miss kernels (their
    times are close on a graph this small); picks, lengths and gains match the
    oracle."""
    g = inputs.erdos_renyi(3000, 4500, 57)
    om = omega_max(g, 20)
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    gg.prepare(alpha, EPS)
    gg.profile_enable(True)
    rg = gg.greedy(6, alpha, EPS, with_score=False)
    kind = gg.profile_read()["dominant_kind"]
    gg.profile_enable(False)
    ro = oracle.greedy(g, 6, alpha, EPS)
    rg_full = gg.greedy(6, alpha, EPS)
    compare_greedy(rg_full, ro, "gain layout")
    assert list(rg["group"]) == list(ro["group"])
    top = (max(int(e) for e in rg["ell"]) + 1) // 2 - 1
    say(f"[gain layout] ells={list(rg['ell'])} kind={kind} top={top}")
    assert all(om[i] < 2.0 ** 32 for i in range(3, top + 2))
    assert top * (g.max_degree + 3) + 2 < 2 ** 19
    assert kind % ged.KIND_BASE in (11, 12, 13, 15), kind
    gg.close()


def test_greedy_forced_prefix(ged):
    g = GRAPHS["ba20k"]()
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    full = gg.greedy(6, alpha, EPS)
    rep = gg.greedy(6, alpha, EPS, forced=full["group"][:3], forced_ell=int(full["ell"][2]))
    assert list(rep["group"]) == list(full["group"])
    gg.close()


def test_greedy_ties_smallest_id(ged):
    src = [0, 0, 0, 4, 4, 4]
    dst = [1, 2, 3, 5, 6, 7]
    g = inputs.from_edges(8, src, dst)
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    r = gg.greedy(4, alpha, EPS)
    assert list(r["group"]) == [0, 4, 1, 2]
    ro = oracle.greedy(g, 4, alpha, EPS)
    compare_greedy(r, ro, "double star")
    gg.close()


def test_batch_matches_solo_and_oracle(ged):
    g = GRAPHS["ba20k"]()
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    off, mem = inputs.groups(g.n, 150, 1, 200, 104)
    # add an empty group at the end
    off = np.concatenate([off, [off[-1]]])
    say(f"[batch] groups={len(off) - 1}")
    b = gg.score_batch(off, mem, alpha, EPS)
    tile = gg.batch_tile()
    assert tile in (4, 8, 16, 32, 64)
    for j in range(len(off) - 1):
        S = mem[off[j]:off[j + 1]]
        solo = gg.score(S, alpha, EPS)
        assert rel(b[j], solo) <= 1e-12, (j, b[j], solo)
        if j % 25 == 0:
            c = oracle.score(g, S, alpha, EPS)[0]
            assert rel(b[j], c) <= REL
    assert b[-1] == 0.0
    # a second, smaller call reuses the workspace; its tiles keep the same
    # width, so each group's score is bit-identical to the larger call's
    b2 = gg.score_batch(off[:6], mem[:off[5]], alpha, EPS)
    np.testing.assert_array_equal(b2, b[:5])
    gg.close()


@pytest.mark.parametrize("name,nbytes", [("rmat16", 4096), ("ba20k", 65536), ("star", 512),
                                         ("directed", 2048)])
def test_source_buckets_parity(ged, name, nbytes):
    """Every path with the long rows' arcs grouped by source (forced, with
    small buckets so that rows split into many pieces): single scores, a
    batch, the greedy (gain batches, miss chains; the reverse graph when
    directed) against the oracle, and against the same graph without
    buckets (rounding only).  Setting the layout once a partition exists is
    refused."""
    if name == "star":
        g = inputs.from_edges(9000, np.zeros(8999, np.int32), np.arange(1, 9000, dtype=np.int32),
                              name="star9k")
    elif name == "directed":
        g = directed_graph()
    else:
        g = GRAPHS[name]()
    say(f"[source buckets] {name} n={g.n} nnz={g.nnz} bucket bytes={nbytes}")
    gb = ged.GedGraph.from_graph(g)
    gb.set_source_buckets(nbytes)
    assert gb.source_buckets() == nbytes
    gp = ged.GedGraph.from_graph(g)
    gp.set_source_buckets(-1)
    alpha = oracle.default_alpha(g)
    rev = inputs.reverse(g) if g.directed else None
    for seed, size in [(11, 1), (12, 5), (13, 40), (14, 300)]:
        S = inputs.group(g.n, size, seed)
        s = check_score(gb, g, S, alpha, tag=(name, seed))
        assert rel(s, gp.score(S, alpha, EPS)) <= 1e-12
    with pytest.raises(ged.GedError) as e:
        gb.set_source_buckets(0)
    assert e.value.code == -8
    off, mem = inputs.groups(g.n, 40, 1, 120, 170)
    b = gb.score_batch(off, mem, alpha, EPS)
    bp = gp.score_batch(off, mem, alpha, EPS)
    for j in range(len(off) - 1):
        assert rel(b[j], bp[j]) <= 1e-12, (j, b[j], bp[j])
        if j % 8 == 0:
            assert rel(b[j], oracle.score(g, mem[off[j]:off[j + 1]], alpha, EPS)[0]) <= REL
    np.testing.assert_array_equal(gb.score_batch(off, mem, alpha, EPS), b)
    k = 8
    rg = gb.greedy(k, alpha, EPS)
    ro = oracle.greedy(g, k, alpha, EPS, rev=rev)
    compare_greedy(rg, ro, name)
    assert list(gp.greedy(k, alpha, EPS)["group"]) == list(rg["group"])
    gb.close()
    gp.close()


# ------------------------------------------------------------ full sizes --

def load_golden(name):
    p = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(p):
        pytest.skip(f"{p} not generated")
    with open(p) as f:
        return json.load(f)


def check_by_complement(g, S, alpha, ell, score, tag, w=None):
    """Pinned without the oracle: all walks minus the walks of the subgraph
    induced by V \\ S (weighted by the product of arc weights when given)."""
    from closed_forms import group_score
    c = group_score(g, S, alpha, ell, w=w)
    say(f"  complement {tag}: |S|={len(S)} score={score!r} closed form={c!r}")
    assert rel(score, c) <= REL, (tag, score, c)


def check_gains_by_complement(g, rg, alpha, picks, tag):
    """Full size, pinned without the oracle: each pick's recorded gain is the
    count of walks that avoid the previous picks and meet this one.  picks is
    a count (the first picks) or a list of pick indices."""
    from closed_forms import gain
    for j in (range(picks) if isinstance(picks, int) else picks):
        grp = rg["group"]
        c = gain(g, grp[:j], int(grp[j]), alpha, int(rg["ell"][j]))
        say(f"  gain {tag} pick {j}: ell={rg['ell'][j]} L={rg['L1'][j]!r} closed form={c!r}")
        assert rel(rg["L1"][j], c) <= REL, (tag, j, rg["L1"][j], c)


def check_whole_set(gg, g, alpha):
    """Full size, pinned without the oracle: the score of the whole vertex set
    is the alpha-weighted count of all walks up to ell*."""
    from closed_forms import whole_set_score
    s, ell, B = gg.score(np.arange(g.n, dtype=np.int32), alpha, EPS, with_info=True)
    c = whole_set_score(g, alpha, ell)
    say(f"  whole set: ell={ell} score={s!r} closed form={c!r}")
    assert rel(s, c) <= REL, (s, c)


@pytest.mark.timeout(600)
def test_full_size_ba1m(ged):
    """BA n=1e6, m=5 at full size: oracle scores and the oracle's greedy k=10 trace."""
    gold = load_golden("ba1m")
    g = inputs.workload_graph("ba1m")
    assert g.fingerprint() == gold["fingerprint"]
    say(f"[full ba1m] n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g)
    alpha = gold["alpha"]
    for rec in gold["scores"]:
        S = inputs.group(g.n, rec["size"], rec["seed"])
        s, ell, B = gg.score(S, alpha, EPS, with_info=True)
        assert ell == rec["ell"] and rel(s, rec["score"]) <= REL, (rec["seed"], s, rec["score"])
        check_by_complement(g, S, alpha, ell, s, rec["seed"])
    check_whole_set(gg, g, alpha)
    gr = gold["greedy"]
    rg = gg.greedy(gr["k"], alpha, EPS)
    compare_greedy(rg, gr, "ba1m")
    check_gains_by_complement(g, rg, alpha, gr["k"], "ba1m")
    gg.close()


@pytest.mark.timeout(600)
def test_full_size_batch_ba2m(ged):
    """The batched workload at full size (BA n=2e6, m=8, 4,096 groups |S|~U[1,200])
    with the autotuned tile: sampled columns against the oracle, every column
    against its solo score, and a repeated call bit for bit."""
    gold = load_golden("ba2m")
    g = inputs.workload_graph("ba2m")
    assert g.fingerprint() == gold["fingerprint"]
    say(f"[full ba2m batch] n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g)
    alpha = gold["alpha"]
    bt = gold["batch"]
    off, mem = inputs.groups(g.n, bt["groups"], 1, 200, bt["seed"])
    b = gg.score_batch(off, mem, alpha, EPS)
    say(f"  tile {gg.batch_tile()}")
    for q, rec in enumerate(bt["sample"]):
        j = rec["index"]
        assert off[j + 1] - off[j] == rec["size"]
        assert rel(b[j], rec["score"]) <= REL, (j, b[j], rec["score"])
        if q < 3:
            check_by_complement(g, mem[off[j]:off[j + 1]], alpha, gg.prepare(alpha, EPS)[0],
                                b[j], j)
    for j in range(len(off) - 1):
        solo = gg.score(mem[off[j]:off[j + 1]], alpha, EPS)
        assert rel(b[j], solo) <= 1e-12, (j, b[j], solo)
    np.testing.assert_array_equal(gg.score_batch(off, mem, alpha, EPS), b)
    # the whole vertex set as a batch of one, and as a single score: the
    # closed form (all walks), pinned without the oracle
    from closed_forms import whole_set_score
    whole = np.arange(g.n, dtype=np.int32)
    bw = gg.score_batch(np.array([0, g.n], dtype=np.int64), whole, alpha, EPS)
    s, ell, B = gg.score(whole, alpha, EPS, with_info=True)
    c = whole_set_score(g, alpha, ell)
    say(f"  whole set: ell={ell} batch={bw[0]!r} single={s!r} closed form={c!r}")
    assert rel(bw[0], c) <= REL and rel(s, c) <= REL, (bw[0], s, c)
    gg.close()


@pytest.mark.timeout(900)
def test_full_size_rmat22(ged):
    """R-MAT scale 22 at full size (the greedy k=100 workload): oracle scores,
    the oracle's whole k=100 trace (picks, walk lengths, L1, U2, L2 at every
    pick, through the doubling of ell from 8 to 16), and the recorded gains of
    picks at both walk lengths against the complement closed form."""
    gold = load_golden("rmat22")
    gk = load_golden("rmat22_k100")
    g = inputs.workload_graph("rmat22")
    assert g.fingerprint() == gold["fingerprint"]
    say(f"[full rmat22] n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g)
    alpha = gold["alpha"]
    for rec in gold["scores"]:
        S = inputs.group(g.n, rec["size"], rec["seed"])
        s, ell, B = gg.score(S, alpha, EPS, with_info=True)
        assert ell == rec["ell"] and rel(s, rec["score"]) <= REL, (rec["seed"], s, rec["score"])
        check_by_complement(g, S, alpha, ell, s, rec["seed"])
    check_whole_set(gg, g, alpha)
    k = 100
    assert gk["fingerprint"] == gold["fingerprint"] and gk["k"] == k
    rg = gg.greedy(k, alpha, EPS)
    kk = len(gk["group"])
    say(f"  oracle trace: {kk} of {k} picks stored, ells {sorted(set(gk['ell']))}")
    assert kk >= 1
    for j in range(kk):
        assert int(rg["group"][j]) == gk["group"][j], (j, rg["group"][j], gk["group"][j])
        assert int(rg["ell"][j]) == gk["ell"][j], (j, rg["ell"][j], gk["ell"][j])
        assert rel(rg["L1"][j], gk["L1"][j]) <= REL, (j, rg["L1"][j], gk["L1"][j])
        if gk["U2"][j] == gk["U2"][j]:  # not NaN
            assert rel(rg["U2"][j], gk["U2"][j]) <= REL, (j, rg["U2"][j], gk["U2"][j])
            assert rel(rg["L2"][j], gk["L2"][j]) <= REL, (j, rg["L2"][j], gk["L2"][j])
    if "score" in gk:
        assert rel(rg["score"], gk["score"]) <= REL and rg["score_ell"] == gk["score_ell"]
    check_gains_by_complement(g, rg, alpha, [j for j in (0, 1, 6, 50, 99) if j < kk], "rmat22")
    # any-size properties of the whole run
    assert len(set(int(x) for x in rg["group"])) == k
    assert np.all(np.diff(rg["ell"]) >= 0)
    for j in range(k):
        assert rg["L1"][j] > rg["U2"][j] - EPS / k
        assert rg["L1"][j] >= rg["L2"][j]
    # the greedy's score is the plain score of its group
    assert rg["score"] == gg.score(rg["group"], alpha, EPS)
    gg.close()


def test_weighted_parity(ged):
    """Weighted variant with the paper's symmetric normalisation D^-1/2 A D^-1/2."""
    g = inputs.barabasi_albert(20000, 4, 33)
    deg = g.degrees.astype(np.float64)
    rows = np.repeat(np.arange(g.n), g.degrees)
    w = 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])
    say(f"[weighted] n={g.n}")
    gg = ged.GedGraph.from_graph(g, weights=w)
    alpha = 0.5 / oracle.max_weighted_out_degree(g, w)
    for seed, size in [(1, 3), (2, 50), (3, 500)]:
        S = inputs.group(g.n, size, seed)
        s, ell, B = gg.score(S, alpha, EPS, with_info=True)
        c, ell_o, B_o, _ = oracle.score(g, S, alpha, EPS, w=w)
        assert ell == ell_o and rel(s, c) <= REL, (seed, s, c)
        check_by_complement(g, S, alpha, ell, s, ("weighted", seed), w=w)
    rg = gg.greedy(5, alpha, EPS)
    ro = oracle.greedy(g, 5, alpha, EPS, w=w)
    compare_greedy(rg, ro, "weighted")
    gg.close()


def test_stochastic_greedy_parity(ged):
    g = GRAPHS["ba20k"]()
    gg = ged.GedGraph.from_graph(g)
    alpha = g.default_alpha()
    for eta, seed in [(0.5, 3), (0.05, 11)]:
        rg = gg.greedy_stochastic(8, alpha, EPS, eta=eta, seed=seed)
        ro = oracle.greedy(g, 8, alpha, EPS, stochastic=True, eta=eta, seed=seed)
        compare_greedy(rg, ro, f"stochastic eta={eta}")
    gg.close()


@pytest.mark.parametrize("name", ["er", "ba", "weighted", "hub", "rmat"])
def test_split_ell_sweep(ged, name):
    """Split scoring for every plan shape: ell* = 1..9 (a = 1, 2, 3+; odd and
    even ell; integer levels s = 0, 1, 2; weighted has s = 0), single and
    batched, against the oracle.  "hub" has a vertex of degree 70,000 and a few
    doubled arcs, which takes the 64-bit count path (32-bit counts need max
    degree < 2^16 or no duplicate arcs); "rmat" takes 32-bit counts through
    the no-duplicates rule (its max degree is below 2^16 too at this size, so it
    mainly adds an R-MAT degree profile)."""
    if name == "er":
        g, w = inputs.erdos_renyi(3000, 12000, 51), None
    elif name == "rmat":
        g, w = inputs.rmat(17, 16, seed=54), None
    elif name == "hub":
        rng = np.random.default_rng(53)
        leaves = np.arange(1, 70001, dtype=np.int32)
        src = np.concatenate([np.zeros(70000, np.int32), rng.integers(1, 70001, 30000).astype(np.int32)])
        dst = np.concatenate([leaves, rng.integers(1, 70001, 30000).astype(np.int32)])
        keep = src != dst
        g0 = inputs.from_edges(70001, src[keep], dst[keep], symmetrize=True)
        # double the arcs between the hub (vertex 0) and leaves 1..5, both ways
        rows = [list(g0.col_idx[g0.row_ptr[v]:g0.row_ptr[v + 1]]) for v in range(g0.n)]
        for leaf in range(1, 6):
            rows[0].append(leaf)
            rows[leaf].append(0)
        rows = [sorted(r) for r in rows]
        rp = np.zeros(g0.n + 1, dtype=np.int64)
        rp[1:] = np.cumsum([len(r) for r in rows])
        ci = np.fromiter((u for r in rows for u in r), dtype=np.int32, count=int(rp[-1]))
        g, w = inputs.Graph(n=g0.n, row_ptr=rp, col_idx=ci, name="hub_multi"), None
        assert g.max_degree >= 65536
    else:
        g, w = inputs.barabasi_albert(4000, 4, 52), None
        if name == "weighted":
            deg = g.degrees.astype(np.float64)
            rows = np.repeat(np.arange(g.n), g.degrees)
            w = 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])
    say(f"[split sweep] {name} n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g, weights=w)
    alpha = 0.9 * oracle.default_alpha(g, w)
    sizes = [(1, 1), (2, 7), (3, 60), (4, 700), (5, g.n)]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    groups = [inputs.group(g.n, size, seed) for seed, size in sizes]
    for j, S in enumerate(groups):
        off[j + 1] = off[j] + S.size
    mem = np.concatenate(groups).astype(np.int32)
    for ell in range(1, 10):
        B = oracle.comb_bound(g, alpha, ell, w)
        eps = 4.0 * B if ell == 1 else float(np.sqrt(B * oracle.comb_bound(g, alpha, ell - 1, w)))
        say(f"  ell={ell} eps={eps:.3e}")
        ref = []
        for S in groups:
            c, ell_o, _, _ = oracle.score(g, S, alpha, eps, w=w)
            assert ell_o == ell
            s, ell_g, _ = gg.score(S, alpha, eps, with_info=True)
            assert ell_g == ell and rel(s, c) <= REL, (name, ell, S.size, s, c)
            ref.append(c)
        b = gg.score_batch(off, mem, alpha, eps)
        for j, c in enumerate(ref):
            assert rel(b[j], c) <= REL, (name, ell, j, b[j], c)
    gg.close()


def omega_max(g, top):
    """max_v omega_i(v) (walks of length i ending at v) for i = 0..top, in float64
    (exact while below 2^53, which covers every comparison with 2^32 here)."""
    om = np.ones(g.n)
    out = [1.0]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for _ in range(top):
        om = np.bincount(rows, weights=om[g.col_idx], minlength=g.n)
        out.append(float(om.max()))
    return out


def _prepare_graph(name):
    if name == "sparse_er":
        return inputs.erdos_renyi(3000, 4500, 57), None
    if name == "ba20k":
        return GRAPHS["ba20k"](), None
    if name == "multigraph":
        return ba_multigraph(), None
    if name == "directed":
        r = inputs.uniform_ints(2 * 9000, 2000, 61)
        return inputs.from_edges(2000, r[0::2], r[1::2], symmetrize=False, name="dir2k"), None
    if name == "edgeless":
        return inputs.from_edges(50, [], [], symmetrize=True), None
    g = inputs.barabasi_albert(5000, 4, 33)  # weighted
    deg = g.degrees.astype(np.float64)
    rows = np.repeat(np.arange(g.n), g.degrees)
    return g, 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])


@pytest.mark.parametrize("name", ["sparse_er", "ba20k", "multigraph", "directed", "edgeless",
                                  "weighted"])
def test_prepare_from_counts(ged, name):
    """Precomputation levels written from the graph's integer walk counts:
    level 1 from the degrees on a fresh handle, and after scores have built
    the omega tables (undirected graphs) every level they hold, so the
    precomputation runs fewer steps.  ell*, B and the walk total equal those of
    the first precomputation (1e-12) and the oracle's, and scores after it
    match the oracle, over eps values whose ell* ends inside and past the
    levels held.  Weighted graphs take every level by steps."""
    g, w = _prepare_graph(name)
    gg = ged.GedGraph.from_graph(g, weights=w)
    alpha = (0.5 / oracle.max_weighted_out_degree(g, w) if w is not None
             else oracle.default_alpha(g))
    eps_list = [1e-1, 1e-3, 1e-4, 1e-7, 1e-10, 1e-13]
    first = {}
    for eps in eps_list:
        gg.invalidate()
        gg.profile_enable(True)
        first[eps] = gg.prepare(alpha, eps)
        steps = gg.profile_read()["launches"]
        gg.profile_enable(False)
        ell = first[eps][0]
        say(f"[prepare counts] {name} eps={eps:g} ell={ell} fresh steps={steps}")
        assert steps == (ell if w is not None else max(ell - 1, 0)), (eps, ell, steps)
    groups = [inputs.group(g.n, 5, 11), inputs.group(g.n, 40, 12)]
    for S in groups:  # builds the omega tables on undirected graphs
        gg.score(S, alpha, eps_list[-1])
    for eps in eps_list:
        gg.invalidate()
        gg.profile_enable(True)
        again = gg.prepare(alpha, eps)
        steps = gg.profile_read()["launches"]
        gg.profile_enable(False)
        ell = again[0]
        say(f"[prepare counts] {name} eps={eps:g} ell={ell} steps after scores={steps}")
        assert ell == first[eps][0]
        assert rel(again[1], first[eps][1]) <= 1e-12 and rel(again[2], first[eps][2]) <= 1e-12
        if w is not None:
            assert steps == ell
            B_o = oracle.comb_bound(g, alpha, ell, w=w)
        else:
            assert steps <= max(ell - 1, 0)
            if not g.directed and g.nnz > 0:
                assert steps <= max(ell - 2, 0)
            B_o = oracle.comb_bound(g, alpha, ell)
        assert rel(again[1], B_o) <= REL, (again[1], B_o)
        if w is None:
            for S in groups:
                check_score(gg, g, S, alpha, eps, tag=(name, eps))
        else:
            for S in groups:
                s, ell_s, _ = gg.score(S, alpha, eps, with_info=True)
                c, ell_o, _, _ = oracle.score(g, S, alpha, eps, w=w)
                assert ell_s == ell_o and rel(s, c) <= REL, (eps, s, c)
    if name == "sparse_er":  # the 32-bit omega levels are held and used
        gg.invalidate()
        gg.profile_enable(True)
        ell = gg.prepare(alpha, eps_list[-1])[0]
        steps = gg.profile_read()["launches"]
        gg.profile_enable(False)
        assert steps < ell - 2, (ell, steps)
    gg.close()


def push3_arcs(g, S):
    """Arcs the level-3 push of one group would touch: the degrees of every
    vertex holding a level-2 count (members with arcs, and non-members
    adjacent to S or to a neighbour of S)."""
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(g.n), deg)
    m = np.zeros(g.n, bool)
    m[np.asarray(S)] = True
    n1 = np.zeros(g.n, bool)
    n1[g.col_idx[m[rows]]] = True  # neighbours of S
    n2 = np.zeros(g.n, bool)
    n2[g.col_idx[(m | n1)[rows]]] = True  # neighbours of S and of N(S)
    src = (m & (deg > 0)) | (n2 & ~m)
    return int(deg[src].sum())


def push3_vertex_bounds(g):
    """deg + omega_2 + omega_3 per vertex."""
    deg = np.diff(g.row_ptr).astype(np.float64)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    om2 = np.bincount(rows, weights=deg[g.col_idx], minlength=g.n)
    om3 = np.bincount(rows, weights=om2[g.col_idx], minlength=g.n)
    return deg + om2 + om3


def push3_bound(g, S, vb=None):
    """The library's host bound on push3_arcs: the vertex bounds summed over
    S; the push is taken when it is at most nnz/32."""
    vb = push3_vertex_bounds(g) if vb is None else vb
    return float(vb[np.unique(np.asarray(S))].sum())


@pytest.mark.parametrize("name", ["sparse_er", "ba20k", "multigraph"])
def test_score_pushed_level3(ged, name):
    """Single scores whose first stored level (walk length 3, 32-bit counts)
    is pushed from the vertices holding level-2 counts when a host bound on
    the arcs that push touches (deg + omega_2 + omega_3 summed over S, which
    is at least the true count) is at most nnz/32, and gathered otherwise:
    groups on both sides of that threshold, in an order that moves between
    the two and through walk lengths with no stored level or FP64 stored
    levels, so the zeroed-level invariant is exercised.  Every score matches
    the oracle and the batched score of the same groups."""
    g, _ = _prepare_graph(name)
    gg = ged.GedGraph.from_graph(g)
    alpha = oracle.default_alpha(g)
    lim = g.nnz // 32
    sizes = [1, 5, 40, 400, 5, 2000, 3]
    groups = [inputs.group(g.n, min(k, g.n), 900 + i) for i, k in enumerate(sizes)]
    vb = push3_vertex_bounds(g)
    low = np.argsort(vb, kind="stable")
    groups[1:1] = [low[:1].astype(np.int32), low[:3].astype(np.int32)]  # smallest bounds
    bound = [push3_bound(g, S, vb) for S in groups]
    pushed = [b <= lim for b in bound]
    for S, b in zip(groups, bound):
        assert push3_arcs(g, S) <= b
    say(f"[pushed level 3] {name} nnz={g.nnz} limit={lim} bounds={bound}")
    assert any(pushed) and not all(pushed), "both regimes must be covered"
    eps_seq = [1e-7, 100.0, 1e-7, 1e-13, 1e-2] if name == "sparse_er" else [1e-7, 1.0, 1e-2]
    for eps in eps_seq:
        ell = gg.prepare(alpha, eps)[0]
        for S in groups:
            s = check_score(gg, g, S, alpha, eps, tag=(name, eps, len(S)))
        off = np.concatenate([[0], np.cumsum([len(S) for S in groups])]).astype(np.int64)
        mem = np.concatenate(groups).astype(np.int32)
        batch = gg.score_batch(off, mem, alpha, eps)
        for j, S in enumerate(groups):
            assert rel(batch[j], gg.score(S, alpha, eps)) <= 1e-12, (eps, j)
        say(f"[pushed level 3] {name} eps={eps:g} ell={ell} ok")
    if name == "ba20k":
        # ell* = 7: levels 1-2 pushed, level 3 pushed or dense, level 4 combining
        assert gg.prepare(alpha, 1e-2)[0] == 7
        for S, p in zip(groups, pushed):
            gg.profile_enable(True)
            s = gg.score(S, alpha, 1e-2)
            launches = gg.profile_read()["launches"]
            gg.profile_enable(False)
            assert launches == (1 if p else 2), (len(S), p, launches)
            assert s == gg.score(S, alpha, 1e-2)  # profiled and captured runs agree
    gg.close()


def omega_rows(g, top):
    """omega_i(v) for i = 0..top as float64 rows (exact while below 2^53)."""
    om = [np.ones(g.n)]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for _ in range(top):
        om.append(np.bincount(rows, weights=om[-1][g.col_idx], minlength=g.n))
    return om


def group_levels_fit(om, S, a):
    """A single score's own bound on its stored level-i hit counts, i = 3 ..
    a-1: a walk of length i meeting S splits at its last member s into a walk
    ending at s and one leaving it, so count_i(v) <= sum_s sum_{j<i}
    omega_j(s) omega_{i-j}(s).  True when every such bound is below 2^32 (with
    the library's 0.1 % margin)."""
    if a - 1 < 3:
        return False
    S = np.unique(np.asarray(S))
    for i in range(3, a):
        b = sum(float(np.dot(om[j][S], om[i - j][S])) for j in range(i))
        if not b < 0.999 * 2.0 ** 32:
            return False
    return True


@pytest.mark.parametrize("name", ["sparse_er", "star"])
def test_split_count_layout(ged, name):
    """Dense split levels stored as unscaled 32-bit counts when every stored
    level's omega maximum is below 2^32, or, for a single score, when the
    group's own bound on its hit counts is (member-wise sums of omega_j omega_
    {i-j}); FP64 otherwise.  "sparse_er" (average degree 3) keeps omega small
    for many levels, so ell* = 7..17 stores 1..6 levels as 32-bit counts (the
    combining step's four-level loop and its remainder), while ell* = 29 needs
    omega_14 > 2^32 and only groups of small bound stay 32-bit; "star" (70,000
    leaves, no duplicate arcs) has omega_3 = 70,000^2 > 2^32, so a group
    holding the centre keeps FP64 levels while groups of leaves fit on their
    own bound.  The profiled dominant step kernel shows which layout ran;
    scores single and batched against the oracle (batches use the graph-wide
    layout)."""
    if name == "sparse_er":
        g = inputs.erdos_renyi(3000, 4500, 57)
        ells = list(range(7, 18, 2)) + [29]  # 29: omega_14 > 2^32
    else:
        g = inputs.from_edges(70001, np.zeros(70000, np.int32),
                              np.arange(1, 70001, dtype=np.int32), name="star70k")
        ells = [7, 8]
    say(f"[count layout] {name} n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g)
    alpha = 0.9 * oracle.default_alpha(g, None)
    om = omega_max(g, 20)
    orow = omega_rows(g, 15)
    sizes = [(1, 1), (2, 9), (3, 120)]
    groups = [inputs.group(g.n, size, seed) for seed, size in sizes]
    if name == "star":
        groups.append(np.array([0, 5], np.int32))  # the centre: omega_3 = 4.9e9
    off = np.zeros(len(groups) + 1, dtype=np.int64)
    for j, S in enumerate(groups):
        off[j + 1] = off[j] + S.size
    mem = np.concatenate(groups).astype(np.int32)
    seen = {False: 0, True: 0}
    for ell in ells:
        B = oracle.comb_bound(g, alpha, ell, None)
        eps = float(np.sqrt(B * oracle.comb_bound(g, alpha, ell - 1, None)))
        a = (ell + 1) // 2
        u32 = all(om[i] < 2.0 ** 32 for i in range(3, a))
        say(f"  ell={ell} stored levels={a - 3} 32-bit={u32}")
        ref = []
        gg.prepare(alpha, eps)  # t-levels outside the profiled calls
        for j, S in enumerate(groups):
            c, ell_o, _, _ = oracle.score(g, S, alpha, eps)
            assert ell_o == ell
            gg.profile_enable(True)
            s = gg.score(S, alpha, eps)
            kind = gg.profile_read()["dominant_kind"]
            gg.profile_enable(False)
            out = kind % ged.KIND_BASE
            want = u32 or group_levels_fit(orow, S, a)
            if a - 1 >= 3:
                seen[want] += 1
            assert (out in (9, 10)) == want, (name, ell, S.size, kind)
            assert rel(s, c) <= REL, (name, ell, S.size, s, c)
            ref.append(c)
        b = gg.score_batch(off, mem, alpha, eps)
        for j, c in enumerate(ref):
            assert rel(b[j], c) <= REL, (name, ell, j, b[j], c)
    if name == "sparse_er":
        assert om[(17 + 1) // 2 - 1] < 2.0 ** 32  # the last ell still stores 32-bit levels
    else:
        assert om[3] > 2.0 ** 32
        # leaves fit on their own bound, the centre's group does not
        assert group_levels_fit(orow, groups[0], 4) and not group_levels_fit(orow, groups[-1], 4)
    assert seen[True] > 0 and seen[False] > 0, seen
    gg.close()


@pytest.mark.parametrize("name", ["ba", "star"])
def test_batch_every_tile_width(ged, name):
    """Batched split scoring forced to each tile width 1..64: the step kernels'
    column-pair gathers (32-bit inputs at C >= 2, blocks of twice the arcs),
    32-bit stored levels ("ba": omega fits) and FP64 stored levels ("star":
    omega_3 > 2^32), partials reduced over the matching partition.  Every column
    equals the solo score; a sample against the oracle."""
    if name == "ba":
        g = inputs.barabasi_albert(20000, 5, 59)
    else:
        g = inputs.from_edges(70001, np.zeros(70000, np.int32),
                              np.arange(1, 70001, dtype=np.int32), name="star70k")
    gg = ged.GedGraph.from_graph(g)
    alpha = 0.9 * oracle.default_alpha(g, None)
    B = oracle.comb_bound(g, alpha, 7, None)
    eps = float(np.sqrt(B * oracle.comb_bound(g, alpha, 6, None)))  # ell* = 7: one stored level
    off, mem = inputs.groups(g.n, 70, 1, 60, 160)
    solo = [gg.score(mem[off[j]:off[j + 1]], alpha, eps) for j in range(70)]
    for j in (0, 33, 69):
        c, ell_o, _, _ = oracle.score(g, mem[off[j]:off[j + 1]], alpha, eps)
        assert ell_o == 7 and rel(solo[j], c) <= REL, (name, j, solo[j], c)
    for tile in (1, 2, 4, 8, 16, 32, 64):
        say(f"[tile widths] {name} tile={tile}")
        gg.set_batch_tile(tile)
        b = gg.score_batch(off, mem, alpha, eps)
        worst = max(rel(b[j], solo[j]) for j in range(70))
        assert worst <= 1e-12, (name, tile, worst)
    gg.close()


@pytest.mark.parametrize("name", ["ba", "star", "directed"])
def test_batch_row_cuts(ged, name):
    """Batched scoring at each row-split threshold (cut_div 1, 2, 4: rows above
    2048/C/cut_div arcs become segments) and several tile widths, on the split
    path ("ba", "star": one row of 70,000 arcs) and the level-by-level column
    path ("directed"): every column equals its solo score to 1e-12, a sample
    the oracle to 1e-9; with both knobs left to the autotuner it records a
    width and a threshold, and a repeated batch is bit for bit the same."""
    if name == "ba":
        g = inputs.barabasi_albert(20000, 5, 59)
    elif name == "star":
        g = inputs.from_edges(70001, np.zeros(70000, np.int32),
                              np.arange(1, 70001, dtype=np.int32), name="star70k")
    else:
        g = directed_graph()
    gg = ged.GedGraph.from_graph(g)
    alpha = oracle.default_alpha(g, None)
    off, mem = inputs.groups(g.n, 40, 1, 60, 161)
    solo = [gg.score(mem[off[j]:off[j + 1]], alpha, EPS) for j in range(40)]
    for j in (0, 39):
        c, _, _, _ = oracle.score(g, mem[off[j]:off[j + 1]], alpha, EPS)
        assert rel(solo[j], c) <= REL, (name, j, solo[j], c)
    for tile in (4, 16, 64):
        for cut in (1, 2, 4):
            say(f"[row cuts] {name} tile={tile} cut_div={cut}")
            gg.set_batch_tile(tile)
            gg.set_batch_row_cut(cut)
            assert gg.batch_row_cut() == cut
            b = gg.score_batch(off, mem, alpha, EPS)
            worst = max(rel(b[j], solo[j]) for j in range(40))
            assert worst <= 1e-12, (name, tile, cut, worst)
    gg.set_batch_tile(0)  # both knobs back to the autotuner
    assert gg.batch_row_cut() == 0
    b = gg.score_batch(off, mem, alpha, EPS)
    say(f"  autotuned: tile {gg.batch_tile()} cut_div {gg.batch_row_cut()}")
    assert gg.batch_tile() in (4, 8, 16, 32, 64) and gg.batch_row_cut() in (1, 2, 4)
    assert max(rel(b[j], solo[j]) for j in range(40)) <= 1e-12
    np.testing.assert_array_equal(gg.score_batch(off, mem, alpha, EPS), b)
    gg.close()


@pytest.mark.parametrize("ell", [5, 8])
def test_batch_count16(ged, ell):
    """Level-2 counts of batch tiles in the 16-bit layout (rows below the hub
    cut stay 32-bit).  On BA n=200,000, m=8 (ten vertices with omega_2 above
    2^16 - 2, all among the first eleven by degree) the batch at the
    library's cut and at a cut of n/4 (a quarter of the rows in the 32-bit
    table) is bit for bit the same, at tile widths 4, 8 and 32 (one, two and
    eight 4-column units per arc), with the row partition's long-row
    segments and, on a second handle, with source buckets forced on; sampled
    columns equal the oracle to 1e-9.  ell* = 8 has one stored level (level 3
    gathers the 16-bit level 2 and also stores a 16-bit copy of itself, which
    the combining step gathers, marked values from the 32-bit level); ell* =
    5 has none (the combining step gathers the 16-bit level 2).  With the
    layout off the combining step sums its rows in blocks of a quarter of the
    arcs, so the scores agree to the column sums' rounding."""
    g = inputs.barabasi_albert(200000, 8, 5)
    alpha = oracle.default_alpha(g, None)
    B = oracle.comb_bound(g, alpha, ell, None)
    eps = float(np.sqrt(B * oracle.comb_bound(g, alpha, ell - 1, None)))
    G = 80
    off, mem = inputs.groups(g.n, G, 1, 200, 177)
    say(f"[count16] n={g.n} nnz={g.nnz} ell*={ell} eps={eps:.3e}")
    ref = {}
    for j in (0, 37, G - 1):
        c, ell_o, _, _ = oracle.score(g, mem[off[j]:off[j + 1]], alpha, eps)
        assert ell_o == ell
        ref[j] = c
    for buckets in (0, 1 << 16):
        gg = ged.GedGraph.from_graph(g)
        if buckets:
            gg.set_source_buckets(buckets)
        for tile in (4, 8, 32):
            gg.set_batch_tile(tile)
            gg.set_batch_row_cut(1)
            out = []
            for hub in (-1, 0, g.n // 4):
                gg.set_count16(hub)
                b = gg.score_batch(off, mem, alpha, eps)
                used = gg.count16_hub()
                say(f"  buckets={buckets} tile={tile} setting={hub}: cut {used}")
                if hub == -1:
                    assert used == -1
                elif hub == 0:
                    assert 0 < used <= 64, used
                else:
                    assert used == hub
                out.append(b)
            np.testing.assert_array_equal(out[2], out[1])
            assert max(rel(x, y) for x, y in zip(out[1], out[0])) <= 1e-14
            for j, c in ref.items():
                assert rel(out[1][j], c) <= REL, (tile, buckets, j, out[1][j], c)
        with pytest.raises(ged.GedError):
            gg.set_count16(5)  # below the least cut
        gg.close()


@pytest.mark.parametrize("ell", [8, 9])
def test_batch_count16_stored_levels(ged, ell):
    """The 16-bit level-2 layout with one and with two stored levels.  On
    G(n, M) with n = 200,000 and average degree 10 every omega_2 fits 16
    bits (the library's cut is 0: all rows packed) and the deeper levels stay
    32-bit counts.  ell* = 8: level 3 is the only stored level, so its 32-bit
    counts are kept only where its 16-bit copy marks them and the combining
    step reads the copy; ell* = 9: levels 3 and 4 are stored, both in full,
    and the combining step gathers the copy of level 4.  Bit-identical among
    the cuts (0 and n/4), equal to the 32-bit layout to the column sums'
    rounding, sampled columns equal to the oracle to 1e-9, at tile widths 8
    and 64."""
    g = inputs.erdos_renyi(200000, 1000000, 9)
    alpha = oracle.default_alpha(g, None)
    B = oracle.comb_bound(g, alpha, ell, None)
    eps = float(np.sqrt(B * oracle.comb_bound(g, alpha, ell - 1, None)))
    G = 72
    off, mem = inputs.groups(g.n, G, 1, 200, 179)
    say(f"[count16 levels] n={g.n} nnz={g.nnz} ell*={ell} eps={eps:.3e}")
    ref = {}
    for j in (0, 35, G - 1):
        c, ell_o, _, _ = oracle.score(g, mem[off[j]:off[j + 1]], alpha, eps)
        assert ell_o == ell
        ref[j] = c
    gg = ged.GedGraph.from_graph(g)
    for tile in (8, 64):
        gg.set_batch_tile(tile)
        out = []
        for hub in (-1, 0, g.n // 4):
            gg.set_count16(hub)
            out.append(gg.score_batch(off, mem, alpha, eps))
            used = gg.count16_hub()
            say(f"  tile={tile} setting={hub}: cut {used}")
            assert used == (hub if hub != 0 else 0), (tile, hub, used)
        np.testing.assert_array_equal(out[2], out[1])
        assert max(rel(x, y) for x, y in zip(out[1], out[0])) <= 1e-14
        for j, c in ref.items():
            assert rel(out[1][j], c) <= REL, (tile, j, out[1][j], c)
    gg.close()


def test_batch_count16_not_applicable(ged):
    """Where the 16-bit level-2 layout does not apply -- a directed graph
    (level-by-level chains), a weighted graph (no integer levels) and an
    undirected graph at ell* = 4 (a = 2: level 2 is combined directly, no dense
    level gathers it) -- the automatic and a forced cut both leave it off: the
    batch reports no cut and equals the batch with the layout off bit for bit,
    and sampled columns equal the oracle to 1e-9."""
    gd = directed_graph()
    gw = inputs.barabasi_albert(20000, 4, 33)
    deg = gw.degrees.astype(np.float64)
    rows = np.repeat(np.arange(gw.n), gw.degrees)
    w = 1.0 / np.sqrt(deg[rows] * deg[gw.col_idx])
    gb = inputs.barabasi_albert(20000, 8, 34)
    a_b = oracle.default_alpha(gb, None)
    eps_b = float(np.sqrt(oracle.comb_bound(gb, a_b, 4, None) * oracle.comb_bound(gb, a_b, 3, None)))
    cases = [("directed", gd, None, oracle.default_alpha(gd, None), EPS),
             ("weighted", gw, w, 0.5 / oracle.max_weighted_out_degree(gw, w), EPS),
             ("ell4", gb, None, a_b, eps_b)]
    for name, g, wt, alpha, eps in cases:
        off, mem = inputs.groups(g.n, 24, 1, 50, 178)
        gg = ged.GedGraph.from_graph(g, weights=wt)
        gg.set_batch_tile(8)
        out = []
        for hub in (-1, 0, g.n - 1):
            gg.set_count16(hub)
            out.append(gg.score_batch(off, mem, alpha, eps))
            assert gg.count16_hub() == -1, (name, hub)
        say(f"[count16 n/a] {name}: n={g.n} nnz={g.nnz}")
        np.testing.assert_array_equal(out[1], out[0])
        np.testing.assert_array_equal(out[2], out[0])
        for j in (0, 11, 23):
            c, ell_o, _, _ = oracle.score(g, mem[off[j]:off[j + 1]], alpha, eps, w=wt)
            if name == "ell4":
                assert ell_o == 4
            assert rel(out[0][j], c) <= REL, (name, j, out[0][j], c)
        gg.close()


def test_batch_count16_wide_rows(ged):
    """The 16-bit level-2 layout with members among the rows kept in 32 bits.
    The graph's 600 highest-degree vertices (a K_{300,300} core, omega_2 =
    90,000) are exactly those above 2^16 - 2, more than n/8, so the library
    leaves the layout off by itself; forced cuts of 600 (the least) and n - 1
    put them, and then almost every row, in the 32-bit table.  Groups hold
    core vertices, an empty group and single members; tiles of 8 and 32
    columns; ell* = 5 and 8.  Scores equal the oracle to 1e-9, the two cuts
    agree bit for bit, and with the layout off the batch agrees to the column
    sums' rounding; a cut below 600 is refused."""
    from wide_prefix import wide_prefix_graph
    g = wide_prefix_graph()
    alpha = oracle.default_alpha(g, None)
    core = np.argsort(-g.degrees, kind="stable")[:600].astype(np.int32)
    assert sorted(core.tolist()) == list(range(600))
    groups = [core[:3], np.zeros(0, np.int32), core[599:600], np.arange(650, 651, dtype=np.int32),
              np.concatenate([core[100:140], np.arange(600, 700, dtype=np.int32)]),
              inputs.group(g.n, 50, 7), inputs.group(g.n, 200, 8), core[:300]]
    off = np.zeros(len(groups) + 1, np.int64)
    for j, S in enumerate(groups):
        off[j + 1] = off[j] + S.size
    mem = np.concatenate(groups).astype(np.int32)
    say(f"[count16 wide rows] n={g.n} nnz={g.nnz} groups={len(groups)}")
    gg = ged.GedGraph.from_graph(g)
    with pytest.raises(ged.GedError):
        gg.set_count16(599)
    for ell in (5, 8):
        B = oracle.comb_bound(g, alpha, ell, None)
        eps = float(np.sqrt(B * oracle.comb_bound(g, alpha, ell - 1, None)))
        ref = []
        for S in groups:
            c, ell_o, _, _ = oracle.score(g, S, alpha, eps)
            assert ell_o == ell
            ref.append(c)
        for tile in (8, 32):
            gg.set_batch_tile(tile)
            gg.set_batch_row_cut(1)
            out = {}
            for hub in (-1, 0, 600, g.n - 1):
                gg.set_count16(hub)
                out[hub] = gg.score_batch(off, mem, alpha, eps)
                used = gg.count16_hub()
                say(f"  ell*={ell} tile={tile} setting={hub}: cut {used}")
                assert used == (-1 if hub in (-1, 0) else hub)
            np.testing.assert_array_equal(out[600], out[g.n - 1])
            np.testing.assert_array_equal(out[0], out[-1])
            assert max(rel(x, y) for x, y in zip(out[600], out[-1]) if y) <= 1e-14
            for j, c in enumerate(ref):
                if c == 0.0:
                    assert out[600][j] == 0.0
                else:
                    assert rel(out[600][j], c) <= REL, (ell, tile, j, out[600][j], c)
    gg.close()


@pytest.mark.parametrize("name", ["ba", "directed", "weighted"])
def test_spectral_bound(ged, name):
    """sigma_max estimate, ell* and scores / greedy under the spectral tail bound
    with alpha beyond 1/deg_max (where the combinatorial bound does not apply)."""
    rev = w = None
    if name == "ba":
        g = inputs.barabasi_albert(20000, 4, 71)
    elif name == "directed":
        r = inputs.uniform_ints(2 * 40000, 5000, 72)
        g = inputs.from_edges(5000, r[0::2], r[1::2], symmetrize=False, name="dir5k")
        g.directed = True
        rev = inputs.reverse(g)
    else:
        g = inputs.barabasi_albert(8000, 3, 73)
        deg = g.degrees.astype(np.float64)
        rows = np.repeat(np.arange(g.n), g.degrees)
        w = 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])
    say(f"[spectral] {name} n={g.n} nnz={g.nnz}")
    gg = ged.GedGraph.from_graph(g, weights=w)
    s_gpu = gg.sigma_max()
    s_ora = oracle.sigma_max(g, rev=rev, w=w, w_rev=None if rev is not None else w)
    assert rel(s_gpu, s_ora) <= 1e-9, (s_gpu, s_ora)
    alpha = 0.5 / s_gpu
    D = oracle.max_weighted_out_degree(g, w) if w is not None else oracle.max_out_degree(g)
    assert alpha * D >= 1.0  # outside the combinatorial bound's range
    with pytest.raises(ged.GedError) as e:
        gg.score([0], alpha, EPS)
    assert e.value.code == -3
    gg.set_tail_bound("spectral")
    with pytest.raises(ged.GedError):
        gg.score([0], 1.0 / s_gpu, EPS)
    groups = [inputs.group(g.n, size, seed) for seed, size in [(1, 1), (2, 9), (3, 120)]]
    for S in groups:
        s, ell, B = gg.score(S, alpha, EPS, with_info=True)
        c, ell_o, B_o, _ = oracle.score(g, S, alpha, EPS, w=w, sigma=s_gpu)
        assert ell == ell_o and rel(s, c) <= REL and rel(B, B_o) <= 1e-9, (name, S.size, s, c)
    if rev is None:
        off = np.array([0, groups[0].size, groups[0].size + groups[1].size], dtype=np.int64)
        b = gg.score_batch(off, np.concatenate(groups[:2]).astype(np.int32), alpha, EPS)
        for j in range(2):
            assert rel(b[j], oracle.score(g, groups[j], alpha, EPS, w=w, sigma=s_gpu)[0]) <= REL
    rg = gg.greedy(4, alpha, EPS)
    ro = oracle.greedy(g, 4, alpha, EPS, rev=rev, w=w, sigma=s_gpu,
                       w_rev=None if rev is not None else w)
    compare_greedy(rg, ro, f"spectral {name}")
    gg.set_tail_bound("combinatorial")
    with pytest.raises(ged.GedError):
        gg.score([0], alpha, EPS)
    gg.close()


def test_keep_order_parity(ged):
    """A handle that keeps the caller's vertex order (no degree relabelling):
    single scores (pushed and gathered third levels), a batch and the greedy
    against the oracle, and against a relabelled handle."""
    g = GRAPHS["ba20k"]()
    alpha = g.default_alpha()
    kept = ged.GedGraph.from_graph(g, keep_order=True)
    relab = ged.GedGraph.from_graph(g)
    vb = push3_vertex_bounds(g)
    low = np.argsort(vb, kind="stable")
    groups = [low[:1].astype(np.int32), low[:4].astype(np.int32), inputs.group(g.n, 5, 31),
              inputs.group(g.n, 60, 32), inputs.group(g.n, 700, 33)]
    for eps in (1e-2, 1e-7):
        for S in groups:
            s = check_score(kept, g, S, alpha, eps, tag=("kept", eps, len(S)))
            assert rel(s, relab.score(S, alpha, eps)) <= 1e-12
        off = np.concatenate([[0], np.cumsum([len(S) for S in groups])]).astype(np.int64)
        b = kept.score_batch(off, np.concatenate(groups).astype(np.int32), alpha, eps)
        for j, S in enumerate(groups):
            assert rel(b[j], kept.score(S, alpha, eps)) <= 1e-12
    compare_greedy(kept.greedy(8, alpha, EPS), oracle.greedy(g, 8, alpha, EPS), "kept order")
    kept.close()
    relab.close()
