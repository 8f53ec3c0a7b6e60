"""The split identity behind split scoring, checked without the GPU.

* exactly, by enumerating every walk of tiny undirected graphs;
* that it fails on a directed graph (why directed graphs keep the
  level-by-level chain);
* the push formulation of the level-1/2 counts against enumeration;
* the whole split scheme (tests/split_model.py) against the oracle for every
  plan shape (a = 1, 2, 3+, odd and even ell, weighted);
* the same split for marginal gains (walks that avoid S and contain x);
* the bound count_i <= omega_i that lets the dense levels be stored as 32-bit
  integers, and split scoring with integer levels against the oracle;
* split gains with integer gain levels (the candidate's miss counts recovered
  by rounding the FP64 miss chain) against the oracle and exact counts.
"""
import numpy as np
import pytest

import oracle
from exact import WalkTable
from paper_1910_13874_amd import inputs
from wide_prefix import wide_prefix_graph
from split_model import (count_levels, push3_bound, push3_counts, push_counts, split_gain,
                         split_gain_counts, split_score, split_score_counts)


def tiny_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    keep = src != dst
    return inputs.from_edges(n, src[keep], dst[keep], symmetrize=True)


def hit_end(tab, i, S, v):
    """# i-walks ending at v that contain a vertex of S."""
    m = tab._mask(S)
    return sum(c for (_, e, mk), c in tab.tab[i].items() if e == v and mk & m)


def all_end(tab, i, v):
    return sum(c for (_, e, _), c in tab.tab[i].items() if e == v)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_split_identity_exact(seed):
    g = tiny_graph(7, 11, seed)
    tab = WalkTable(g.n, g.row_ptr, g.col_idx, 6)
    rng = np.random.default_rng(seed)
    for S in ([0], [1, 4], list(rng.choice(g.n, 3, replace=False))):
        S = [int(s) for s in S]
        for a in range(0, 4):
            for c in range(0, 7 - a):
                H_a = [hit_end(tab, a, S, v) for v in range(g.n)]
                H_c = [hit_end(tab, c, S, v) for v in range(g.n)]
                T_a = [all_end(tab, a, v) for v in range(g.n)]
                T_c = [all_end(tab, c, v) for v in range(g.n)]
                rhs = sum(H_a[v] * T_c[v] for v in range(g.n))
                rhs += sum((T_a[v] - H_a[v]) * H_c[v] for v in range(g.n) if v not in S)
                assert tab.phi(a + c, S) == rhs, (seed, S, a, c)


def test_split_identity_fails_directed():
    # arcs 0 -> 1, 2 -> 1, 1 -> 3 and S = {3}: both 2-walks (0-1-3, 2-1-3)
    # meet S, but the split at a = c = 1 sees one walk of length 1 ending at
    # 1 that meets S (none) and one ending at 3 (1-3), and the walks of length
    # 1 ending at v do not stand for those leaving v.
    g = inputs.from_edges(4, np.array([0, 2, 1], np.int32), np.array([1, 1, 3], np.int32),
                          symmetrize=False)
    tab = WalkTable(g.n, g.row_ptr, g.col_idx, 2)
    S = [3]
    H1 = [hit_end(tab, 1, S, v) for v in range(g.n)]
    T1 = [all_end(tab, 1, v) for v in range(g.n)]
    rhs = sum(H1[v] * T1[v] for v in range(g.n)) + sum(
        (T1[v] - H1[v]) * H1[v] for v in range(g.n) if v not in S)
    assert tab.phi(2, S) == 2 and rhs == 1


@pytest.mark.parametrize("seed", [4, 5])
def test_push_counts_match_enumeration(seed):
    g = tiny_graph(8, 14, seed)
    tab = WalkTable(g.n, g.row_ptr, g.col_idx, 2)
    for S in ([0], [2, 5], [1, 3, 6, 7]):
        cnt1, cnt2 = push_counts(g.row_ptr, g.col_idx, np.array(S), 2)
        for v in range(g.n):
            assert cnt1[v] == hit_end(tab, 1, S, v), (S, v)
            assert cnt2[v] == hit_end(tab, 2, S, v), (S, v)


def eps_for(g, alpha, ell, w=None):
    """An eps whose ell* is exactly `ell` (geometric mean of consecutive bounds)."""
    B = oracle.comb_bound(g, alpha, ell, w)
    if ell == 1:
        return 4.0 * B
    return float(np.sqrt(B * oracle.comb_bound(g, alpha, ell - 1, w)))


@pytest.mark.parametrize("name", ["er", "ba", "weighted"])
def test_split_model_matches_oracle(name):
    if name == "er":
        g, w = inputs.erdos_renyi(300, 900, 41), None
    else:
        g = inputs.barabasi_albert(300, 3, 42)
        w = None
        if name == "weighted":
            deg = g.degrees.astype(np.float64)
            rows = np.repeat(np.arange(g.n), g.degrees)
            w = 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])
    alpha = 0.9 * oracle.default_alpha(g, w)
    for ell in range(1, 10):
        eps = eps_for(g, alpha, ell, w)
        for seed, size in [(1, 1), (2, 7), (3, 60), (4, g.n)]:
            S = inputs.group(g.n, size, seed)
            c, ell_o, _, _ = oracle.score(g, S, alpha, eps, w=w)
            assert ell_o == ell
            m = split_score(g.row_ptr, g.col_idx, S, alpha, ell, w)
            assert abs(m - c) <= 1e-12 * abs(c), (name, ell, size, m, c)


def miss_end_x(tab, i, S, x, v, contains):
    """# i-walks ending at v that avoid S and do (contains=True) or do not contain x."""
    m = tab._mask(S)
    bx = 1 << int(x)
    return sum(c for (_, e, mk), c in tab.tab[i].items()
               if e == v and not (mk & m) and bool(mk & bx) == contains)


@pytest.mark.parametrize("seed", [6, 7])
def test_gain_split_identity_exact(seed):
    g = tiny_graph(7, 12, seed)
    tab = WalkTable(g.n, g.row_ptr, g.col_idx, 6)
    for S, x in (([0], 3), ([1, 4], 2), ([], 5)):
        for a in range(0, 4):
            for c in range(0, 7 - a):
                D_a = [miss_end_x(tab, a, S, x, v, True) for v in range(g.n)]
                D_c = [miss_end_x(tab, c, S, x, v, True) for v in range(g.n)]
                N_a = [miss_end_x(tab, a, S, x, v, False) for v in range(g.n)]
                M_c = [tab.miss_end(c, S, v) for v in range(g.n)]
                rhs = sum(D_a[v] * M_c[v] + N_a[v] * D_c[v] for v in range(g.n))
                assert tab.gain_count(a + c, S, x) == rhs, (seed, S, x, a, c)


@pytest.mark.parametrize("weighted", [False, True])
def test_split_gain_model_matches_oracle(weighted):
    g = inputs.barabasi_albert(300, 3, 43)
    w = None
    if weighted:
        deg = g.degrees.astype(np.float64)
        rows = np.repeat(np.arange(g.n), g.degrees)
        w = 1.0 / np.sqrt(deg[rows] * deg[g.col_idx])
    alpha = 0.9 * oracle.default_alpha(g, w)
    for ell in (1, 2, 3, 4, 7, 8, 16):
        for S, x in (([], 0), ([0, 5], 1), (list(range(10, 40)), 7), ([2], 250)):
            o = oracle.gain(g, S, x, alpha, ell, w=w)
            m = split_gain(g.row_ptr, g.col_idx, S, x, alpha, ell, w)
            assert abs(m - o) <= 1e-12 * abs(o), (weighted, ell, len(S), x, m, o)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_count_levels_bounded_by_omega(seed):
    """count_i(v) <= omega_i(v) for every level, vertex and group: a level
    whose omega maximum is below 2^32 fits 32 bits for any group.  Also checks
    count_i against exact enumeration of the walks that meet S."""
    g = tiny_graph(9, 16, seed)
    tab = WalkTable(g.n, g.row_ptr, g.col_idx, 5)
    rng = np.random.default_rng(seed)
    for size in (1, 2, 4, g.n):
        S = np.sort(rng.choice(g.n, size, replace=False))
        cnt, om = count_levels(g.row_ptr, g.col_idx, S, 5)
        for i in range(1, 6):
            for v in range(g.n):
                assert cnt[i][v] <= om[i][v]
                assert cnt[i][v] == hit_end(tab, i, S, v), (i, v)
                assert om[i][v] == all_end(tab, i, v)


@pytest.mark.parametrize("name", ["er", "ba", "star"])
def test_split_count_model_matches_oracle(name):
    """Split scoring with unscaled integer dense levels (alpha^i applied in the
    combination) equals the oracle's score, for ell with 1..5 stored levels."""
    if name == "er":
        g = inputs.erdos_renyi(200, 600, 43)
    elif name == "ba":
        g = inputs.barabasi_albert(200, 3, 44)
    else:
        g = inputs.from_edges(60, np.zeros(59, np.int32), np.arange(1, 60, dtype=np.int32))
    alpha = 0.9 * oracle.default_alpha(g, None)
    for ell in range(7, 15):
        eps = eps_for(g, alpha, ell, None)
        for seed, size in [(1, 1), (2, 5), (3, 40)]:
            S = inputs.group(g.n, size, seed)
            c, ell_o, _, _ = oracle.score(g, S, alpha, eps)
            assert ell_o == ell
            m = split_score_counts(g.row_ptr, g.col_idx, S, alpha, ell)
            assert abs(m - c) <= 1e-12 * abs(c), (name, ell, size, m, c)


@pytest.mark.parametrize("name", ["ba", "er"])
def test_split_gain_count_model_matches_oracle(name):
    """Gain chains as unscaled integer counts equal the oracle's L_ell(S, x);
    the miss counts injected at the candidate, recovered by rounding
    m_i(x) / alpha^i, equal the exact number of walks avoiding S that end at x
    (enumerated with Python integers)."""
    g = inputs.barabasi_albert(300, 3, 45) if name == "ba" else inputs.erdos_renyi(300, 900, 46)
    alpha = 0.9 * oracle.default_alpha(g, None)
    rp, ci = g.row_ptr, g.col_idx
    for ell in (3, 4, 7, 8, 12, 16):
        for S, x in (([], 0), ([0, 5], 1), (list(range(10, 40)), 7), ([2], 250)):
            o = oracle.gain(g, S, x, alpha, ell)
            m, inj = split_gain_counts(rp, ci, S, x, alpha, ell)
            assert abs(m - o) <= 1e-12 * abs(o), (name, ell, len(S), x, m, o)
            # exact miss counts at x: walks avoiding S, by end vertex
            inS = set(S)
            mc = [0 if v in inS else 1 for v in range(g.n)]
            for i in range(1, max(inj) + 1 if inj else 1):
                mc = [0 if v in inS else sum(mc[int(u)] for u in ci[rp[v]:rp[v + 1]])
                      for v in range(g.n)]
                if i in inj:
                    assert inj[i] == mc[x], (name, ell, i, inj[i], mc[x])


def multigraph(seed):
    """tiny_graph with some edges listed twice."""
    g = tiny_graph(12, 20, seed)
    rows = [list(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    for v in range(0, g.n, 3):
        if rows[v]:
            u = rows[v][0]
            rows[v].append(u)
            rows[u].append(v)
    rows = [sorted(r) for r in rows]
    rp = np.zeros(g.n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.fromiter((u for r in rows for u in r), dtype=np.int32, count=int(rp[-1]))
    return inputs.Graph(n=g.n, row_ptr=rp, col_idx=ci, name="multi")


@pytest.mark.parametrize("kind", ["simple", "multi", "ba"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_push3_level_and_bound(kind, seed):
    """The single-group third push: its sources (members with arcs, and every
    vertex whose level-2 count the level-2 pushes touch first) give level-3
    counts equal to the gathered chain's, and the host bound sum_S (deg +
    omega_2 + omega_3) is at least the sources' degree sum, so a worklist of
    bound + bound/512 + 1 entries (one per source and per further 512 arcs)
    never overflows."""
    g = (tiny_graph(12, 20, seed) if kind == "simple" else multigraph(seed) if kind == "multi"
         else inputs.barabasi_albert(200, 3, seed))
    deg = np.diff(g.row_ptr)
    rng = np.random.default_rng(seed)
    for size in (1, 2, 3, 6, g.n // 2):
        S = np.sort(rng.choice(g.n, size, replace=False))
        cnt, _ = count_levels(g.row_ptr, g.col_idx, S, 3)
        cnt3, src = push3_counts(g.row_ptr, g.col_idx, S)
        assert list(cnt3) == cnt[3]
        assert len(src) == len(set(src))  # each source listed once
        b = push3_bound(g.row_ptr, g.col_idx, S)
        arcs = int(deg[src].sum())
        entries = int(sum((deg[u] + 511) // 512 for u in src))
        assert arcs <= b and entries <= b + b // 512 + 1, (arcs, entries, b)


def _miss_counts(g, S, top):
    """Integer miss counts: walks ending at v that avoid S, levels 0..top."""
    inS = np.zeros(g.n, dtype=bool)
    inS[np.asarray(S, dtype=np.int64)] = True
    m = [(~inS).astype(np.int64)]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for _ in range(top):
        y = np.bincount(rows, weights=m[-1][g.col_idx], minlength=g.n).astype(np.int64)
        y[inS] = 0
        m.append(y)
    return m


def _gain_counts(g, S, x, top, m):
    """The greedy's stored gain levels of candidate x as counts: level 1 is 1
    on N(x) outside S and x's miss count at x; each deeper level sums its
    in-neighbours' counts outside S and takes x's miss count at x."""
    inS = np.zeros(g.n, dtype=bool)
    inS[np.asarray(S, dtype=np.int64)] = True
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    nb = g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]
    d1 = np.zeros(g.n, dtype=np.int64)
    d1[nb[~inS[nb] & (nb != x)]] = 1
    d1[x] = m[1][x]
    d = [None, d1]
    for i in range(2, top + 1):
        y = np.bincount(rows, weights=d[-1][g.col_idx], minlength=g.n).astype(np.int64)
        y[inS] = 0
        y[x] = m[i][x]
        d.append(y)
    return d


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_miss_counts_by_subtraction(seed):
    """After x joins S the greedy takes the new miss counts (walks ending at v
    that avoid S + {x}) as the old ones minus x's stored gain-level counts:
    exact integers, so equal to the recomputed chain, which is itself checked
    against explicit walk enumeration here; x's rows become 0."""
    g = tiny_graph(10, 18, seed)
    tab = WalkTable(g.n, g.row_ptr, g.col_idx, 5)
    rng = np.random.default_rng(seed)
    for size in (1, 2, 3):
        S = list(rng.choice(g.n, size, replace=False))
        for x in range(g.n):
            if x in S:
                continue
            m = _miss_counts(g, S, 5)
            d = _gain_counts(g, S, x, 5, m)
            m2 = _miss_counts(g, S + [x], 5)
            for i in range(1, 6):
                assert list(m[i] - d[i]) == list(m2[i]), (S, x, i)
                for v in range(g.n):
                    assert m2[i][v] == tab.miss_end(i, S + [x], v)
                    assert d[i][v] == (tab.miss_end(i, S, v) - tab.miss_end(i, S + [x], v))


@pytest.mark.parametrize("forced", [False, True])
def test_count16_packed_pushes(forced):
    """The 16-bit level-2 layout of batch tiles, emulated on the CPU in the
    library's vertex order (decreasing degree, stable): rows below the cut in
    a 32-bit table, every other row's count as one 16-bit half of a 32-bit
    word shared with the adjacent column.  The kernels' pushes add value <<
    16*(c & 1) to the word (member pushes of deg(s), then the level-2 push of
    count_1(y) from each non-member y reached first, skipping member targets),
    and member rows are raised to omega_2 by adding the difference.  Pinned
    here: no half ever exceeds 2^16 - 2 (so no add carries into the other
    column and the gather's 2^16 - 1 marker is never a count), the raise adds
    a nonnegative difference, and the decoded counts (marker rows read from
    the table, as the gather does) equal the plain level-2 counts of every
    column.  forced: a cut of n/4, above the least one."""
    g = wide_prefix_graph()
    rp0, ci0 = np.asarray(g.row_ptr, np.int64), np.asarray(g.col_idx, np.int64)
    n = g.n
    deg0 = np.diff(rp0)
    order = np.argsort(-deg0, kind="stable")
    new = np.empty(n, np.int64)
    new[order] = np.arange(n)
    rows = new[np.repeat(np.arange(n), deg0)]
    cols = new[ci0]
    idx = np.lexsort((cols, rows))
    ci = cols[idx]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    deg = np.diff(rp)
    omega2 = np.array([deg[ci[rp[v]:rp[v + 1]]].sum() for v in range(n)], dtype=np.int64)
    wide = np.nonzero(omega2 > 0xFFFE)[0]
    least = int(wide.max()) + 1 if wide.size else 0
    assert least == 600 and wide.size == 600
    cut = n // 4 if forced else least
    C = 8
    rng = np.random.default_rng(17)
    groups = [np.unique(rng.integers(0, n, int(rng.integers(1, 80)))) for _ in range(C)]
    groups[0] = np.array([0, 1, 300])  # members inside the wide prefix
    hub = np.zeros((cut, C), np.uint32)
    words = np.zeros((n, C // 2), np.uint32)

    def add(v, c, val):
        if v < cut:
            hub[v, c] += np.uint32(val)
        else:
            words[v, c // 2] += np.uint32(int(val) << (16 * (c & 1)))

    def half(v, c):
        return int(words[v, c // 2] >> np.uint32(16 * (c & 1))) & 0xFFFF

    def check_halves():
        assert int((words & 0xFFFF).max()) <= 0xFFFE and int((words >> 16).max()) <= 0xFFFE

    cnt1 = np.zeros((n, C), np.int64)
    inS = np.zeros((n, C), bool)
    claimed = [[] for _ in range(C)]
    for c, S in enumerate(groups):
        inS[S, c] = True
    for c, S in enumerate(groups):  # member pushes (k_push)
        for s in S:
            for y in ci[rp[s]:rp[s + 1]]:
                old = cnt1[y, c]
                cnt1[y, c] += 1
                add(int(y), c, deg[s])
                if old == 0 and not inS[y, c]:
                    claimed[c].append(int(y))
    check_halves()
    for c in range(C):  # level-2 push (k_push_wl) and the member raise
        for s in groups[c]:
            cur = int(hub[s, c]) if s < cut else half(s, c)
            assert omega2[s] >= cur
            if s < cut:
                hub[s, c] = omega2[s]
            else:
                add(int(s), c, omega2[s] - cur)
        for y in claimed[c]:
            for x in ci[rp[y]:rp[y + 1]]:
                if not inS[x, c]:
                    add(int(x), c, cnt1[y, c])
        check_halves()
    # the gather's decode: 16-bit halves, rows below the cut from the table
    for c, S in enumerate(groups):
        _, want = push_counts(rp, ci, S, 2)
        got = np.array([int(hub[v, c]) if v < cut else half(v, c) for v in range(n)])
        np.testing.assert_array_equal(got, want)
        assert (want[cut:] <= omega2[cut:]).all()
