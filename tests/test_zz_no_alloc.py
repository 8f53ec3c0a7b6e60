"""ged_score_noalloc: the single-group score for callers that cannot allocate.
Called through the C ABI and checked against ged_score on the same graph and
group (FP64, 1e-9 relative, the same ell*) and against the oracle; two graphs
in a row, the second smaller, so the second call runs on the working memory
the first one left behind."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1910_13874_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 1e-4
REL = 1e-9


@pytest.fixture(scope="module")
def ged():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_13874_amd import ged as mod
    return mod


def rel(a, b):
    return 0.0 if a == b else abs(a - b) / max(abs(a), abs(b))


def noalloc(ged, gg, S, alpha, eps=EPS):
    """Returns (status, score, ell*)."""
    fn = ged._lib.ged_score_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                   ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                   ctypes.POINTER(ged.ScoreInfo)]
    arr = np.ascontiguousarray(S, dtype=np.int32)
    out = ctypes.c_double(np.nan)
    info = ged.ScoreInfo()
    rc = fn(gg.handle, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if arr.size else None,
            int(arr.size), alpha, eps, ctypes.byref(out), ctypes.byref(info))
    return rc, out.value, info.ell


def check(ged, g, gg, S, alpha, tag, w=None):
    rc, s, ell = noalloc(ged, gg, S, alpha)
    assert rc == 0, (tag, rc, ged._lib.ged_last_error())
    ref, ell_ref, _ = gg.score(S, alpha, EPS, with_info=True)
    c, ell_o, _, _ = oracle.score(g, S, alpha, EPS, w=w)
    print(f"  {tag}: |S|={len(S)} noalloc={s!r} ged_score={ref!r} oracle={c!r}", flush=True)
    assert ell == ell_ref == ell_o, (tag, ell, ell_ref, ell_o)
    assert rel(s, ref) <= REL, (tag, s, ref)
    assert rel(s, c) <= REL, (tag, s, c)


def test_noalloc_matches_score_two_graphs(ged):
    big = inputs.barabasi_albert(200000, 5, 91)
    small = inputs.erdos_renyi(3000, 9000, 92)
    for name, g, sizes in (("ba200k", big, [(1, 60), (2, 7)]), ("er3k", small, [(3, 4)])):
        print(f"[noalloc] {name} n={g.n} nnz={g.nnz}", flush=True)
        gg = ged.GedGraph.from_graph(g)
        alpha = gg.default_alpha()
        rc, _, _ = noalloc(ged, gg, [0, 1], alpha)
        assert rc == -1, rc  # not prepared yet: refused, nothing computed
        gg.prepare(alpha, EPS)
        for seed, size in sizes:
            S = inputs.group(g.n, size, seed)
            # duplicates count once, as in ged_score
            check(ged, g, gg, np.concatenate([S, S[:2]]), alpha, (name, seed))
        assert noalloc(ged, gg, [], alpha)[:2] == (0, 0.0)
        assert noalloc(ged, gg, [g.n], alpha)[0] == -2
        gg.close()


def test_noalloc_directed_weighted_and_limit(ged):
    n = 2000
    r = inputs.uniform_ints(2 * 9000, n, 61)
    gd = inputs.from_edges(n, r[0::2], r[1::2], symmetrize=False, name="dir2k")
    gw = inputs.barabasi_albert(20000, 4, 25)
    deg = gw.degrees.astype(np.float64)
    rows = np.repeat(np.arange(gw.n), gw.degrees)
    w = 1.0 / np.sqrt(deg[rows] * deg[gw.col_idx])
    for name, g, wt in (("directed", gd, None), ("weighted", gw, w)):
        print(f"[noalloc] {name} n={g.n}", flush=True)
        gg = ged.GedGraph.from_graph(g, weights=wt)
        alpha = gg.default_alpha()
        gg.prepare(alpha, EPS)
        check(ged, g, gg, inputs.group(g.n, 9, 5), alpha, name, w=wt)
        gg.close()
    # a graph whose two hit-chain vectors alone exceed the fixed working memory
    big = inputs.from_edges(6_000_000, [0], [1])
    gg = ged.GedGraph.from_graph(big)
    alpha = gg.default_alpha()
    gg.prepare(alpha, EPS)
    rc, _, _ = noalloc(ged, gg, [0, 5], alpha)
    assert rc == -6, rc
    assert "maximum" in ged._lib.ged_last_error().decode()
    gg.close()
