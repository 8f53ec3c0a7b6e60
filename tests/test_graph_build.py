"""Host-side graph construction (graph_build.h), driven on the CPU: the
header is built with g++ into a small shared library, and its output -- the
internal vertex order, the in- and out-rows in internal ids, the maximum
(weighted) degree and the multigraph flag -- is compared with a direct
construction in numpy, at thread counts 1 to 16; validation errors are the
same at every thread count."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1910_13874_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
F64P = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("gbuild") / "libgbuild.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-pthread",
                    "-I", os.path.join(ROOT, "paper_1910_13874_amd", "csrc"),
                    os.path.join(ROOT, "tests", "build_shim.cpp"), "-o", out], check=True)
    L = ctypes.CDLL(out)
    L.gb_build.restype = ctypes.c_char_p
    L.gb_build.argtypes = [ctypes.c_int64, ctypes.c_int64, I64P, I32P, F64P, ctypes.c_int,
                           ctypes.c_int, ctypes.c_int, I32P, I32P, I32P, I32P, F64P, I32P, I32P,
                           F64P, I32P, F64P, I32P]
    L.gb_threads.restype = ctypes.c_int
    L.gb_threads.argtypes = [ctypes.c_int64, ctypes.c_int64]
    L.gb_threads_rethrow.restype = ctypes.c_int
    L.gb_threads_rethrow.argtypes = [ctypes.c_int, ctypes.c_int]
    return L


def build(L, n, rp, ci, w=None, undirected=True, keep_order=False, threads=1):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci if len(ci) else np.zeros(1), dtype=np.int32)
    nnz = int(rp[-1])
    ne = max(1, nnz)
    o = {"new_id": np.zeros(n, np.int32), "old_id": np.zeros(n, np.int32),
         "irp": np.zeros(n + 1, np.int32), "ici": np.zeros(ne, np.int32),
         "iw": np.zeros(ne), "orp": np.zeros(n + 1, np.int32), "oci": np.zeros(ne, np.int32),
         "ow": np.zeros(ne)}
    md, mw, simple = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float64)
        wp = w.ctypes.data_as(F64P)
    p = lambda a: a.ctypes.data_as(F64P if a.dtype == np.float64 else I32P)  # noqa: E731
    msg = L.gb_build(n, nnz, rp.ctypes.data_as(I64P), ci.ctypes.data_as(I32P), wp,
                     int(undirected), int(keep_order), threads, p(o["new_id"]), p(o["old_id"]),
                     p(o["irp"]), p(o["ici"]), p(o["iw"]), p(o["orp"]), p(o["oci"]), p(o["ow"]),
                     ctypes.byref(md), ctypes.byref(mw), ctypes.byref(simple))
    if msg is not None:
        return msg.decode()
    o.update(max_deg=md.value, max_wdeg=mw.value, simple=bool(simple.value), nnz=nnz)
    return o


def reference(n, rp, ci, w=None, keep_order=False):
    """The same arrays by definition: vertices by decreasing out-degree (ties
    in caller order), row v of the in-rows lists the internal sources of the
    arcs into v in increasing order (equal sources in arc order), the out-rows
    likewise for the reverse graph."""
    rp = np.asarray(rp, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int64)
    nnz = int(rp[-1])
    rows = np.repeat(np.arange(n), np.diff(rp))
    outdeg = np.bincount(ci, minlength=n)
    old = np.arange(n) if keep_order else np.argsort(-outdeg, kind="stable")
    new = np.empty(n, dtype=np.int64)
    new[old] = np.arange(n)
    nv, nu, j = new[rows], new[ci], np.arange(nnz)
    oi = np.lexsort((j, nu, nv))
    oo = np.lexsort((j, nv, nu))
    r = {"new_id": new, "old_id": old,
         "irp": np.concatenate([[0], np.cumsum(np.bincount(nv, minlength=n))]),
         "orp": np.concatenate([[0], np.cumsum(np.bincount(nu, minlength=n))]),
         "ici": nu[oi], "oci": nv[oo], "max_deg": int(outdeg.max()) if n else 0}
    key = nv[oi] * n + nu[oi]
    r["simple"] = bool(np.all(np.diff(key) != 0)) if nnz > 1 else True
    if w is not None:
        w = np.asarray(w, dtype=np.float64)
        r["iw"], r["ow"] = w[oi], w[oo]
        wout = np.zeros(n)
        np.add.at(wout, ci, w)  # in arc order, as the builder adds them
        r["max_wdeg"] = float(wout.max())
    return r


def check_same(o, r, weighted, directed):
    """The out-row entries are built for directed graphs only (an undirected
    graph's equal its in-rows)."""
    nnz = o["nnz"]
    for k in ("new_id", "old_id", "irp", "orp"):
        np.testing.assert_array_equal(o[k], r[k], err_msg=k)
    np.testing.assert_array_equal(o["ici"][:nnz], r["ici"], err_msg="ici")
    if directed:
        np.testing.assert_array_equal(o["oci"][:nnz], r["oci"], err_msg="oci")
    else:
        np.testing.assert_array_equal(r["oci"], r["ici"])
        np.testing.assert_array_equal(r["orp"], r["irp"])
    assert o["max_deg"] == r["max_deg"] and o["simple"] == r["simple"]
    if weighted:
        np.testing.assert_array_equal(o["iw"][:nnz], r["iw"])
        if directed:
            np.testing.assert_array_equal(o["ow"][:nnz], r["ow"])
        assert o["max_wdeg"] == r["max_wdeg"]


def csr_from_arcs(n, src, dst):
    """Rows by destination, sources in the order given (not sorted)."""
    order = np.argsort(dst, kind="stable")
    rp = np.concatenate([[0], np.cumsum(np.bincount(dst, minlength=n))])
    return rp, np.asarray(src)[order].astype(np.int32), order


def multigraph():
    """Undirected, with doubled and tripled edges and shuffled rows."""
    rng = np.random.default_rng(7)
    n = 400
    e = rng.integers(0, n, size=(3000, 2))
    e = e[e[:, 0] != e[:, 1]]
    e = np.concatenate([e, e[:200], e[:50]])
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    perm = rng.permutation(src.size)
    rp, ci, _ = csr_from_arcs(n, src[perm], dst[perm])
    return n, rp, ci


def cases():
    ba = inputs.barabasi_albert(5000, 4, 11)
    rm = inputs.rmat(12, 8)
    r = inputs.uniform_ints(2 * 6000, 1500, 62)
    dg = inputs.from_edges(1500, r[0::2], r[1::2], symmetrize=False, name="dir")
    deg = ba.degrees.astype(np.float64)
    rows = np.repeat(np.arange(ba.n), ba.degrees)
    wsym = 1.0 / np.sqrt(deg[rows] * deg[ba.col_idx])
    mn, mrp, mci = multigraph()
    return [("ba", ba.n, ba.row_ptr, ba.col_idx, None, True),
            ("rmat12", rm.n, rm.row_ptr, rm.col_idx, None, True),
            ("directed", dg.n, dg.row_ptr, dg.col_idx, None, False),
            ("weighted", ba.n, ba.row_ptr, ba.col_idx, wsym, True),
            ("multigraph", mn, mrp, mci, None, True),
            ("directed_weighted", dg.n, dg.row_ptr, dg.col_idx,
             0.25 + 0.5 * inputs.uniform_doubles(dg.nnz, 63), False),
            ("single", 1, np.array([0, 0]), np.array([], dtype=np.int32), None, True),
            ("isolated", 5, np.zeros(6, dtype=np.int64), np.array([], dtype=np.int32), None, True)]


@pytest.mark.parametrize("keep_order", [False, True])
def test_build_matches_definition(lib, keep_order):
    for name, n, rp, ci, w, und in cases():
        r = reference(n, rp, ci, w, keep_order)
        for T in (1, 2, 3, 7, 16):
            o = build(lib, n, rp, ci, w, und, keep_order, T)
            assert isinstance(o, dict), (name, T, o)
            check_same(o, r, w is not None, not und)


def test_build_default_threads(lib):
    """Above 2^20 arcs the default uses several threads (at most 16 and
    nnz / n), and the result is the single-threaded one."""
    g = inputs.barabasi_albert(100000, 8, 12)
    T = lib.gb_threads(g.n, g.nnz)
    hw = os.cpu_count() or 1
    assert T == max(1, min(16, hw, g.nnz // g.n))
    assert lib.gb_threads(1000, 5000) == 1
    o = build(lib, g.n, g.row_ptr, g.col_idx, threads=0)
    check_same(o, reference(g.n, g.row_ptr, g.col_idx), False, False)


def test_build_errors(lib):
    """The first error by row, whatever the thread count: a decreasing
    row_ptr before any arc check, then (row by row) a source out of range, a
    self-loop or a weight outside (0, 1], then asymmetry."""
    g = inputs.barabasi_albert(3000, 3, 13)
    n, rp, ci = g.n, g.row_ptr.astype(np.int64), g.col_idx.copy()

    def expect(msg, rp_, ci_, w=None, und=True):
        for T in (1, 2, 5, 16):
            assert build(lib, n, rp_, ci_, w, und, False, T) == msg, (msg, T)

    bad = rp.copy()
    bad[n // 2] = bad[n // 2 + 1] + 1  # a decrease in the middle
    c2 = ci.copy()
    c2[-1] = n  # out of range in the last row
    expect("row_ptr decreases", bad, c2)
    expect("col_idx out of range", rp, c2)
    c3 = c2.copy()
    c3[rp[n // 3]] = n // 3  # a self-loop in an earlier row comes first
    expect("self-loop", rp, c3)
    w = np.full(g.nnz, 0.5)
    w[rp[n - 1]] = 0.0
    expect("weights must be in (0, 1]", rp, ci, w)
    w2 = np.full(g.nnz, 0.5)
    w2[rp[10]] = 0.25  # one direction of an edge weighted differently
    expect("GED_UNDIRECTED graph is not symmetric", rp, ci, w2)
    c4 = ci.copy()
    row = int(np.argmax(np.diff(rp)))
    c4[rp[row]] = (c4[rp[row]] + 1) % n if (c4[rp[row]] + 1) % n != row else (c4[rp[row]] + 2) % n
    expect("GED_UNDIRECTED graph is not symmetric", rp, c4)
    assert isinstance(build(lib, n, rp, c4, None, False, False, 3), dict)  # fine as directed


def test_thread_failure_reaches_the_caller(lib):
    """A part that throws (a failed host allocation) does not end the process:
    the exception reaches the builder's caller, which turns it into an error
    code, after the other parts have run."""
    for T, bad in ((1, 0), (4, 0), (4, 3), (16, 7)):
        assert lib.gb_threads_rethrow(T, bad) == 1, (T, bad)
