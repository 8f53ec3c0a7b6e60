"""Seeded input generators: determinism and the structure each family promises."""
import numpy as np
import pytest

from paper_1910_13874_amd import inputs


def assert_simple_undirected(g):
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == ci.size
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(ci != rows), "self-loop"
    assert ci.min() >= 0 and ci.max() < g.n
    # sorted strictly increasing inside each row (no duplicates)
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    # symmetric
    a = rows.astype(np.int64) * g.n + ci
    b = ci.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(a), np.sort(b))


def test_er_exact_edge_count_and_determinism():
    g = inputs.erdos_renyi(1000, 5000, 1)
    assert g.n == 1000 and g.nnz == 10000
    assert_simple_undirected(g)
    h = inputs.erdos_renyi(1000, 5000, 1)
    assert np.array_equal(g.col_idx, h.col_idx)
    k = inputs.erdos_renyi(1000, 5000, 2)
    assert not np.array_equal(g.col_idx, k.col_idx)


def test_ba_structure():
    n, m = 5000, 5
    g = inputs.barabasi_albert(n, m, 2)
    assert_simple_undirected(g)
    # seed clique on m+1 vertices, then m distinct edges per new vertex
    assert g.nnz == 2 * ((m + 1) * m // 2 + (n - m - 1) * m)
    assert g.degrees.min() >= m
    # preferential attachment: heavy tail
    assert g.max_degree > 10 * m


def test_rmat_structure_and_thread_independence():
    g = inputs.rmat(12, 16, seed=4)
    assert g.n == 4096
    assert_simple_undirected(g)
    assert (g.degrees == 0).sum() > 0  # isolated vertices kept
    h = inputs.rmat(12, 16, seed=4)
    assert np.array_equal(g.col_idx, h.col_idx)


def test_groups_distinct_sorted_in_range():
    off, mem = inputs.groups(1000, 300, 1, 200, 104)
    sizes = np.diff(off)
    assert sizes.min() >= 1 and sizes.max() <= 200
    assert mem.min() >= 0 and mem.max() < 1000
    for i in range(300):
        grp = mem[off[i]:off[i + 1]]
        assert np.all(np.diff(grp) > 0)
    # small n: full group
    o2, m2 = inputs.groups(5, 1, 5, 5, 9)
    assert list(m2) == [0, 1, 2, 3, 4]


def test_directed_and_reverse():
    g = inputs.from_edges(4, [0, 0, 1, 2], [1, 2, 2, 3], symmetrize=False)
    # rows list in-neighbours
    assert list(g.col_idx[g.row_ptr[2]:g.row_ptr[3]]) == [0, 1]
    r = inputs.reverse(g)
    assert list(r.col_idx[r.row_ptr[0]:r.row_ptr[1]]) == [1, 2]


def test_bad_arguments():
    with pytest.raises(ValueError):
        inputs.erdos_renyi(3, 10, 1)
    with pytest.raises(ValueError):
        inputs.barabasi_albert(3, 5, 1)
