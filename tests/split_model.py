"""CPU model of split scoring (test helper, numpy).

Mirrors the steps the HIP split path takes for an undirected graph, so the
design can be checked on the host against the oracle and against exact walk
enumeration: integer pushes for levels 1..s, dense levels s+1..a with member
injection, and the combination of the last level a = ceil(ell/2) with the
lower ones,

    phi_{a+c}(S) = sum_v h_a(v) t_c(v) + sum_{v not in S} (t_a(v) - h_a(v)) h_c(v),

which holds because on an undirected graph a walk of length c leaving v is the
reversal of one ending at v.  Independent of the oracle (shares no code).
"""
from __future__ import annotations

import numpy as np


def _spmv(row_ptr, col_idx, w, x):
    """y(v) = sum over the in-row of v of w * x(u)."""
    n = len(row_ptr) - 1
    y = np.zeros(n)
    for v in range(n):
        j0, j1 = int(row_ptr[v]), int(row_ptr[v + 1])
        if j1 > j0:
            vals = x[col_idx[j0:j1]]
            if w is not None:
                vals = vals * w[j0:j1]
            y[v] = vals.sum()
    return y


def plan(ell: int, weighted: bool):
    a = (ell + 1) // 2
    r = ell - a
    s = 0 if weighted else min(2, a - 1)
    return a, r, s


def push_counts(row_ptr, col_idx, S, s_levels):
    """Level-1/2 integer counts by pushes from the members, as the kernels do."""
    n = len(row_ptr) - 1
    deg = np.diff(row_ptr).astype(np.int64)
    inS = np.zeros(n, dtype=bool)
    inS[S] = True
    cnt1 = np.zeros(n, dtype=np.int64)
    cnt2 = np.zeros(n, dtype=np.int64)
    claimed = []
    for m in S:
        for y in col_idx[row_ptr[m]:row_ptr[m + 1]]:
            old = cnt1[y]
            cnt1[y] += 1
            if s_levels >= 2:
                cnt2[y] += deg[m]
                if old == 0 and not inS[y]:
                    claimed.append(int(y))
    if s_levels >= 2:
        for y in claimed:
            for x in col_idx[row_ptr[y]:row_ptr[y + 1]]:
                cnt2[x] += cnt1[y]
    # member rows hold the unrestricted walk counts
    cnt1[inS] = deg[inS]
    if s_levels >= 2:
        omega2 = np.array([deg[col_idx[row_ptr[v]:row_ptr[v + 1]]].sum() for v in range(n)],
                          dtype=np.int64)
        cnt2[inS] = omega2[inS]
    return cnt1, cnt2


def push3_counts(row_ptr, col_idx, S):
    """Level-3 counts of a single group by the third push, as the kernels do:
    the level-2 pushes list every vertex whose level-2 count they touch first
    (members list themselves), and each listed vertex adds its final level-2
    count to its non-member neighbours; member rows hold omega_3.  Returns
    (count_3, sources)."""
    n = len(row_ptr) - 1
    deg = np.diff(row_ptr).astype(np.int64)
    inS = np.zeros(n, dtype=bool)
    inS[S] = True
    cnt1 = np.zeros(n, dtype=np.int64)
    cnt2 = np.zeros(n, dtype=np.int64)
    level1, sources = [], [int(m) for m in S if deg[m] > 0]
    for m in S:
        for y in col_idx[row_ptr[m]:row_ptr[m + 1]]:
            if cnt1[y] == 0 and not inS[y]:
                level1.append(int(y))
            cnt1[y] += 1
            if cnt2[y] == 0 and not inS[y]:
                sources.append(int(y))
            cnt2[y] += deg[m]
    for y in level1:
        for x in col_idx[row_ptr[y]:row_ptr[y + 1]]:
            if inS[x]:
                continue
            if cnt2[x] == 0:
                sources.append(int(x))
            cnt2[x] += cnt1[y]
    om = omega_levels(row_ptr, col_idx, 3)
    cnt2[inS] = np.array(om[2], dtype=np.int64)[inS]
    cnt3 = np.zeros(n, dtype=np.int64)
    for u in sources:
        for x in col_idx[row_ptr[u]:row_ptr[u + 1]]:
            if not inS[x]:
                cnt3[x] += cnt2[u]
    cnt3[inS] = np.array(om[3], dtype=np.int64)[inS]
    return cnt3, sources


def push3_bound(row_ptr, col_idx, S) -> int:
    """sum over S of deg + omega_2 + omega_3: what the host compares with
    nnz/32 before taking the third push; it bounds the sources' degrees."""
    om = omega_levels(row_ptr, col_idx, 3)
    return int(sum(om[1][v] + om[2][v] + om[3][v] for v in set(int(v) for v in S)))


def split_score(row_ptr, col_idx, S, alpha: float, ell: int, w=None) -> float:
    n = len(row_ptr) - 1
    S = np.unique(np.asarray(S, dtype=np.int64))
    if S.size == 0:
        return 0.0
    inS = np.zeros(n, dtype=bool)
    inS[S] = True
    T = [np.ones(n)]
    for _ in range(ell):
        T.append(alpha * _spmv(row_ptr, col_idx, w, T[-1]))
    a, r, s = plan(ell, w is not None)
    H = {}
    cnt1 = cnt2 = None
    if s >= 1:
        cnt1, cnt2 = push_counts(row_ptr, col_idx, S, s)
        H[1] = alpha * cnt1.astype(np.float64)
        if s >= 2:
            H[2] = (alpha * alpha) * cnt2.astype(np.float64)
    for i in range(s + 1, a + 1):
        if i == 1:
            x, scale = inS.astype(np.float64), alpha
        elif i == s + 1:
            x = (cnt1 if s == 1 else cnt2).astype(np.float64)
            scale = alpha ** (s + 1)
        else:
            x, scale = H[i - 1], alpha
        y = scale * _spmv(row_ptr, col_idx, w, x)
        y[inS] = T[i][inS]
        H[i] = y
    q = np.zeros(n)
    for i in range(1, a):
        q = q + H[i]
    ha = H[a]
    tr = np.zeros(n)
    for c in range(1, r + 1):
        tr = tr + T[c]
    rs = q + ha if r == a else q
    contrib = (q + ha) + ha * tr + np.where(inS, 0.0, (T[a] - ha) * rs)
    return float(contrib.sum())


def omega_levels(row_ptr, col_idx, top: int):
    """omega_i(v) = # walks of length i ending at v, i = 0..top, as exact Python ints."""
    n = len(row_ptr) - 1
    om = [[1] * n]
    for _ in range(top):
        prev = om[-1]
        om.append([sum(prev[int(u)] for u in col_idx[row_ptr[v]:row_ptr[v + 1]])
                   for v in range(n)])
    return om


def count_levels(row_ptr, col_idx, S, top: int):
    """count_i(v) = h_i(v) / alpha^i for i = 1..top as exact Python ints: the
    hit chain's integer walk counts (members hold omega_i)."""
    n = len(row_ptr) - 1
    inS = set(int(v) for v in S)
    om = omega_levels(row_ptr, col_idx, top)
    cnt = [[1 if v in inS else 0 for v in range(n)]]
    for i in range(1, top + 1):
        prev = cnt[-1]
        cnt.append([om[i][v] if v in inS else
                    sum(prev[int(u)] for u in col_idx[row_ptr[v]:row_ptr[v + 1]])
                    for v in range(n)])
    return cnt, om


def split_score_counts(row_ptr, col_idx, S, alpha: float, ell: int) -> float:
    """Split scoring with the dense levels s+1..a-1 kept as unscaled integer
    counts (the 32-bit layout of the kernels): level i weighted by alpha^i in
    the combination, and h_a = alpha^a * (sum of level a-1 counts) outside S."""
    n = len(row_ptr) - 1
    S = np.unique(np.asarray(S, dtype=np.int64))
    if S.size == 0:
        return 0.0
    inS = np.zeros(n, dtype=bool)
    inS[S] = True
    T = [np.ones(n)]
    for _ in range(ell):
        T.append(alpha * _spmv(row_ptr, col_idx, None, T[-1]))
    a, r, s = plan(ell, False)
    assert s == 2 and a - 1 > s, "the count layout has stored levels"
    cnt, _ = count_levels(row_ptr, col_idx, S, a - 1)
    q = np.zeros(n)
    wgt = alpha
    for i in range(1, a):
        q = q + wgt * np.array(cnt[i], dtype=np.float64)
        wgt *= alpha
    alpha_a = alpha ** (s + 1)
    for _ in range(s + 1, a):
        alpha_a *= alpha
    ha = alpha_a * _spmv(row_ptr, col_idx, None, np.array(cnt[a - 1], dtype=np.float64))
    ha[inS] = T[a][inS]
    tr = np.zeros(n)
    for c in range(1, r + 1):
        tr = tr + T[c]
    rs = q + ha if r == a else q
    contrib = (q + ha) + ha * tr + np.where(inS, 0.0, (T[a] - ha) * rs)
    return float(contrib.sum())


def split_gain(row_ptr, col_idx, S, x: int, alpha: float, ell: int, w=None) -> float:
    """L_ell(S, x) from the miss chain and the gain chain up to a = ceil(ell/2),
    as the greedy's split evaluation does:
        L_{a+c} = sum_v d_a(v) m_c(v) + (m_a(v) - d_a(v)) d_c(v)."""
    n = len(row_ptr) - 1
    inS = np.zeros(n, dtype=bool)
    inS[np.asarray(S, dtype=np.int64)] = True
    a = (ell + 1) // 2
    r = ell - a
    m = [(~inS).astype(np.float64)]
    for _ in range(a):
        y = alpha * _spmv(row_ptr, col_idx, w, m[-1])
        y[inS] = 0.0
        m.append(y)
    d = [np.zeros(n)]
    d[0][x] = 1.0
    for i in range(1, a + 1):
        y = alpha * _spmv(row_ptr, col_idx, w, d[-1])
        y[inS] = 0.0
        y[x] = m[i][x]
        d.append(y)
    q = np.zeros(n)
    for i in range(1, a):
        q = q + d[i]
    Mr = np.zeros(n)
    for c in range(1, r + 1):
        Mr = Mr + m[c]
    da = d[a]
    rs = q + da if r == a else q
    contrib = (q + da) + da * Mr + (m[a] - da) * rs
    return float(contrib.sum())


def split_gain_counts(row_ptr, col_idx, S, x: int, alpha: float, ell: int):
    """split_gain with the gain levels 1..a-1 as unscaled integer counts (the
    32-bit layout of the greedy, unweighted graphs without repeated arcs):
    level 1 is 1 on N(x) outside S and the number of x's arcs from outside S
    at x; deeper levels inject the candidate's miss count recovered from the
    FP64 miss chain by rounding m_i(x) / alpha^i; level a is
    alpha^a * (sum of level a-1 counts).  Returns (L, injected counts)."""
    n = len(row_ptr) - 1
    inS = np.zeros(n, dtype=bool)
    inS[np.asarray(S, dtype=np.int64)] = True
    a = (ell + 1) // 2
    r = ell - a
    assert a >= 2
    m = [(~inS).astype(np.float64)]
    for _ in range(a):
        y = alpha * _spmv(row_ptr, col_idx, None, m[-1])
        y[inS] = 0.0
        m.append(y)
    deg = np.diff(row_ptr)
    nbrs = col_idx[row_ptr[x]:row_ptr[x + 1]]
    d1 = np.zeros(n, dtype=np.int64)
    d1[nbrs[~inS[nbrs] & (nbrs != x)]] = 1
    d1[x] = int(deg[x]) - int(inS[nbrs].sum())
    d = [None, d1]
    inj = {}
    ap = alpha
    for i in range(2, a):
        ap *= alpha
        inj[i] = int(np.rint(m[i][x] / ap))
        y = _spmv(row_ptr, col_idx, None, d[-1].astype(np.float64)).astype(np.int64)
        y[inS] = 0
        y[x] = inj[i]
        d.append(y)
    alpha_a = alpha
    for _ in range(1, a):
        alpha_a *= alpha
    da = alpha_a * _spmv(row_ptr, col_idx, None, d[a - 1].astype(np.float64))
    da[inS] = 0.0
    da[x] = m[a][x]
    q = np.zeros(n)
    wgt = alpha
    for i in range(1, a):
        q = q + wgt * d[i].astype(np.float64)
        wgt *= alpha
    Mr = np.zeros(n)
    for c in range(1, r + 1):
        Mr = Mr + m[c]
    rs = q + da if r == a else q
    contrib = (q + da) + da * Mr + (m[a] - da) * rs
    return float(contrib.sum()), inj
