"""Exact-rational reference values for tiny graphs (test helper).

Nothing here uses the paper's recurrences: walk counts come from enumerating
every walk explicitly (the definition of phi_i in Section 2.1, Definition
"GED-Walk"), and the infinite series comes from the matrix identity

    sum_{i>=1} alpha^i * #(i-walks touching S)
        = 1^T [(I - alpha A)^{-1} - I] 1  -  1^T [(I - alpha A_SS)^{-1} - I] 1,

where A_SS is the adjacency of the subgraph induced on V \\ S (a walk misses
S iff it is a walk of that subgraph).  Arithmetic is in ``fractions.Fraction``.
"""
from __future__ import annotations

from collections import Counter
from fractions import Fraction
from itertools import combinations


def out_adjacency(n, row_ptr, col_idx):
    """Arcs u -> v for every u listed in row v (rows are in-neighbour lists)."""
    out = [[] for _ in range(n)]
    for v in range(n):
        for j in range(int(row_ptr[v]), int(row_ptr[v + 1])):
            out[int(col_idx[j])].append(v)
    return out


class WalkTable:
    """All walks of length <= L, tallied by (length, start, end, vertex-set mask)."""

    def __init__(self, n, row_ptr, col_idx, L):
        self.n = n
        self.L = L
        out = out_adjacency(n, row_ptr, col_idx)
        self.tab = [Counter() for _ in range(L + 1)]
        for s in range(n):
            stack = [(s, 1 << s, 0)]
            while stack:
                v, mask, ln = stack.pop()
                self.tab[ln][(s, v, mask)] += 1
                if ln < L:
                    for w in out[v]:
                        stack.append((w, mask | (1 << w), ln + 1))

    @staticmethod
    def _mask(S):
        m = 0
        for s in S:
            m |= 1 << int(s)
        return m

    def phi(self, i, S):
        """# i-walks containing at least one vertex of S."""
        m = self._mask(S)
        return sum(c for (_, _, mk), c in self.tab[i].items() if mk & m)

    def total(self, i):
        return sum(self.tab[i].values())

    def gain_count(self, i, S, x):
        """# i-walks containing x and no vertex of S."""
        m = self._mask(S)
        bx = 1 << int(x)
        return sum(c for (_, _, mk), c in self.tab[i].items() if (mk & bx) and not (mk & m))

    def miss_end(self, i, S, x):
        """# i-walks ending at x that contain no vertex of S."""
        m = self._mask(S)
        return sum(c for (_, e, mk), c in self.tab[i].items() if e == x and not (mk & m))

    def miss_start(self, i, S, x):
        """# i-walks starting at x that contain no vertex of S."""
        m = self._mask(S)
        return sum(c for (s, _, mk), c in self.tab[i].items() if s == x and not (mk & m))

    def ged_partial(self, S, alpha, ell):
        """sum_{i=1}^{ell} alpha^i phi_i(S) as a Fraction."""
        a = Fraction(alpha)
        return sum((a ** i * self.phi(i, S) for i in range(1, ell + 1)), Fraction(0))

    def gain_partial(self, S, x, alpha, ell):
        a = Fraction(alpha)
        return sum((a ** i * self.gain_count(i, S, x) for i in range(1, ell + 1)), Fraction(0))

    def P(self, i, S, x):
        """P_i(S, x) of Lemma "initialize", from explicit walk counts."""
        return sum(self.miss_end(i - j, S, x) * self.miss_start(j, S, x) for j in range(i + 1))


def _solve(M, b):
    """Solve M x = b exactly (Gaussian elimination with Fractions)."""
    n = len(M)
    A = [list(map(Fraction, row)) + [Fraction(bb)] for row, bb in zip(M, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [vr - f * vc for vr, vc in zip(A[r], A[c])]
    return [A[r][n] for r in range(n)]


def _katz_total(vertices, arcs, alpha):
    """1^T [(I - alpha A)^{-1} - I] 1 over the subgraph on `vertices`."""
    idx = {v: i for i, v in enumerate(vertices)}
    m = len(vertices)
    if m == 0:
        return Fraction(0)
    a = Fraction(alpha)
    M = [[Fraction(int(i == j)) for j in range(m)] for i in range(m)]
    for (u, v) in arcs:
        if u in idx and v in idx:
            M[idx[u]][idx[v]] -= a
    x = _solve(M, [1] * m)
    return sum(x) - m


def arcs_of(n, row_ptr, col_idx):
    return [(int(col_idx[j]), v) for v in range(n) for j in range(int(row_ptr[v]), int(row_ptr[v + 1]))]


def ged_exact(n, row_ptr, col_idx, S, alpha):
    """GED(S) = sum_{i>=1} alpha^i phi_i(S) exactly (requires alpha < 1/spectral radius)."""
    arcs = arcs_of(n, row_ptr, col_idx)
    Sset = set(int(s) for s in S)
    rest = [v for v in range(n) if v not in Sset]
    return _katz_total(list(range(n)), arcs, alpha) - _katz_total(rest, arcs, alpha)


def opt_exact(n, row_ptr, col_idx, k, alpha):
    """max over |S| = k of GED(S), by brute force (exact)."""
    arcs = arcs_of(n, row_ptr, col_idx)
    tot = _katz_total(list(range(n)), arcs, alpha)
    best = None
    for S in combinations(range(n), k):
        Sset = set(S)
        val = tot - _katz_total([v for v in range(n) if v not in Sset], arcs, alpha)
        if best is None or val > best[0]:
            best = (val, S)
    return best


def induced_walk_counts(n, arcs, keep, ell):
    """w_i = 1^T (A_keep)^i 1 for i = 0..ell: walk counts of the induced subgraph."""
    keep = set(keep)
    out = {v: [] for v in keep}
    for (u, v) in arcs:
        if u in keep and v in keep:
            out[u].append(v)
    x = {v: 1 for v in keep}  # x_i(v) = # i-walks ending at v
    res = [len(keep)]
    for _ in range(ell):
        y = {v: 0 for v in keep}
        for u in keep:
            for v in out[u]:
                y[v] += x[u]
        x = y
        res.append(sum(x.values()))
    return res


def exact_gain(n, arcs, S, x, alpha, ell):
    """L_ell(S, x): alpha-weighted i-walks (i <= ell) containing x, avoiding S.

    Walks avoiding S are the walks of the subgraph induced on V \\ S; those that
    also avoid x live on V \\ (S + x).  Exact integers, so the difference is exact.
    """
    a = Fraction(alpha)
    Sset = set(int(s) for s in S)
    U = [v for v in range(n) if v not in Sset]
    Ux = [v for v in U if v != x]
    w1 = induced_walk_counts(n, arcs, U, ell)
    w2 = induced_walk_counts(n, arcs, Ux, ell)
    return sum((a ** i * (w1[i] - w2[i]) for i in range(1, ell + 1)), Fraction(0))


def exact_bound(n, arcs, alpha, delta, ell):
    """alpha^{ell+1} * delta/(1 - alpha*delta) * sum_x omega_ell(x) (Eq. comb-bound)."""
    a = Fraction(alpha)
    w = induced_walk_counts(n, arcs, range(n), ell)
    return a ** (ell + 1) * Fraction(delta) / (1 - a * delta) * w[ell]


def exact_greedy(n, arcs, k, alpha, eps, delta, max_ell=1 << 12, follow=None):
    """Eager greedy with (eps/k)-separation and doubling walk length, in exact
    arithmetic (decision rule of Section 3.2.2; ties to the smaller id).

    ``follow``: a pick sequence to follow inside classes of exactly tied best
    gains (a floating-point run may break an exact tie either way).  Returns
    (picks, ells, tie_flags) where tie_flags[p] says whether the best and the
    runner-up gains were exactly equal at the accepted step.
    """
    eps = Fraction(eps)
    S, ells, ties = [], [], []
    ell = 1
    while len(S) < k:
        if ell > max_ell:
            raise RuntimeError("walk length limit")
        B = exact_bound(n, arcs, alpha, delta, ell)
        while len(S) < k:
            cand = [v for v in range(n) if v not in S]
            gains = sorted(((exact_gain(n, arcs, S, x, alpha, ell), -x) for x in cand), reverse=True)
            L1, u = gains[0][0], -gains[0][1]
            if len(gains) > 1:
                L2 = gains[1][0]
                if L1 <= L2 + B - eps / k:
                    break
                ties.append(L1 == L2)
                if follow is not None and len(follow) > len(S):
                    tied = {-x for (gv, x) in gains if gv == L1}
                    if int(follow[len(S)]) in tied:
                        u = int(follow[len(S)])
            else:
                ties.append(False)
            S.append(u)
            ells.append(ell)
        if len(S) < k:
            ell *= 2
    return S, ells, ties


def weighted_arcs(n, row_ptr, col_idx, w):
    """(u, v, weight) for every arc u -> v (row v lists u), weights as Fractions."""
    return [(int(col_idx[j]), v, Fraction(float(w[j])))
            for v in range(n) for j in range(int(row_ptr[v]), int(row_ptr[v + 1]))]


def weighted_walk_sums(n, warcs, S, L):
    """phi^w_i(S) = sum over i-walks touching S of the product of arc weights,
    i = 0..L, by explicit enumeration."""
    out = {u: [] for u in range(n)}
    for (u, v, wt) in warcs:
        out[u].append((v, wt))
    Sset = set(int(s) for s in S)
    res = [Fraction(0)] * (L + 1)
    for s in range(n):
        stack = [(s, s in Sset, Fraction(1), 0)]
        while stack:
            v, hit, prod, ln = stack.pop()
            if hit:
                res[ln] += prod
            if ln < L:
                for (w2, wt) in out[v]:
                    stack.append((w2, hit or (w2 in Sset), prod * wt, ln + 1))
    return res


def weighted_ged_exact(n, warcs, S, alpha):
    """Closed form with the weighted adjacency: 1^T[(I-aW)^-1 - I]1 minus the
    same over the subgraph induced on V \\ S."""
    a = Fraction(alpha)

    def katz(vertices):
        idx = {v: i for i, v in enumerate(vertices)}
        m = len(vertices)
        if m == 0:
            return Fraction(0)
        M = [[Fraction(int(i == j)) for j in range(m)] for i in range(m)]
        for (u, v, wt) in warcs:
            if u in idx and v in idx:
                M[idx[u]][idx[v]] -= a * wt
        x = _solve(M, [1] * m)
        return sum(x) - m

    Sset = set(int(s) for s in S)
    return katz(list(range(n))) - katz([v for v in range(n) if v not in Sset])
