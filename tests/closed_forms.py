"""Closed forms that pin scores without sharing code with the oracle or the
HIP path (scipy sparse products only)."""
import numpy as np


def whole_set_score(g, alpha, ell):
    """GED(V): every walk meets V, so the score truncated at ell is the
    weighted count of all walks, sum_{i<=ell} alpha^i 1^T A^i 1."""
    import scipy.sparse as sp
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    x = np.ones(g.n)
    total = 0.0
    for i in range(1, ell + 1):
        x = A @ x
        total += alpha ** i * float(x.sum())
    return total


def group_score(g, S, alpha, ell, w=None):
    """GED(S) from its definition by complement: the walks that meet S are all
    walks minus those whose every vertex lies outside S, i.e. the walks of the
    subgraph induced by V \\ S.  y_i(v) counts walks of length i ending at v
    that avoid S: y_0 = 1_{V\\S}, y_i = 1_{V\\S} * (A y_{i-1}).  Row v of A
    holds the in-arcs u -> v, so directed graphs count walks along the arcs;
    per-arc weights w (aligned with col_idx) weight a walk by their product."""
    import scipy.sparse as sp
    data = np.ones(g.nnz) if w is None else np.asarray(w, dtype=np.float64)
    A = sp.csr_matrix((data, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    keep = np.ones(g.n)
    keep[np.asarray(S, dtype=np.int64)] = 0.0
    x = np.ones(g.n)
    y = keep.copy()
    total = 0.0
    for i in range(1, ell + 1):
        x = A @ x
        y = keep * (A @ y)
        total += alpha ** i * (float(x.sum()) - float(y.sum()))
    return total


def gain(g, S, u, alpha, ell):
    """Marginal gain GED_{<=ell}(S + u) - GED_{<=ell}(S): the walks that avoid S
    but not u, i.e. the avoiding-walk counts of V \\ S minus those of V \\ (S + u)."""
    import scipy.sparse as sp
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    k1 = np.ones(g.n)
    k1[np.asarray(S, dtype=np.int64)] = 0.0
    k2 = k1.copy()
    k2[u] = 0.0
    y1, y2 = k1.copy(), k2.copy()
    total = 0.0
    for i in range(1, ell + 1):
        y1 = k1 * (A @ y1)
        y2 = k2 * (A @ y2)
        total += alpha ** i * (float(y1.sum()) - float(y2.sum()))
    return total
