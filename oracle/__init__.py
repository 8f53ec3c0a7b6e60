"""ORACLE -- test infrastructure only.

ctypes wrapper around ``ged_oracle.c``: a plain single-threaded FP64 CPU
implementation of GED-Walk scoring (Section 3.1, Algorithm "GED-Walk
Computation") and lazy greedy maximisation (Section 3.2.2, Algorithm "lazy
greedy", with the initialisation of Lemma "initialize").  Only ``tests/``, the
smoke check and the benchmark's CPU-baseline leg use it; the GPU library never
imports, links or calls anything here.

Graphs are passed as any object with ``n``, ``row_ptr`` (int64[n+1]) and
``col_idx`` (int32[nnz]) attributes, rows listing in-neighbours.  For directed
graphs the reverse graph (rows = out-neighbours) must be given as ``rev``.

Parity pinning: every function here is checked by ``tests/test_oracle_pins.py``
against brute-force walk enumeration in exact rational arithmetic, the
closed-form value of the infinite series, the paper's structural properties
(monotonicity, submodularity, GED(V) = sum of Katz scores, vertex covers) and
the greedy approximation guarantee.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libged_oracle.so")
_lib = None

P_I64 = ctypes.POINTER(ctypes.c_int64)
P_I32 = ctypes.POINTER(ctypes.c_int32)
P_F64 = ctypes.POINTER(ctypes.c_double)
P_U8 = ctypes.POINTER(ctypes.c_uint8)

ERRORS = {-1: "bad argument", -2: "vertex out of range", -3: "alpha out of range",
          -4: "eps out of range", -6: "out of memory", -9: "walk length limit reached"}


def build():
    """Compile the oracle with gcc (used by the build step; never by the GPU path)."""
    import subprocess
    src = os.path.join(_HERE, "ged_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", src, "-o", _LIB_PATH + ".tmp",
           "-lm"]
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} missing: run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.or_max_out_degree.argtypes = [ctypes.c_int64, P_I64, P_I32]
    lib.or_max_out_degree.restype = ctypes.c_int64
    lib.or_walk_totals.argtypes = [ctypes.c_int64, P_I64, P_I32, ctypes.c_double, ctypes.c_int32,
                                   P_F64]
    lib.or_comb_bound.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.or_set_weights.argtypes = [P_F64, P_F64]
    lib.or_set_weights.restype = None
    lib.or_max_weighted_out_degree.argtypes = [ctypes.c_int64, P_I64, P_I32, P_F64]
    lib.or_max_weighted_out_degree.restype = ctypes.c_double
    lib.or_greedy_ex.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I64, P_I32, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_uint64, P_I32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P_I32, P_I32,
                                 P_F64, P_F64, P_F64, P_F64, P_I64, P_F64, P_I32]
    lib.or_greedy_ex.restype = ctypes.c_int
    lib.or_sample.argtypes = [ctypes.c_int64, P_I32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, P_I32]
    lib.or_sample.restype = ctypes.c_int64
    lib.or_comb_bound.restype = ctypes.c_double
    lib.or_score.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I32, ctypes.c_int32, ctypes.c_double,
                             ctypes.c_double, ctypes.c_int32, P_F64, P_I32, P_F64, P_F64]
    lib.or_score_fixed.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_int32, P_F64, P_F64]
    lib.or_gain_ext.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P_F64]
    lib.or_pinit_ext.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I64, P_I32, P_I32,
                                 ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P_F64]
    lib.or_greedy.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I64, P_I32, ctypes.c_int32,
                              ctypes.c_double, ctypes.c_double, ctypes.c_int32, P_I32,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P_I32, P_I32,
                              P_F64, P_F64, P_F64, P_F64, P_I64, P_F64, P_I32]
    lib.or_set_spectral.argtypes = [ctypes.c_double]
    lib.or_set_spectral.restype = None
    lib.or_spectral_bound.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                      ctypes.c_double]
    lib.or_spectral_bound.restype = ctypes.c_double
    lib.or_sigma_max.argtypes = [ctypes.c_int64, P_I64, P_I32, P_I64, P_I32, ctypes.c_int32,
                                 P_F64]
    for f in ("or_walk_totals", "or_score", "or_score_fixed", "or_gain_ext", "or_pinit_ext",
              "or_greedy", "or_sigma_max"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


class _Weights:
    """Install arc weights (aligned with col_idx; rev aligned with the reverse
    graph's col_idx) for the duration of one oracle call.  Unweighted calls
    leave the library's (unweighted) default untouched, so they may run
    concurrently from several threads."""

    def __init__(self, w, w_rev):
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        self.w_rev = None if w_rev is None else np.ascontiguousarray(w_rev, dtype=np.float64)

    def __enter__(self):
        if self.w is None and self.w_rev is None:
            return
        lib = _load()
        lib.or_set_weights(self.w.ctypes.data_as(P_F64) if self.w is not None else None,
                           self.w_rev.ctypes.data_as(P_F64) if self.w_rev is not None else None)

    def __exit__(self, *a):
        if self.w is not None or self.w_rev is not None:
            _load().or_set_weights(None, None)


class _Spectral:
    """Select the spectral tail bound with upper estimate `sigma` of sigma_max
    (None: the combinatorial bound, the library's default, left untouched)
    for the duration of one oracle call."""

    def __init__(self, sigma):
        self.sigma = 0.0 if sigma is None else float(sigma)

    def __enter__(self):
        if self.sigma != 0.0:
            _load().or_set_spectral(self.sigma)

    def __exit__(self, *a):
        if self.sigma != 0.0:
            _load().or_set_spectral(0.0)


def _ck(rc):
    if rc != 0:
        raise ValueError(f"oracle error {rc}: {ERRORS.get(rc, '?')}")


def _arrs(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci


def _grp(S):
    S = np.ascontiguousarray(np.asarray(S, dtype=np.int32).reshape(-1))
    buf = S if S.size else np.zeros(1, dtype=np.int32)
    return buf, int(S.size)


def max_out_degree(g) -> int:
    rp, ci = _arrs(g)
    return int(_load().or_max_out_degree(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32)))


def max_weighted_out_degree(g, w) -> float:
    rp, ci = _arrs(g)
    w = np.ascontiguousarray(w, dtype=np.float64)
    return float(_load().or_max_weighted_out_degree(g.n, rp.ctypes.data_as(P_I64),
                                                    ci.ctypes.data_as(P_I32),
                                                    w.ctypes.data_as(P_F64)))


def default_alpha(g, w=None) -> float:
    if w is not None:
        return 1.0 / (max_weighted_out_degree(g, w) + 1.0)
    return 1.0 / (max_out_degree(g) + 1)


def walk_totals(g, alpha: float, ell: int) -> np.ndarray:
    """W[i] = alpha^i * sum_x omega_i(x), i = 0..ell."""
    rp, ci = _arrs(g)
    W = np.zeros(ell + 1)
    _ck(_load().or_walk_totals(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32), alpha,
                               ell, W.ctypes.data_as(P_F64)))
    return W


def comb_bound(g, alpha: float, ell: int, w=None) -> float:
    """B_ell(V), the combinatorial tail bound (Section 3.1.2, Eq. comb-bound)."""
    with _Weights(w, None):
        W = walk_totals(g, alpha, ell)
    D = max_weighted_out_degree(g, w) if w is not None else max_out_degree(g)
    return float(_load().or_comb_bound(alpha, float(D), W[ell]))


SIGMA_ITERS = 100


def sigma_max(g, rev=None, w=None, w_rev=None, iters: int = SIGMA_ITERS) -> float:
    """Upper estimate of sigma_max(A) (Collatz-Wielandt on A^T A, power steps
    on A^T A + I from the all-ones vector); what the spectral bound uses."""
    rp, ci = _arrs(g)
    rr, cr = _arrs(rev if rev is not None else g)
    out = ctypes.c_double()
    with _Weights(w, w_rev if w_rev is not None else w):
        rc = _load().or_sigma_max(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                                  rr.ctypes.data_as(P_I64), cr.ctypes.data_as(P_I32), iters,
                                  ctypes.byref(out))
    _ck(rc)
    return out.value


def spectral_bound(g, alpha: float, ell: int, sigma: float, w=None) -> float:
    """B_ell(V) by the spectral bound (Lemma "spectral-bound") with sigma."""
    with _Weights(w, None):
        W = walk_totals(g, alpha, ell)
    return float(_load().or_spectral_bound(alpha, float(sigma), g.n, W[ell]))


def score(g, S, alpha: float, eps: float, max_ell: int = 100000, w=None, sigma=None):
    """GED_{<=ell*}(S) by the paper's score algorithm.

    Returns (c, ell*, B_ell*, phi) with phi[i] = alpha^i phi_i(S), i = 0..ell*.
    sigma (an upper estimate of sigma_max) selects the spectral tail bound.
    """
    rp, ci = _arrs(g)
    Sb, sl = _grp(S)
    c = ctypes.c_double()
    ell = ctypes.c_int32()
    B = ctypes.c_double()
    phi = np.zeros(max_ell + 1)
    with _Weights(w, None), _Spectral(sigma):
        rc = _load().or_score(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                         Sb.ctypes.data_as(P_I32), sl, alpha, eps, max_ell, ctypes.byref(c),
                         ctypes.byref(ell), ctypes.byref(B), phi.ctypes.data_as(P_F64))
    _ck(rc)
    return c.value, ell.value, B.value, phi[: ell.value + 1].copy()


def score_fixed(g, S, alpha: float, ell: int, w=None):
    """GED_{<=ell}(S) at a fixed walk length; returns (c, phi[0..ell])."""
    rp, ci = _arrs(g)
    Sb, sl = _grp(S)
    c = ctypes.c_double()
    phi = np.zeros(ell + 1)
    with _Weights(w, None):
        rc = _load().or_score_fixed(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                                    Sb.ctypes.data_as(P_I32), sl, alpha, ell, ctypes.byref(c),
                                    phi.ctypes.data_as(P_F64))
    _ck(rc)
    return c.value, phi


def gain(g, S, x: int, alpha: float, ell: int, w=None) -> float:
    """L_ell(S, x) = GED_{<=ell}(S + x) - GED_{<=ell}(S), walk-counted."""
    rp, ci = _arrs(g)
    Sb, sl = _grp(S)
    out = ctypes.c_double()
    with _Weights(w, None):
        rc = _load().or_gain_ext(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                                 Sb.ctypes.data_as(P_I32), sl, int(x), alpha, ell,
                                 ctypes.byref(out))
    _ck(rc)
    return out.value


def pinit(g, S, alpha: float, ell: int, rev=None, w=None, w_rev=None) -> np.ndarray:
    """I(x) = sum_{i=1}^{ell} alpha^i P_i(S, x) for every x (0 for x in S)."""
    rp, ci = _arrs(g)
    rr, cr = _arrs(rev if rev is not None else g)
    Sb, sl = _grp(S)
    out = np.zeros(g.n)
    with _Weights(w, w_rev if w_rev is not None else (w if rev is None else None)):
        rc = _load().or_pinit_ext(g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                                  rr.ctypes.data_as(P_I64), cr.ctypes.data_as(P_I32),
                                  Sb.ctypes.data_as(P_I32), sl, alpha, ell,
                                  out.ctypes.data_as(P_F64))
    _ck(rc)
    return out


def greedy(g, k: int, alpha: float, eps: float, lazy: bool = True, forced=None,
           forced_ell: int = 1, max_ell: int = 1 << 16, rev=None, with_score: bool = True,
           stochastic: bool = False, eta: float = 0.1, seed: int = 1, w=None, w_rev=None,
           sigma=None, stop_after: int = 0):
    """Greedy GED-Walk maximisation (lazy greedy with P-initialisation).

    Returns a dict: group (pick order), ell/L1/U2/L2/B/evals per pick, score
    (GED_{<=ell*} of the final group) and score_ell.  stop_after = m > 0
    returns after the first m picks of the k-pick run (the separation
    threshold stays eps/k); the arrays then hold m valid entries.
    """
    rp, ci = _arrs(g)
    rr, cr = _arrs(rev if rev is not None else g)
    fb, nf = _grp(forced if forced is not None else [])
    grp = np.zeros(k, dtype=np.int32)
    t_ell = np.zeros(k, dtype=np.int32)
    t_L1 = np.zeros(k)
    t_U2 = np.zeros(k)
    t_L2 = np.zeros(k)
    t_B = np.zeros(k)
    t_ev = np.zeros(k, dtype=np.int64)
    sc = ctypes.c_double(math.nan)
    sc_ell = ctypes.c_int32(0)
    if w is not None and rev is not None and w_rev is None:
        raise ValueError("a weighted directed graph needs the reverse graph's weights")
    with _Weights(w, w_rev if w_rev is not None else w), _Spectral(sigma):
        rc = _load().or_greedy_ex(
                          g.n, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                          rr.ctypes.data_as(P_I64), cr.ctypes.data_as(P_I32), k, alpha, eps,
                          1 if lazy else 0, 1 if stochastic else 0, eta, seed,
                          fb.ctypes.data_as(P_I32), nf, forced_ell, max_ell, stop_after,
                          grp.ctypes.data_as(P_I32), t_ell.ctypes.data_as(P_I32),
                          t_L1.ctypes.data_as(P_F64), t_U2.ctypes.data_as(P_F64),
                          t_L2.ctypes.data_as(P_F64), t_B.ctypes.data_as(P_F64),
                          t_ev.ctypes.data_as(P_I64),
                          ctypes.byref(sc) if with_score else None,
                          ctypes.byref(sc_ell) if with_score else None)
    _ck(rc)
    return {"group": grp, "ell": t_ell, "L1": t_L1, "U2": t_U2, "L2": t_L2, "B": t_B,
            "evals": t_ev, "score": sc.value, "score_ell": sc_ell.value}


def stochastic_sample(g, S, k: int, eta: float, seed: int, p: int) -> np.ndarray:
    """Vertices the stochastic greedy samples for addition p with group S."""
    Sb, sl = _grp(S)
    out = np.zeros(g.n, dtype=np.int32)
    m = _load().or_sample(g.n, Sb.ctypes.data_as(P_I32), sl, k, eta, seed, p,
                          out.ctypes.data_as(P_I32))
    if m < 0:
        raise ValueError("oracle error (out of memory)")
    return out[:m].copy()
