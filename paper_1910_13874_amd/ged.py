"""Python binding of the GED-Walk HIP library (``libged_hip.so``, C ABI in
``include/ged.h``).

Argument marshalling only: every step of scoring and maximisation runs in the
library's HIP kernels.  If the library is missing this module raises at import
time -- there is no CPU fallback.  PyTorch is used only to hand the library a
HIP stream (``GedGraph.set_stream``).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libged_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(the GED-Walk path has no CPU fallback)")

# The library links libamdhip64.so.7, and PyTorch-ROCm ships its own copy of
# the HIP runtime under that soname.  With torch loaded first the library binds
# to torch's copy and the process holds one HIP runtime; loaded first, it would
# bring in the system copy and torch would then add its own, and two runtimes
# in one process do not share the device.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

P_I64 = ctypes.POINTER(ctypes.c_int64)
P_I32 = ctypes.POINTER(ctypes.c_int32)
P_F64 = ctypes.POINTER(ctypes.c_double)
c_graph_p = ctypes.c_void_p

GED_UNDIRECTED = 1
GED_DIRECTED = 2
GED_KEEP_ORDER = 8
GED_BOUND_COMBINATORIAL = 0
GED_BOUND_SPECTRAL = 1

STATUS = {0: "ok", -1: "bad argument", -2: "vertex out of range", -3: "alpha out of range",
          -4: "eps out of range", -5: "malformed graph", -6: "out of memory",
          -7: "device error", -8: "busy", -9: "walk length limit", -10: "cancelled",
          -11: "deadline passed"}


class ScoreInfo(ctypes.Structure):
    _fields_ = [("ell", ctypes.c_int32), ("bound", ctypes.c_double),
                ("walk_total", ctypes.c_double)]


class GreedyTrace(ctypes.Structure):
    _fields_ = [("ell", P_I32), ("L1", P_F64), ("U2", P_F64), ("L2", P_F64), ("B", P_F64),
                ("evals", P_I64), ("forced", P_I32), ("n_forced", ctypes.c_int32),
                ("forced_ell", ctypes.c_int32), ("score_ell", ctypes.c_int32),
                ("n_rounds", ctypes.c_int32)]


class PartitionCounts(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("n_grid2", ctypes.c_int32),
                ("n_segs", ctypes.c_int32), ("n_long", ctypes.c_int32),
                ("cut", ctypes.c_int32), ("bucketed", ctypes.c_int32),
                ("bucket_rows", ctypes.c_int64), ("bk_arcs", ctypes.c_int64)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("edges", ctypes.c_double),
                ("dominant_launches", ctypes.c_int64), ("dominant_ms", ctypes.c_double),
                ("dominant_bytes", ctypes.c_double), ("dominant_columns", ctypes.c_int32),
                ("dominant_kind", ctypes.c_int32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ged_graph_create", ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, P_I64, P_I32,
                                        ctypes.c_uint32, ctypes.POINTER(c_graph_p)])
_sig("ged_graph_create_weighted", ctypes.c_int,
     [ctypes.c_int64, ctypes.c_int64, P_I64, P_I32, P_F64, ctypes.c_uint32,
      ctypes.POINTER(c_graph_p)])
_sig("ged_graph_destroy", ctypes.c_int, [c_graph_p])
_sig("ged_graph_info", ctypes.c_int, [c_graph_p, P_I64, P_I64, P_I32])
_sig("ged_default_alpha", ctypes.c_double, [c_graph_p])
_sig("ged_set_stream", ctypes.c_int, [c_graph_p, ctypes.c_void_p])
_sig("ged_prepare", ctypes.c_int, [c_graph_p, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(ScoreInfo)])
_sig("ged_invalidate", ctypes.c_int, [c_graph_p])
_sig("ged_set_tail_bound", ctypes.c_int, [c_graph_p, ctypes.c_int32])
_sig("ged_sigma_max", ctypes.c_int, [c_graph_p, P_F64])
_sig("ged_score", ctypes.c_int, [c_graph_p, P_I32, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double, P_F64, ctypes.POINTER(ScoreInfo)])
_sig("ged_score_batch", ctypes.c_int, [c_graph_p, P_I64, P_I32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_double, P_F64])
_sig("ged_batch_tile", ctypes.c_int32, [c_graph_p])
_sig("ged_set_batch_tile", ctypes.c_int, [c_graph_p, ctypes.c_int32])
_sig("ged_set_source_buckets", ctypes.c_int, [c_graph_p, ctypes.c_int64])
_sig("ged_source_buckets", ctypes.c_int64, [c_graph_p])
_sig("ged_partition_plan", ctypes.c_int,
     [P_I32, P_I32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
      ctypes.POINTER(PartitionCounts), P_I32, P_I32, P_I32, P_I32, P_I32, P_I32, P_I32])
_sig("ged_set_batch_row_cut", ctypes.c_int, [c_graph_p, ctypes.c_int32])
_sig("ged_batch_row_cut", ctypes.c_int32, [c_graph_p])
_sig("ged_set_greedy_width", ctypes.c_int, [c_graph_p, ctypes.c_int32])
_sig("ged_set_count16", ctypes.c_int, [c_graph_p, ctypes.c_int32])
_sig("ged_count16_hub", ctypes.c_int32, [c_graph_p])
_sig("ged_greedy_width", ctypes.c_int32, [c_graph_p])
_sig("ged_greedy_footprint", ctypes.c_int, [c_graph_p, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_double, P_I64, P_I64])
_sig("ged_greedy", ctypes.c_int, [c_graph_p, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  P_I32, P_F64, ctypes.POINTER(GreedyTrace)])
_sig("ged_greedy_stochastic", ctypes.c_int,
     [c_graph_p, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
      ctypes.c_uint64, P_I32, P_F64, ctypes.POINTER(GreedyTrace)])
_sig("ged_profile_enable", ctypes.c_int, [c_graph_p, ctypes.c_int])
_sig("ged_profile_read", ctypes.c_int, [c_graph_p, ctypes.POINTER(Profile)])
_sig("ged_last_error", ctypes.c_char_p, [])


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("score_slots", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("greedy_workers", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("kind", ctypes.c_int32), ("status", ctypes.c_int32),
                ("score", ctypes.c_double), ("k", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("t_submit_us", ctypes.c_double), ("t_done_us", ctypes.c_double)]


c_server_p = ctypes.c_void_p
_sig("ged_server_create", ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(c_server_p)])
_sig("ged_server_add_graph", ctypes.c_int, [c_server_p, c_graph_p, ctypes.c_double,
                                            ctypes.c_double, P_I32])
_sig("ged_server_submit_score", ctypes.c_int, [c_server_p, ctypes.c_int32, P_I32, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_uint64)])
_sig("ged_server_submit_greedy", ctypes.c_int, [c_server_p, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_uint64)])
_sig("ged_server_poll", ctypes.c_int, [c_server_p, ctypes.POINTER(Result), ctypes.c_int32, P_I32,
                                       ctypes.c_int64])
_sig("ged_server_group", ctypes.c_int, [c_server_p, ctypes.c_uint64, P_I32, ctypes.c_int32])
_sig("ged_server_stats", ctypes.c_int, [c_server_p, P_I64])
_sig("ged_server_cancel", ctypes.c_int, [c_server_p, ctypes.c_uint64])
_sig("ged_server_set_deadline", ctypes.c_int, [c_server_p, ctypes.c_uint64, ctypes.c_double])
_sig("ged_server_destroy", ctypes.c_int, [c_server_p])


class GedError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.ged_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


def _ck(rc, where):
    if rc != 0:
        raise GedError(rc, where)


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
    return a, a.ctypes.data_as(P_I32)


class GedGraph:
    """A graph resident on the GPU (CSR copied at construction)."""

    def __init__(self, n, row_ptr, col_idx, directed=False, weights=None, keep_order=False):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        if ci.size == 0:
            ci = np.zeros(1, dtype=np.int32)
        h = c_graph_p()
        flags = GED_DIRECTED if directed else GED_UNDIRECTED
        if keep_order:
            flags |= GED_KEEP_ORDER
        nnz = int(rp[-1])
        if weights is None:
            rc = _lib.ged_graph_create(n, nnz, rp.ctypes.data_as(P_I64), ci.ctypes.data_as(P_I32),
                                       flags, ctypes.byref(h))
        else:
            w = np.ascontiguousarray(weights, dtype=np.float64)
            rc = _lib.ged_graph_create_weighted(n, nnz, rp.ctypes.data_as(P_I64),
                                                ci.ctypes.data_as(P_I32),
                                                w.ctypes.data_as(P_F64), flags, ctypes.byref(h))
        _ck(rc, "ged_graph_create")
        self._h = h
        self.n = int(n)
        self.nnz = nnz
        self.directed = directed
        self.weighted = weights is not None

    @classmethod
    def from_graph(cls, g, weights=None, keep_order=False):
        return cls(g.n, g.row_ptr, g.col_idx, directed=getattr(g, "directed", False),
                   weights=weights, keep_order=keep_order)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("graph handle closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.ged_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        md = ctypes.c_int32()
        _ck(_lib.ged_graph_info(self.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(md)),
            "ged_graph_info")
        return n.value, nnz.value, md.value

    @property
    def max_degree(self):
        return self.info()[2]

    def default_alpha(self):
        return _lib.ged_default_alpha(self.handle)

    def set_stream(self, stream=None):
        """Launch on a torch.cuda.Stream (or raw hipStream_t int); None = own stream."""
        if stream is None:
            ptr = None
        elif isinstance(stream, int):
            ptr = stream
        else:
            ptr = stream.cuda_stream
        _ck(_lib.ged_set_stream(self.handle, ctypes.c_void_p(ptr) if ptr else None),
            "ged_set_stream")

    def _alpha(self, alpha):
        return self.default_alpha() if alpha is None else float(alpha)

    def prepare(self, alpha=None, eps=1e-4):
        info = ScoreInfo()
        _ck(_lib.ged_prepare(self.handle, self._alpha(alpha), eps, ctypes.byref(info)),
            "ged_prepare")
        return info.ell, info.bound, info.walk_total

    def invalidate(self):
        """Drop the cached per-(alpha, eps) precomputation."""
        _ck(_lib.ged_invalidate(self.handle), "ged_invalidate")

    def set_tail_bound(self, kind):
        """"combinatorial" (Eq. comb-bound, the default) or "spectral"
        (Lemma spectral-bound, valid for alpha < 1/sigma_max)."""
        code = {"combinatorial": GED_BOUND_COMBINATORIAL, "spectral": GED_BOUND_SPECTRAL}[kind]
        _ck(_lib.ged_set_tail_bound(self.handle, code), "ged_set_tail_bound")

    def sigma_max(self):
        """Upper estimate of the largest singular value of the adjacency matrix."""
        out = ctypes.c_double()
        _ck(_lib.ged_sigma_max(self.handle, ctypes.byref(out)), "ged_sigma_max")
        return out.value

    def score(self, S, alpha=None, eps=1e-4, with_info=False):
        arr, ptr = _i32(S)
        out = ctypes.c_double()
        info = ScoreInfo()
        _ck(_lib.ged_score(self.handle, ptr if arr.size else None, arr.size, self._alpha(alpha),
                           eps, ctypes.byref(out), ctypes.byref(info)), "ged_score")
        if with_info:
            return out.value, info.ell, info.bound
        return out.value

    def score_batch(self, offsets, members, alpha=None, eps=1e-4):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        mem = np.ascontiguousarray(members, dtype=np.int32)
        G = off.size - 1
        out = np.zeros(max(G, 1))
        _ck(_lib.ged_score_batch(self.handle, off.ctypes.data_as(P_I64),
                                 mem.ctypes.data_as(P_I32) if mem.size else None, G,
                                 self._alpha(alpha), eps, out.ctypes.data_as(P_F64)),
            "ged_score_batch")
        return out[:G]

    def batch_tile(self):
        return _lib.ged_batch_tile(self.handle)

    def set_batch_tile(self, tile):
        """Fix the batched-scoring tile width (0 = autotune on the next call)."""
        _ck(_lib.ged_set_batch_tile(self.handle, int(tile)), "ged_set_batch_tile")

    def batch_row_cut(self):
        return _lib.ged_batch_row_cut(self.handle)

    def set_batch_row_cut(self, cut_div):
        """Row-split threshold divisor of batched tiles (1, 2, 4; 0 = autotune)."""
        _ck(_lib.ged_set_batch_row_cut(self.handle, int(cut_div)), "ged_set_batch_row_cut")

    def set_source_buckets(self, nbytes):
        """Source-bucket size of the long rows' pieces in bytes of gathered
        vector (0 = library's choice, < 0 = off); before the first step."""
        _ck(_lib.ged_set_source_buckets(self.handle, int(nbytes)), "ged_set_source_buckets")

    def source_buckets(self):
        return _lib.ged_source_buckets(self.handle)

    def set_count16(self, hub):
        """Level-2 counts of batch tiles in 16 bits below a hub cut (0 = library's
        choice, -1 = off, > 0 = this cut)."""
        _ck(_lib.ged_set_count16(self.handle, int(hub)), "ged_set_count16")

    def count16_hub(self):
        """Hub cut of the last batch's 16-bit level-2 counts, -1 if 32-bit."""
        return _lib.ged_count16_hub(self.handle)

    def set_greedy_width(self, width):
        """Candidates per gain SpMM of the greedy (2, 4, 8, 16; 0 = library's choice)."""
        _ck(_lib.ged_set_greedy_width(self.handle, int(width)), "ged_set_greedy_width")

    def greedy_width(self):
        return _lib.ged_greedy_width(self.handle)

    def greedy_footprint(self, k, alpha=None, eps=1e-4):
        """(upper bound of the greedy's device bytes for k picks, bytes its
        workspace holds now)."""
        est, held = ctypes.c_int64(), ctypes.c_int64()
        _ck(_lib.ged_greedy_footprint(self.handle, int(k), self._alpha(alpha), eps,
                                      ctypes.byref(est), ctypes.byref(held)),
            "ged_greedy_footprint")
        return est.value, held.value

    def _greedy(self, fn, k, alpha, eps, extra, forced, forced_ell, with_score):
        grp = np.zeros(k, dtype=np.int32)
        t_ell = np.zeros(k, dtype=np.int32)
        t_L1 = np.zeros(k)
        t_U2 = np.zeros(k)
        t_L2 = np.zeros(k)
        t_B = np.zeros(k)
        t_ev = np.zeros(k, dtype=np.int64)
        tr = GreedyTrace()
        tr.ell = t_ell.ctypes.data_as(P_I32)
        tr.L1 = t_L1.ctypes.data_as(P_F64)
        tr.U2 = t_U2.ctypes.data_as(P_F64)
        tr.L2 = t_L2.ctypes.data_as(P_F64)
        tr.B = t_B.ctypes.data_as(P_F64)
        tr.evals = t_ev.ctypes.data_as(P_I64)
        if forced is not None and len(forced):
            farr, fptr = _i32(forced)
            tr.forced = fptr
            tr.n_forced = farr.size
            tr.forced_ell = int(forced_ell)
        sc = ctypes.c_double(math.nan)
        rc = fn(self.handle, k, self._alpha(alpha), eps, *extra, grp.ctypes.data_as(P_I32),
                ctypes.byref(sc) if with_score else None, ctypes.byref(tr))
        _ck(rc, fn.__name__)
        return {"group": grp, "ell": t_ell, "L1": t_L1, "U2": t_U2, "L2": t_L2, "B": t_B,
                "evals": t_ev, "score": sc.value, "score_ell": tr.score_ell,
                "rounds": tr.n_rounds}

    def greedy(self, k, alpha=None, eps=1e-4, forced=None, forced_ell=1, with_score=True):
        """Greedy maximisation; returns group (pick order) and the per-pick trace."""
        return self._greedy(_lib.ged_greedy, k, alpha, eps, (), forced, forced_ell, with_score)

    def greedy_stochastic(self, k, alpha=None, eps=1e-4, eta=0.1, seed=1, forced=None,
                          forced_ell=1, with_score=True):
        return self._greedy(_lib.ged_greedy_stochastic, k, alpha, eps,
                            (ctypes.c_double(eta), ctypes.c_uint64(seed)), forced, forced_ell,
                            with_score)

    def profile_enable(self, on=True):
        _ck(_lib.ged_profile_enable(self.handle, 1 if on else 0), "ged_profile_enable")

    def profile_read(self):
        p = Profile()
        _ck(_lib.ged_profile_read(self.handle, ctypes.byref(p)), "ged_profile_read")
        return {f: getattr(p, f) for f, _ in Profile._fields_}


class Server:
    """Continuous-batching request server over resident graphs (C ABI ged_server_*)."""

    def __init__(self, hbm_budget_bytes=64 << 30, score_slots=0, max_queue=1 << 20,
                 greedy_workers=2):
        cfg = ServerConfig(int(hbm_budget_bytes), int(score_slots), int(max_queue),
                           int(greedy_workers))
        h = c_server_p()
        _ck(_lib.ged_server_create(ctypes.byref(cfg), ctypes.byref(h)), "ged_server_create")
        self._h = h
        self.graphs = []

    def add_graph(self, gg, alpha=None, eps=1e-4):
        gid = ctypes.c_int32()
        a = gg.default_alpha() if alpha is None else float(alpha)
        _ck(_lib.ged_server_add_graph(self._h, gg.handle, a, eps, ctypes.byref(gid)),
            "ged_server_add_graph")
        self.graphs.append(gg)
        return gid.value

    def submit_score(self, gid, S):
        arr, ptr = _i32(S)
        rid = ctypes.c_uint64()
        _ck(_lib.ged_server_submit_score(self._h, gid, ptr if arr.size else None, arr.size,
                                         ctypes.byref(rid)), "ged_server_submit_score")
        return rid.value

    def submit_greedy(self, gid, k):
        rid = ctypes.c_uint64()
        _ck(_lib.ged_server_submit_greedy(self._h, gid, int(k), ctypes.byref(rid)),
            "ged_server_submit_greedy")
        return rid.value

    def poll(self, max_results=1024, timeout_us=0):
        buf = (Result * max_results)()
        n = ctypes.c_int32()
        _ck(_lib.ged_server_poll(self._h, buf, max_results, ctypes.byref(n), int(timeout_us)),
            "ged_server_poll")
        return [buf[i] for i in range(n.value)]

    def cancel(self, rid):
        """Ask request rid to stop; returns the status code (0: it will complete
        cancelled; -8: a score already on the device; -1: unknown or done)."""
        return _lib.ged_server_cancel(self._h, int(rid))

    def set_deadline(self, rid, deadline_us):
        """Absolute deadline in the clock of Result.t_submit_us (0 removes it)."""
        return _lib.ged_server_set_deadline(self._h, int(rid), float(deadline_us))

    def group(self, rid, k):
        out = np.zeros(k, dtype=np.int32)
        _ck(_lib.ged_server_group(self._h, rid, out.ctypes.data_as(P_I32), k), "ged_server_group")
        return out

    def stats(self):
        out = np.zeros(6, dtype=np.int64)
        _ck(_lib.ged_server_stats(self._h, out.ctypes.data_as(P_I64)), "ged_server_stats")
        keys = ["admitted", "completed", "steps", "peak_bytes", "peak_columns", "rejected"]
        return dict(zip(keys, (int(x) for x in out)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.ged_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


IN_MODES = ["vec", "ones", "notmask", "mask", "tilemask", "onehot", "fresh", "cnt", "cnt32"]
OUT_MODES = ["plain", "inj", "zero", "tile", "gain", "pool", "combine", "combine32", "gaincomb",
             "tile32", "combine32l", "gain32", "gaincomb32l", "zero32", "gain32d", "gaincomb32s"]
KIND_BASE = 32  # a profile record's kind is input mode * KIND_BASE + output mode


def partition_plan(row_ptr, col_idx, n, units, cut_div=1, bucket_rows=0):
    """The step partition the library builds for a CSR (host-only call):
    dict of counts and int32 arrays (blocks and grid2 as (m, 4))."""
    rp = _i32(row_ptr)[0]
    ci = _i32(col_idx)[0] if col_idx is not None and len(col_idx) else np.zeros(1, np.int32)
    cnt = PartitionCounts()
    p = lambda a: a.ctypes.data_as(P_I32)
    null = ctypes.cast(None, P_I32)
    _ck(_lib.ged_partition_plan(p(rp), p(ci), int(n), int(units), int(cut_div), int(bucket_rows),
                                ctypes.byref(cnt), null, null, null, null, null, null, null),
        "ged_partition_plan")
    out = {f: getattr(cnt, f) for f, _ in PartitionCounts._fields_}
    arr = {"blocks": np.zeros(4 * max(1, cnt.n_blocks), np.int32),
           "grid2": np.zeros(4 * max(1, cnt.n_grid2), np.int32),
           "long_rows": np.zeros(max(1, cnt.n_long), np.int32),
           "long_first": np.zeros(cnt.n_long + 1, np.int32),
           "bk_ptr": np.zeros(cnt.n_segs + 1, np.int32),
           "bk_lsub": np.zeros(max(1, cnt.n_segs), np.int32),
           "bk_ci": np.zeros(max(1, cnt.bk_arcs), np.int32)}
    _ck(_lib.ged_partition_plan(p(rp), p(ci), int(n), int(units), int(cut_div), int(bucket_rows),
                                ctypes.byref(cnt), *[p(arr[k]) for k in
                                                     ("blocks", "grid2", "long_rows", "long_first",
                                                      "bk_ptr", "bk_lsub", "bk_ci")]),
        "ged_partition_plan")
    out["blocks"] = arr["blocks"][:4 * cnt.n_blocks].reshape(-1, 4)
    out["grid2"] = arr["grid2"][:4 * cnt.n_grid2].reshape(-1, 4)
    out["long_rows"] = arr["long_rows"][:cnt.n_long]
    out["long_first"] = arr["long_first"]
    if cnt.bucketed:
        out["bk_ptr"] = arr["bk_ptr"]
        out["bk_lsub"] = arr["bk_lsub"][:cnt.n_segs]
        out["bk_ci"] = arr["bk_ci"][:cnt.bk_arcs]
    return out


def kernel_name(columns, kind, weighted=False):
    """Symbol of the step-kernel instantiation a profile record refers to."""
    return (f"ged::k_step<{columns}, {kind // KIND_BASE}, {kind % KIND_BASE}, "
            f"{'true' if weighted else 'false'}>")


def exported_symbols():
    """Names of the C-ABI entry points this binding found in the library."""
    return [n for n in dir(_lib) if n.startswith("ged_")]
