"""Seeded synthetic inputs: ER / BA / R-MAT graphs as CSR and random groups.

This module carries none of the walk-count arithmetic; it only generates
inputs.  The generators are C code (``graphgen.c``) with published RNG
definitions, so a seed gives the same graph on every machine.  Both the CPU
oracle tests and the GPU path take their inputs from here.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


class _CSR(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col_idx", ctypes.POINTER(ctypes.c_int32)),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing: run __graft_entry__.build() to compile the input generators")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    lib.gg_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P(_CSR)]
    lib.gg_ba.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, P(_CSR)]
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, P(_CSR)]
    lib.gg_from_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, P(ctypes.c_int32),
                                  P(ctypes.c_int32), ctypes.c_int, ctypes.c_int, P(_CSR)]
    lib.gg_free.argtypes = [P(_CSR)]
    lib.gg_groups.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_uint64, P(ctypes.c_int64), P(ctypes.c_int32)]
    lib.gg_uniform_ints.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                    P(ctypes.c_int64)]
    lib.gg_uniform_doubles.argtypes = [ctypes.c_int64, ctypes.c_uint64, P(ctypes.c_double)]
    for f in ("gg_er", "gg_ba", "gg_rmat", "gg_from_edges", "gg_groups", "gg_uniform_ints",
              "gg_uniform_doubles"):
        getattr(lib, f).restype = ctypes.c_int
    lib.gg_free.restype = None
    _lib = lib
    return lib


@dataclass
class Graph:
    """A graph in CSR form.

    Row ``v`` lists the in-neighbours ``u`` of ``v`` (arcs ``u -> v``).  For an
    undirected graph every edge is two arcs, so rows are plain neighbour lists.
    """

    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    name: str = ""
    directed: bool = False

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    @property
    def max_degree(self) -> int:
        return int(self.degrees.max()) if self.n > 0 else 0

    def default_alpha(self) -> float:
        """alpha = 1/(max degree + 1), the setting every workload here uses."""
        return 1.0 / (self.max_degree + 1)

    def fingerprint(self) -> str:
        import hashlib
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr).tobytes())
        h.update(np.ascontiguousarray(self.col_idx).tobytes())
        return h.hexdigest()[:16]


def _take(csr: _CSR, name: str) -> Graph:
    lib = _load()
    n, nnz = csr.n, csr.nnz
    rp = np.ctypeslib.as_array(csr.row_ptr, shape=(n + 1,)).copy()
    ci = (np.ctypeslib.as_array(csr.col_idx, shape=(nnz,)).copy() if nnz > 0
          else np.zeros(0, dtype=np.int32))
    lib.gg_free(ctypes.byref(csr))
    return Graph(n=int(n), row_ptr=rp, col_idx=ci, name=name)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


def erdos_renyi(n: int, m_edges: int, seed: int) -> Graph:
    """G(n, M): ``m_edges`` distinct uniform non-loop undirected edges."""
    csr = _CSR()
    _check(_load().gg_er(n, m_edges, seed, ctypes.byref(csr)), "gg_er")
    return _take(csr, f"er_n{n}_m{m_edges}_s{seed}")


def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    """Preferential attachment, ``m`` distinct targets per new vertex."""
    csr = _CSR()
    _check(_load().gg_ba(n, m, seed, ctypes.byref(csr)), "gg_ba")
    return _take(csr, f"ba_n{n}_m{m}_s{seed}")


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 4) -> Graph:
    """R-MAT, symmetrized and deduplicated, isolated vertices kept."""
    csr = _CSR()
    _check(_load().gg_rmat(scale, edge_factor, a, b, c, seed, ctypes.byref(csr)), "gg_rmat")
    return _take(csr, f"rmat_s{scale}_ef{edge_factor}_s{seed}")


def from_edges(n: int, src, dst, symmetrize: bool = True, name: str = "edges") -> Graph:
    """CSR from an explicit edge list (self-loops and duplicates dropped).

    ``symmetrize=False`` makes a directed graph stored by in-neighbours: row v
    lists every u with an arc u -> v.
    """
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    csr = _CSR()
    P = ctypes.POINTER(ctypes.c_int32)
    rc = _load().gg_from_edges(n, src.size, src.ctypes.data_as(P), dst.ctypes.data_as(P),
                               1 if symmetrize else 0, 0 if symmetrize else 1, ctypes.byref(csr))
    _check(rc, "gg_from_edges")
    g = _take(csr, name)
    g.directed = not symmetrize
    return g


def reverse(g: Graph) -> Graph:
    """The reverse graph (rows list out-neighbours of the original)."""
    src = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.row_ptr))
    # arcs of g are col_idx[j] -> row(j); reversed arcs are row(j) -> col_idx[j]
    r = from_edges(g.n, src, g.col_idx, symmetrize=False, name=g.name + "_rev")
    r.directed = g.directed
    return r


def groups(n: int, n_groups: int, smin: int, smax: int, seed: int):
    """``n_groups`` groups, sizes uniform in [smin, smax], members distinct uniform.

    Returns (offsets int64[n_groups+1], members int32[sum sizes]); each group is
    sorted.
    """
    offsets = np.zeros(n_groups + 1, dtype=np.int64)
    members = np.zeros(max(1, n_groups * smax), dtype=np.int32)
    rc = _load().gg_groups(n, n_groups, smin, smax, seed,
                           offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           members.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    _check(rc, "gg_groups")
    return offsets, members[: offsets[-1]].copy()


def group(n: int, size: int, seed: int) -> np.ndarray:
    """One group of ``size`` distinct uniform vertices (sorted)."""
    _, m = groups(n, 1, size, size, seed)
    return m


def uniform_ints(count: int, hi: int, seed: int) -> np.ndarray:
    out = np.zeros(max(1, count), dtype=np.int64)
    _check(_load().gg_uniform_ints(count, hi, seed,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
           "gg_uniform_ints")
    return out[:count]


def uniform_doubles(count: int, seed: int) -> np.ndarray:
    out = np.zeros(max(1, count), dtype=np.float64)
    _check(_load().gg_uniform_doubles(count, seed,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "gg_uniform_doubles")
    return out[:count]


# Named workloads (sizes of the configurations the benchmarks and tests use).
def workload_graph(name: str) -> Graph:
    """Construct one of the named synthetic graphs.

    er1k    : ER n=1,000, 5,000 edges (average degree 10), seed 1
    ba1m    : BA n=1,000,000, m=5, seed 2
    ba2m    : BA n=2,000,000, m=8, seed 3
    rmat22  : R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), seed 4
    plus smaller variants used by the tests and the serving mix.
    """
    table = {
        "er1k": lambda: erdos_renyi(1000, 5000, 1),
        "ba1m": lambda: barabasi_albert(1_000_000, 5, 2),
        "ba2m": lambda: barabasi_albert(2_000_000, 8, 3),
        "rmat22": lambda: rmat(22, 16, seed=4),
        "er10k": lambda: erdos_renyi(10_000, 40_000, 11),
        "er100k": lambda: erdos_renyi(100_000, 800_000, 12),
        "ba100k": lambda: barabasi_albert(100_000, 4, 13),
        "ba1m_m8": lambda: barabasi_albert(1_000_000, 8, 14),
        "ba2m_m16": lambda: barabasi_albert(2_000_000, 16, 15),
        "rmat17": lambda: rmat(17, 8, seed=16),
        "rmat20": lambda: rmat(20, 16, seed=17),
        "rmat16": lambda: rmat(16, 16, seed=18),
        "ba50k": lambda: barabasi_albert(50_000, 5, 19),
        "er20k": lambda: erdos_renyi(20_000, 100_000, 20),
    }
    if name not in table:
        raise KeyError(f"unknown workload graph {name!r}; known: {sorted(table)}")
    g = table[name]()
    g.name = name
    return g
