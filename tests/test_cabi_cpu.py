"""CPU checks of the boundary: the HIP library loads without a GPU and exports
every function include/ged.h declares; bench.py refuses more than one GPU."""
import ast
import ctypes
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ged.h")
LIB = os.path.join(ROOT, "paper_1910_13874_amd", "libged_hip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ged_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("ged_graph_create", "ged_score", "ged_score_batch", "ged_greedy",
                 "ged_server_create", "ged_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ged_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_binding_loads_one_hip_runtime():
    """Importing the binding alone (torch not imported yet) leaves one HIP
    runtime in the process: torch's copy, which the library binds to."""
    code = ("import re; from paper_1910_13874_amd import ged; "
            "maps = open('/proc/self/maps').read(); "
            "print(sorted(set(re.findall(r'\\S*libamdhip64\\S*', maps))))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         check=True).stdout.strip()
    paths = ast.literal_eval(out)
    assert len(paths) == 1, paths
    try:
        import torch
    except ImportError:
        return
    assert paths[0].startswith(os.path.dirname(torch.__file__)), paths


def test_error_paths_without_gpu_work():
    lib = ctypes.CDLL(LIB)
    lib.ged_last_error.restype = ctypes.c_char_p
    lib.ged_graph_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    rp = np.array([0, 1, 1], dtype=np.int64)
    ci = np.array([1], dtype=np.int32)
    # asymmetric arc set with GED_UNDIRECTED is rejected during host validation
    rc = lib.ged_graph_create(ctypes.c_int64(2), ctypes.c_int64(1),
                              rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              ctypes.c_uint32(1), ctypes.byref(out))
    assert rc == -5 and b"symmetric" in lib.ged_last_error()
    rc = lib.ged_graph_create(ctypes.c_int64(2), ctypes.c_int64(1),
                              rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              ctypes.c_uint32(7), ctypes.byref(out))
    assert rc == -1
    lib.ged_graph_destroy.restype = ctypes.c_int
    assert lib.ged_graph_destroy(None) == 0


def test_bench_refuses_multi_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_request_stream_is_seeded():
    from paper_1910_13874_amd import serve
    ns = [1000, 5000]
    a = serve.make_requests(ns, 500, 1000.0, seed=3)
    b = serve.make_requests(ns, 500, 1000.0, seed=3)
    assert [q["t"] for q in a] == [q["t"] for q in b]
    assert all(np.array_equal(x.get("S", []), y.get("S", [])) for x, y in zip(a, b))
    frac = sum(q["kind"] for q in a) / len(a)
    assert 0.05 < frac < 0.15
    sizes = [len(q["S"]) for q in a if q["kind"] == 0]
    assert min(sizes) >= 1 and max(sizes) <= 100
    assert all(q["k"] in (5, 20, 100) for q in a if q["kind"] == 1)
    t = np.array([q["t"] for q in a])
    assert np.all(np.diff(t) >= 0) and 0.3 < t[-1] < 0.7  # 500 arrivals at 1000/s


def test_plain_loop_clock():
    """The one-at-a-time loop queues requests FIFO on a clock fed by service times."""
    from paper_1910_13874_amd import serve

    class Fake:
        def score(self, S, a, e):
            return float(len(S))

        def greedy(self, k, a, e):
            return {"group": list(range(k))}

    reqs = [{"t": 0.0, "g": 0, "kind": 0, "S": [1]}, {"t": 0.0, "g": 0, "kind": 0, "S": [1, 2]},
            {"t": 10.0, "g": 0, "kind": 1, "k": 2}]
    lat, res, clock, busy = serve.run_plain([Fake()], [0.1], reqs, 1e-4)
    assert res[0] == 1.0 and res[1] == 2.0 and res[2]["group"] == [0, 1]
    assert lat[1] >= lat[0] and clock >= 10.0 and lat[2] < 1.0
