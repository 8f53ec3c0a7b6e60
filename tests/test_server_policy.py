"""The request server's admission, queue limits, deadlines and cancellation
(server_policy.h), driven on the CPU: the policy is built with g++ into a
small shared library and run against a fake executor -- a discrete-event
loop with simulated request durations and a clock -- in place of the GPU."""
import ctypes
import heapq
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OK, BUSY, NOMEM, ARG, CANCELLED, DEADLINE = 0, -8, -6, -1, -10, -11


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("policy") / "libpolicy.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-Wall",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1910_13874_amd", "csrc"),
                    os.path.join(ROOT, "tests", "policy_shim.cpp"), "-o", out], check=True)
    L = ctypes.CDLL(out)
    u64, i32, f64, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sigs = {"pol_new": (vp, [ctypes.c_int64, ctypes.c_int64]), "pol_free": (None, [vp]),
            "pol_add_lane": (i32, [vp, u64]), "pol_set_held": (None, [vp, i32, u64]),
            "pol_submit": (i32, [vp, u64, i32, i32, u64, f64]),
            "pol_greedy_fits": (i32, [vp, u64]), "pol_start": (None, [vp, u64]),
            "pol_finish": (i32, [vp, u64, u64]), "pol_request_stop": (i32, [vp, u64, i32]),
            "pol_set_deadline": (i32, [vp, u64, f64]), "pol_expire": (None, [vp, f64]),
            "pol_take_dropped": (i32, [vp, ctypes.POINTER(u64), i32]),
            "pol_stop_status": (i32, [vp, u64]), "pol_stat": (ctypes.c_int64, [vp, i32]),
            "pol_held": (u64, [vp, i32])}
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    return L


class Pol:
    def __init__(self, lib, budget, max_queue):
        self.L, self.p = lib, lib.pol_new(budget, max_queue)

    def __getattr__(self, name):
        f = getattr(self.L, "pol_" + name)
        return lambda *a: f(self.p, *a)

    def stats(self):
        return {k: self.L.pol_stat(self.p, i) for i, k in
                enumerate(["waiting", "admitted", "completed", "rejected", "peak", "in_use"])}

    def dropped(self):
        buf = (ctypes.c_uint64 * 256)()
        m = self.L.pol_take_dropped(self.p, buf, 256)
        return [buf[i] for i in range(m)]

    def close(self):
        self.L.pol_free(self.p)


def test_queue_limit(lib):
    p = Pol(lib, 1 << 30, 3)
    assert [p.submit(i, 0, 0, 0, 0.0) for i in (1, 2, 3)] == [OK] * 3
    assert p.submit(4, 0, 0, 0, 0.0) == BUSY          # three waiting
    p.start(1)
    assert p.submit(4, 0, 0, 0, 0.0) == OK            # one left the queue
    assert p.stats()["waiting"] == 3 and p.stats()["admitted"] == 4
    for i in (1, 2, 3, 4):
        if i != 1:
            p.start(i)
        p.finish(i, 0)
    assert p.stats()["completed"] == 4 and p.stats()["waiting"] == 0
    p.close()


def test_budget_counts_held_greedy_memory(lib):
    """Budget 1000: a lane of 300; greedy footprints beyond what can ever fit
    are rejected at submission; a running greedy's reservation blocks a second
    one; the memory a finished greedy leaves with its graph stays counted,
    and a later request on that graph reserves only what it may add."""
    p = Pol(lib, 1000, 100)
    assert p.add_lane(300) == OK
    assert p.add_lane(800) == NOMEM
    assert p.submit(1, 1, 0, 800, 0.0) == NOMEM and p.stats()["rejected"] == 1
    assert p.submit(2, 1, 0, 600, 0.0) == OK and p.greedy_fits(2)
    p.start(2)
    assert p.stats()["in_use"] == 900
    assert p.submit(3, 1, 1, 600, 0.0) == OK           # could fit once the first is done
    assert not p.greedy_fits(3)                        # 300 + 600 + 600 > 1000
    p.finish(2, 500)                                   # graph 0 keeps 500 bytes
    assert p.held(0) == 500 and p.stats()["in_use"] == 800
    assert not p.greedy_fits(3)                        # 800 + 600 > 1000: graph 0 holds 500
    assert p.submit(4, 1, 0, 600, 0.0) == OK and p.greedy_fits(4)  # adds at most 100
    p.start(4)
    assert p.stats()["in_use"] == 900
    p.finish(4, 560)
    assert p.held(0) == 560 and p.stats()["peak"] <= 1000
    p.close()


def test_cancel_and_deadline(lib):
    p = Pol(lib, 1 << 30, 100)
    for i, kind in ((1, 0), (2, 0), (3, 1), (4, 1), (5, 0)):
        assert p.submit(i, kind, 0, 10, 0.0) == OK
    p.start(1)                                         # a score on the device
    p.start(3)                                         # a running greedy
    assert p.request_stop(1, CANCELLED) == BUSY        # completes normally
    assert p.request_stop(2, CANCELLED) == OK          # waiting: dropped
    assert p.request_stop(3, CANCELLED) == OK          # running greedy: stops at its next round
    assert p.stop_status(3) == CANCELLED
    assert p.request_stop(99, CANCELLED) == ARG
    assert p.dropped() == [2]
    assert p.finish(2, 0) == CANCELLED
    assert p.set_deadline(4, 1000.0) == OK and p.set_deadline(5, 2000.0) == OK
    assert p.set_deadline(1, 500.0) == OK              # a running score is never stopped
    p.expire(999.0)
    assert p.dropped() == []
    p.expire(1500.0)
    assert p.dropped() == [4] and p.stop_status(4) == DEADLINE and p.stop_status(1) == 0
    p.start(5)                                         # a running score passes its deadline
    p.expire(2500.0)
    assert p.stop_status(5) == 0
    assert p.finish(4, 0) == DEADLINE and p.finish(3, 0) == CANCELLED
    assert p.finish(1, 0) == 0 and p.finish(5, 0) == 0
    assert p.set_deadline(4, 1.0) == ARG               # finished
    s = p.stats()
    assert s["completed"] == 5 and s["waiting"] == 0
    p.close()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fake_executor_never_exceeds_budget(lib, seed):
    """A request stream run by a fake executor (2 greedy workers, one device
    for scores, simulated durations, random cancellations and deadlines): the
    bytes in use never pass the budget, the queue never holds more than its
    limit, every admitted request completes exactly once with a status that
    matches what happened to it, and a cancelled or expired request never
    finishes as OK unless it was a score already on the device."""
    rng = np.random.default_rng(seed)
    budget, max_queue, workers = 10_000, 40, 2
    p = Pol(lib, budget, max_queue)
    assert p.add_lane(2_000) == OK and p.add_lane(1_500) == OK
    now, next_id = 0.0, 1
    waiting_scores, waiting_greedy = [], []
    running = {}          # id -> (kind, graph, footprint)
    events = []           # (time, id) of running requests' ends
    outcome = {}
    admitted = busy = nomem = 0
    for step in range(3000):
        now += float(rng.exponential(10.0))
        # arrivals
        kind = int(rng.random() < 0.3)
        graph = int(rng.integers(0, 2))
        fp = int(rng.integers(500, 7_000)) if kind else 0
        dl = now + float(rng.exponential(200.0)) if rng.random() < 0.3 else 0.0
        rc = p.submit(next_id, kind, graph, fp, dl)
        if rc == OK:
            (waiting_greedy if kind else waiting_scores).append((next_id, graph, fp))
            admitted += 1
        elif rc == BUSY:
            busy += 1
            assert p.stats()["waiting"] >= max_queue
        else:
            assert rc == NOMEM and kind == 1
            nomem += 1
        next_id += 1
        # random cancellations
        if rng.random() < 0.05 and next_id > 2:
            p.request_stop(int(rng.integers(1, next_id)), CANCELLED)
        p.expire(now)
        for rid in p.dropped():           # the scheduler removes them from its queues
            for q in (waiting_scores, waiting_greedy):
                for e in q:
                    if e[0] == rid:
                        q.remove(e)
                        st = p.finish(rid, 0)
                        assert st in (CANCELLED, DEADLINE)
                        outcome[rid] = st
                        break
        # finished work
        while events and events[0][0] <= now:
            _, rid = heapq.heappop(events)
            kind, graph, fp = running.pop(rid)
            st = p.stop_status(rid)
            if kind == 1:
                # the run grows its graph's memory by at most what it reserved
                # (the footprint estimate bounds the allocations)
                extra = max(0, fp - p.held(graph))
                r = p.finish(rid, p.held(graph) + int(rng.integers(0, extra + 1)))
                outcome[rid] = st if st else OK
                assert r == st
            else:
                assert st == 0                 # scores on the device are never stopped
                p.finish(rid, 0)
                outcome[rid] = OK
        # a running greedy asked to stop ends at its next round
        for rid, (kind, graph, end) in list(running.items()):
            if kind == 1 and p.stop_status(rid):
                events = [(t, i) for (t, i) in events if i != rid]
                heapq.heapify(events)
                running.pop(rid)
                st = p.finish(rid, p.held(graph))
                outcome[rid] = st
        # start work: scores one at a time, greedy on free workers in order
        if waiting_scores and not any(k == 0 for k, _, _ in running.values()):
            rid, graph, _ = waiting_scores.pop(0)
            p.start(rid)
            running[rid] = (0, graph, 0)
            heapq.heappush(events, (now + 5.0, rid))
        while (waiting_greedy and sum(k == 1 for k, _, _ in running.values()) < workers
               and p.greedy_fits(waiting_greedy[0][0])):
            rid, graph, fp = waiting_greedy.pop(0)
            p.start(rid)
            end = now + float(rng.exponential(150.0))
            running[rid] = (1, graph, fp)
            heapq.heappush(events, (end, rid))
        s = p.stats()
        assert s["in_use"] <= budget and s["peak"] <= budget
        assert s["waiting"] <= max_queue
    # drain
    for rid in [e[0] for e in waiting_scores + waiting_greedy]:
        p.request_stop(rid, CANCELLED)
    for rid in p.dropped():
        outcome[rid] = p.finish(rid, 0)
    for rid, (kind, graph, _) in list(running.items()):
        st = p.stop_status(rid)
        outcome[rid] = p.finish(rid, p.held(graph)) or OK
    s = p.stats()
    assert s["completed"] == admitted == len(outcome) and s["waiting"] == 0
    assert busy > 0 and nomem > 0 and any(v in (CANCELLED, DEADLINE) for v in outcome.values())
    p.close()


def test_native_server_abi_on_cpu():
    """The native server's request bookkeeping entry points need no device:
    a server with no graphs refuses bad requests and unknown ids."""
    from paper_1910_13874_amd import ged
    srv = ged.Server(hbm_budget_bytes=1 << 20, max_queue=4)
    assert srv.cancel(12345) == ARG
    assert srv.set_deadline(12345, 1.0) == ARG
    with pytest.raises(ged.GedError) as e:
        srv.submit_score(0, [0])
    assert e.value.code == ARG
    assert srv.stats()["admitted"] == 0
    srv.close()
