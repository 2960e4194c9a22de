"""Serving loop (factor cache, memory admission, continuous batching) on the CPU.

A fake backend stands in for the device: factor bytes grow with n**2, workspace
with nrhs * n**2, and a solve returns u = 2 f after a short sleep.  The tests
check what the scheduler decides, not the numerics (the GPU serving test checks
those)."""
import threading
import time

import numpy as np
import pytest

import workloads
from paper_1504_04058_amd.serve import Backend, Request, Server


class FakeBackend(Backend):
    def __init__(self, solve_s=0.01, create_s=0.005):
        self.solve_s, self.create_s = solve_s, create_s
        self.live = {}
        self.created, self.destroyed = [], []
        self.lock = threading.Lock()
        self.concurrent = 0
        self.max_concurrent = 0

    def factor_bytes(self, req):
        return 100 * req.n * req.n

    def workspace_bytes(self, req, nrhs):
        return 10 * nrhs * req.n * req.n

    def create(self, req):
        time.sleep(self.create_s)
        with self.lock:
            h = (req.key, len(self.created))
            self.created.append(req.key)
            self.live[h] = True
        return h

    def solve(self, handle, f):
        assert self.live.get(handle), "solve on a destroyed plan"
        with self.lock:
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
        time.sleep(self.solve_s)
        with self.lock:
            self.concurrent -= 1
        k = f.shape[0]
        return 2 * f, np.full(k, 3, np.int32), np.full(k, 1e-7), "ASP_OK"

    def destroy(self, handle):
        with self.lock:
            assert self.live.pop(handle)
            self.destroyed.append(handle[0])


def req(rid, key_n, arrival, nrhs=1, key_tag=0):
    n = key_n
    f = np.full((nrhs, n * n), rid + 1, dtype=np.complex128)
    return Request(rid, (2, n, key_tag), arrival, 2, n, 1.0, nrhs, np.ones((n, n)), f)


def test_all_complete_and_results_match_requests():
    be = FakeBackend()
    reqs = [req(i, 8 + 4 * (i % 3), 0.001 * i, nrhs=1 + i % 4) for i in range(40)]
    res, summ = Server(be, budget_bytes=10 ** 9, realtime=True).run(reqs)
    assert summ["completed"] == 40 and summ["failed"] == 0
    assert summ["solves"] == sum(r.nrhs for r in reqs)
    for r, q in zip(res, reqs):
        assert r.rid == q.rid and r.status == "ASP_OK"
        assert np.array_equal(r.u, 2 * q.f)           # each slice routed back to its request
        assert r.done >= r.start >= r.arrival - 1e-9
    assert be.live == {}                              # everything released at the end


def test_factor_cache_reuse():
    be = FakeBackend()
    reqs = [req(i, 16, 0.002 * i) for i in range(20)]
    res, summ = Server(be, budget_bytes=10 ** 9).run(reqs)
    assert summ["factorizations"] == 1 and len(be.created) == 1
    assert sum(r.cache_hit for r in res) == 19


def test_continuous_batching_joins_waiting_requests():
    be = FakeBackend(solve_s=0.05)
    # one key; requests arrive while the first solve runs
    reqs = [req(i, 16, 0.0 if i == 0 else 0.01 + 0.001 * i) for i in range(10)]
    srv = Server(be, budget_bytes=10 ** 9, workers=2)
    res, summ = srv.run(reqs)
    assert summ["completed"] == 10
    sizes = [len(ids) for _, ids in srv.batches]
    assert sizes[0] == 1 and max(sizes) > 1           # later arrivals were batched together
    assert sorted(i for _, ids in srv.batches for i in ids) == list(range(10))


def test_max_rhs_caps_a_batch():
    be = FakeBackend(solve_s=0.02)
    reqs = [req(i, 8, 0.0, nrhs=5) for i in range(12)]
    srv = Server(be, budget_bytes=10 ** 9, max_rhs=16)
    res, summ = srv.run(reqs)
    assert summ["completed"] == 12
    for _, ids in srv.batches:
        assert sum(reqs[i].nrhs for i in ids) <= 16


def test_budget_respected_and_lru_eviction():
    be = FakeBackend(solve_s=0.005)
    n = 16
    fb = 100 * n * n
    ws = 10 * n * n
    budget = 2 * fb + 2 * ws              # two plans resident at a time, one RHS each
    keys = [0, 1, 2, 0, 1, 2, 3, 0]
    reqs = [req(i, n, 0.02 * i, key_tag=k) for i, k in enumerate(keys)]
    srv = Server(be, budget_bytes=budget, workers=2)
    res, summ = srv.run(reqs)
    assert summ["completed"] == len(reqs)
    assert summ["peak_bytes"] <= budget
    assert summ["evictions"] > 0
    assert summ["factorizations"] == len(be.created) > 4   # evicted keys were refactored


def test_concurrent_keys_overlap():
    be = FakeBackend(solve_s=0.05)
    reqs = [req(i, 8, 0.0, key_tag=i) for i in range(4)]
    Server(be, budget_bytes=10 ** 9, workers=4).run(reqs)
    assert be.max_concurrent >= 2


def test_over_budget_request_fails_cleanly():
    be = FakeBackend()
    big = req(0, 64, 0.0)                     # 409,600 factor bytes
    small = req(1, 8, 0.0, key_tag=1)
    res, summ = Server(be, budget_bytes=100_000).run([big, small])
    assert res[0].status.startswith("failed") and "budget" in res[0].status
    assert res[1].status == "ASP_OK"
    assert summ["failed"] == 1 and summ["peak_bytes"] <= 100_000


def test_workspace_shrinks_batch_to_fit():
    be = FakeBackend(solve_s=0.01)
    n = 8
    budget = 100 * n * n + 3 * 10 * n * n      # factors + 3 RHS of workspace
    reqs = [req(i, n, 0.0) for i in range(7)]
    srv = Server(be, budget_bytes=budget)
    res, summ = srv.run(reqs)
    assert summ["completed"] == 7
    assert max(len(ids) for _, ids in srv.batches) <= 3
    assert summ["peak_bytes"] <= budget


def test_failing_backend_create_fails_its_requests_only():
    class Broken(FakeBackend):
        def create(self, r):
            if r.key[2] == 1:
                raise RuntimeError("cannot factor")
            return super().create(r)

    be = Broken()
    reqs = [req(0, 8, 0.0, key_tag=1), req(1, 8, 0.0, key_tag=0), req(2, 8, 0.01, key_tag=1)]
    res, summ = Server(be, budget_bytes=10 ** 9).run(reqs)
    assert res[1].status == "ASP_OK"
    for r in (res[0], res[2]):
        assert r.status.startswith("failed") and "cannot factor" in r.status
    assert summ["failed"] == 2 and be.live == {}


def test_request_stream_recipe():
    s = workloads.request_stream(count=400, rate=100.0, seed=5)
    assert len(s) == 400
    arr = np.array([d["arrival"] for d in s])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    gaps = np.diff(arr)
    assert abs(gaps.mean() * 100.0 - 1.0) < 0.2      # Poisson rate 100/s
    assert all(1 <= d["nrhs"] <= 32 for d in s)
    keys = [d["key"] for d in s]
    seen, repeats = set(), 0
    for k in keys:
        repeats += k in seen
        seen.add(k)
    assert 0.42 < repeats / len(keys) < 0.58          # repeat rate 0.5
    for d in s:
        assert abs(d["omega"] - 2 * np.pi * d["n"] / 8) < 1e-12
        assert (d["d"], d["n"]) in {(2, 127), (2, 255), (2, 511), (2, 1023), (3, 31), (3, 63)}
    assert workloads.request_stream(count=50, seed=5) == workloads.request_stream(count=50, seed=5)


def test_stream_requests_materialize_lazily():
    s = workloads.request_stream(count=5, seed=9, sizes=((2, 15),), max_rhs=3)
    r = Request.from_description(s[0])
    f = r.rhs()
    assert f.shape == (s[0]["nrhs"], 15 * 15) and f.dtype == np.complex128
    c = r.velocity()
    assert c.shape == (15, 15) and 0.79 < c.min() <= c.max() < 1.34
    assert r.pml_eta == 12 and r.layer_b == 4


@pytest.mark.parametrize("realtime", [True, False])
def test_stream_through_fake_backend(realtime):
    s = workloads.request_stream(count=60, rate=2000.0, seed=1, sizes=((2, 15), (2, 31)),
                                 max_rhs=4)
    reqs = [Request.from_description(d) for d in s]
    be = FakeBackend(solve_s=0.002, create_s=0.001)
    res, summ = Server(be, budget_bytes=10 ** 9, realtime=realtime).run(reqs)
    assert summ["completed"] == 60
    assert summ["factorizations"] == len({d["key"] for d in s})
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0


def test_saturated_latency_counts_from_the_start():
    """Without real-time arrivals every request is queued at the start: its
    latency runs from there, whatever arrival time the stream gave it."""
    s = workloads.request_stream(count=20, rate=0.5, seed=2, sizes=((2, 15),), max_rhs=2)
    assert max(d["arrival"] for d in s) > 5.0
    reqs = [Request.from_description(d) for d in s]
    res, summ = Server(FakeBackend(solve_s=0.001, create_s=0.001), budget_bytes=10 ** 9,
                       realtime=False).run(reqs)
    assert summ["completed"] == 20 and summ["wall_s"] < 5.0
    assert all(0.0 < r.done - r.arrival <= summ["wall_s"] for r in res)


def test_factorization_work_buffers_are_reserved_while_creating():
    """A plan's creation needs its factors plus the factorization's work
    buffers; the server reserves both and returns the work buffers when the
    creation ends, so a budget that holds the factors and a batch but not the
    work buffers next to another resident plan forces an eviction first."""
    class Working(FakeBackend):
        def __init__(self):
            super().__init__(solve_s=0.002, create_s=0.01)
            self.inflight = 0
            self.peak_true = 0
            self.srv = None

        def factor_work_bytes(self, r):
            return 50 * r.n * r.n

        def create(self, r):
            with self.lock:
                # device bytes really held while this creation runs
                self.peak_true = max(self.peak_true, self.srv._used)
            return super().create(r)

    be = Working()
    n = 16
    fb, fw, ws = 100 * n * n, 50 * n * n, 10 * n * n
    budget = 2 * fb + ws + fw - 1           # two plans fit, but not while a third creates
    reqs = [req(i, n, 0.05 * i, key_tag=i % 3) for i in range(6)]
    srv = Server(be, budget_bytes=budget, workers=1)
    be.srv = srv
    res, summ = srv.run(reqs)
    assert summ["completed"] == 6
    assert summ["peak_bytes"] <= budget
    assert be.peak_true >= fb + fw               # the creation held its work reservation
    assert summ["evictions"] > 0
