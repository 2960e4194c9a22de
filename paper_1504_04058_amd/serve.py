"""Served Helmholtz solves over the C ABI.

A request asks for the solution of one discretized problem (velocity c, omega,
n, dimension, PML and layer settings) for a batch of right-hand sides.  The
server

* keeps the factored auxiliary problems of a key (velocity, omega, n, ...)
  resident in device memory and reuses them for later requests with the same
  key (a factor cache with least-recently-used eviction of idle entries);
* admits work by device memory: a plan is created only when its factors fit
  the budget, and a batch starts only when its workspaces fit as well;
* batches continuously: the right-hand sides of all queued requests for a key
  go into the next GMRES call on that key's plan, so requests that arrive while
  the key is busy join the following batch; different keys run concurrently on
  their own HIP streams from a pool of worker threads;
* records arrival, start and completion times, from which p50/p99 latency and
  solves/s follow.

Each right-hand side is solved in its own Krylov space with reductions in a
fixed order, so its result does not depend on which other right-hand sides
share its batch.  The device work is the library's; this module only decides
what runs when.
"""
import collections
import dataclasses
import threading
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    """One solve request.  ``c`` and ``f`` are host arrays or zero-argument
    callables that build them (so that a long stream need not hold every
    right-hand side in memory before it arrives)."""
    rid: int
    key: tuple            # identifies the discretized problem (factor cache key)
    arrival: float        # seconds from the start of the run
    dim: int
    n: int
    omega: float
    nrhs: int
    c: object             # velocity, (n,)*dim float64
    f: object             # right-hand sides, (nrhs, n**dim) complex128
    layer_b: int = 4
    pml_eta: int = 12
    C: float = 25.0

    def velocity(self):
        return self.c() if callable(self.c) else self.c

    def rhs(self):
        f = self.f() if callable(self.f) else self.f
        if f.shape != (self.nrhs, self.n ** self.dim):
            raise ValueError(f"request {self.rid}: right-hand sides of shape {f.shape}")
        return f

    @classmethod
    def from_description(cls, desc):
        """A request from a stream description (see ``workloads.request_stream``)."""
        import workloads

        return cls(desc["rid"], desc["key"], desc["arrival"], desc["d"], desc["n"],
                   desc["omega"], desc["nrhs"], lambda: workloads.velocity_of(desc),
                   lambda: workloads.sources_of(desc), layer_b=desc["b"], pml_eta=desc["gamma"])


@dataclasses.dataclass
class Result:
    rid: int
    key: tuple
    nrhs: int
    arrival: float
    start: float = 0.0
    done: float = 0.0
    iters: Optional[np.ndarray] = None
    relres: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None
    status: str = "pending"
    cache_hit: bool = False


class Backend:
    """What the server needs from the solver.  `AspBackend` runs the HIP library;
    tests substitute a CPU stand-in."""

    def factor_bytes(self, req: Request) -> int:
        raise NotImplementedError

    def factor_work_bytes(self, req: Request) -> int:
        """Device bytes the factorization needs for the time of `create`
        (work buffers that `create` releases before it returns)."""
        return 0

    def workspace_bytes(self, req: Request, nrhs: int) -> int:
        raise NotImplementedError

    def create(self, req: Request):
        raise NotImplementedError

    def solve(self, handle, f: np.ndarray):
        """Blocking solve of f (nrhs, N); returns (u, iters, relres, status)."""
        raise NotImplementedError

    def trim(self, handle):
        pass

    def destroy(self, handle):
        raise NotImplementedError


class AspBackend(Backend):
    """The HIP library: one plan per key, each on its own device stream."""

    def __init__(self, prec=1, tol=1e-6, restart=20, maxit=400, keep_u=True, cache_bytes=None):
        import torch

        from . import asp

        self.asp, self.torch = asp, torch
        self.prec, self.tol, self.restart, self.maxit = prec, tol, restart, maxit
        self.keep_u = keep_u
        # device memory the library keeps for reuse across plans (None: leave
        # the library's setting); given back by close()
        self._cache_prev = None if cache_bytes is None else asp.asp_set_cache_limit(cache_bytes)
        self._hosts = {}      # shape -> host-only plan (sizes only, no device state)
        self._ws = {}         # (shape, nrhs) -> workspace bytes
        self._lock = threading.Lock()

    def _host_plan(self, req):
        """A host-only plan of the request's shape: the library's own sizes
        (factors, factorization work buffers, workspaces) without a device."""
        k = (req.dim, req.n, req.layer_b, req.pml_eta)
        with self._lock:
            if k not in self._hosts:
                h = self.asp.asp_setup(req.dim, np.ones(req.n ** req.dim), req.omega, req.n,
                                       req.layer_b, req.pml_eta, C=req.C, prec=self.prec,
                                       host_only=True)
                self._hosts[k] = (h, self.asp.asp_info(h))
            return k, self._hosts[k]

    def factor_bytes(self, req):
        return self._host_plan(req)[1][1]["factor_bytes"]

    def factor_work_bytes(self, req):
        return self._host_plan(req)[1][1]["factor_work_bytes"]

    def workspace_bytes(self, req, nrhs):
        k, (h, _) = self._host_plan(req)
        with self._lock:
            if (k, nrhs) not in self._ws:
                self._ws[(k, nrhs)] = self.asp.asp_workspace_estimate(h, nrhs, self.restart)
            return self._ws[(k, nrhs)]

    def create(self, req):
        torch = self.torch
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            plan = self.asp.Plan(req.dim, req.velocity(), req.omega, req.n, req.layer_b, req.pml_eta,
                                 C=req.C, prec=self.prec)
            self.asp.asp_set_stream(plan.handle, stream.cuda_stream)
            plan.factor()
            # the factorization's work buffers go back before the plan is cached
            self.asp.asp_release_workspace(plan.handle)
        return (plan, stream)

    def close(self):
        with self._lock:
            for h, _ in self._hosts.values():
                self.asp.asp_destroy(h)
            self._hosts.clear()
            if self._cache_prev is not None:
                self.asp.asp_set_cache_limit(self._cache_prev)
                self._cache_prev = None

    def solve(self, handle, f):
        torch = self.torch
        plan, stream = handle
        with torch.cuda.stream(stream):
            fd = torch.from_numpy(np.ascontiguousarray(f)).to("cuda", non_blocking=False)
            u = torch.empty_like(fd)
            st, it, rr = self.asp.asp_gmres(plan.handle, fd, u, f.shape[0], self.tol,
                                            self.restart, self.maxit)
            stream.synchronize()
            uh = u.cpu().numpy() if self.keep_u else None
        return uh, it, rr, self.asp.STATUS_NAMES.get(st, str(st))

    def trim(self, handle):
        self.asp.asp_release_workspace(handle[0].handle)

    def destroy(self, handle):
        handle[0].close()


@dataclasses.dataclass
class _Entry:
    key: tuple
    handle: object = None
    fbytes: int = 0
    busy: bool = False
    creating: bool = False
    last_used: float = 0.0


class Server:
    """Continuous-batching request loop.  `run` replays a request stream
    (sorted by arrival) and returns the results and summary statistics."""

    def __init__(self, backend: Backend, budget_bytes: int, max_rhs: int = 64, workers: int = 4,
                 realtime: bool = True, progress_every: int = 0):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_rhs = max_rhs
        self.workers = workers
        self.realtime = realtime
        self._lock = threading.Condition()
        self._queue: Dict[tuple, collections.deque] = collections.OrderedDict()
        self._cache: Dict[tuple, _Entry] = collections.OrderedDict()
        self._used = 0              # bytes of resident factors + running workspaces
        self._peak = 0
        self._arrivals_done = False
        self._results: Dict[int, Result] = {}
        self.evictions = 0
        self.factorizations = 0
        self.batches = []           # (key, request ids) of every solve launched
        self.progress_every = progress_every   # print a line every so many completed requests
        self._completed = 0

    # -- memory ------------------------------------------------------------------------
    def _reserve(self, nbytes):
        """Reserve nbytes, evicting idle cached plans (least recently used first)."""
        if nbytes > self.budget:
            return False
        while self._used + nbytes > self.budget:
            victim = None
            for e in self._cache.values():
                if not e.busy and not e.creating and e.handle is not None \
                        and not self._queue.get(e.key):
                    if victim is None or e.last_used < victim.last_used:
                        victim = e
            if victim is None:
                return False
            self.backend.destroy(victim.handle)
            self._used -= victim.fbytes
            del self._cache[victim.key]
            self.evictions += 1
        self._used += nbytes
        self._peak = max(self._peak, self._used)
        return True

    def _fail(self, reqs, why):
        now = time.perf_counter() - self._t0
        for r in reqs:
            res = self._results[r.rid]
            res.status = f"failed: {why}"
            res.done = now

    # -- scheduling ----------------------------------------------------------------------
    def _pick(self):
        """Next unit of work under the lock: ('create', req) or ('solve', entry, reqs)."""
        for key, q in self._queue.items():
            if not q:
                continue
            e = self._cache.get(key)
            if e is None:
                req = q[0]
                fb = self.backend.factor_bytes(req)
                fw = self.backend.factor_work_bytes(req)
                if max(fb + fw, fb + self.backend.workspace_bytes(req, 1)) > self.budget:
                    # can never run: fail the key's requests instead of waiting
                    self._fail(list(q), "exceeds the device memory budget")
                    q.clear()
                    continue
                # the factors, and the factorization's work buffers while it runs
                if not self._reserve(fb + fw):
                    continue
                e = _Entry(key, fbytes=fb, creating=True)
                self._cache[key] = e
                return ("create", e, req, fw)
            if e.busy or e.creating:
                continue
            batch, total = [], 0
            while q and (not batch or total + q[0].nrhs <= self.max_rhs):
                total += q[0].nrhs
                batch.append(q.popleft())
            e.busy = True                            # its own factors are not evictable
            ws = self.backend.workspace_bytes(batch[0], total)
            reserved = self._reserve(ws)
            while not reserved and len(batch) > 1:
                q.appendleft(batch.pop())            # a smaller batch may fit
                ws = self.backend.workspace_bytes(batch[0], sum(r.nrhs for r in batch))
                reserved = self._reserve(ws)
            if not reserved:
                e.busy = False
                if ws > self.budget - e.fbytes:      # can never fit next to its factors
                    self._fail(batch, "exceeds the device memory budget")
                else:
                    for r in reversed(batch):
                        q.appendleft(r)
                continue
            self.batches.append((key, [r.rid for r in batch]))
            self._cache.move_to_end(key)
            return ("solve", e, batch, ws)
        return None

    def _worker(self, t0):
        while True:
            with self._lock:
                work = self._pick()
                while work is None:
                    if self._arrivals_done and not any(self._queue.values()) and \
                            not any(e.busy or e.creating for e in self._cache.values()):
                        self._lock.notify_all()
                        return
                    self._lock.wait(0.05)
                    work = self._pick()
            if work[0] == "create":
                _, e, req, fw = work
                try:
                    h = self.backend.create(req)
                    err = None
                except Exception as ex:   # the key cannot be served
                    h, err = None, ex
                with self._lock:
                    e.creating = False
                    self._used -= fw           # work buffers released by create
                    if h is None:
                        self._used -= e.fbytes
                        del self._cache[e.key]
                        self._fail(list(self._queue.pop(e.key, [])), str(err))
                    else:
                        e.handle = h
                        e.last_used = time.perf_counter()
                        self.factorizations += 1
                    self._lock.notify_all()
                continue
            _, e, batch, ws = work
            start = time.perf_counter() - t0
            try:
                f = np.concatenate([r.rhs() for r in batch], axis=0)
                u, it, rr, st = self.backend.solve(e.handle, f)
                self.backend.trim(e.handle)
                err = None
            except Exception as ex:
                u = it = rr = None
                st, err = "failed", ex
            done = time.perf_counter() - t0
            with self._lock:
                off = 0
                for r in batch:
                    res = self._results[r.rid]
                    res.start, res.done = start, done
                    if err is None:
                        k = r.nrhs
                        res.iters, res.relres = it[off:off + k], rr[off:off + k]
                        res.u = None if u is None else u[off:off + k]
                        res.status = st
                        off += k
                    else:
                        res.status = f"failed: {err}"
                e.busy = False
                e.last_used = time.perf_counter()
                self._used -= ws
                if self.progress_every:
                    before = self._completed // self.progress_every
                    self._completed += len(batch)
                    if self._completed // self.progress_every > before:
                        print(f"serve: {self._completed} requests done at {done:.1f} s, "
                              f"{self.factorizations} factorizations, {self.evictions} evictions",
                              flush=True)
                self._lock.notify_all()

    def run(self, requests: List[Request]):
        t0 = time.perf_counter()
        self._t0 = t0
        for r in requests:
            # without real-time arrivals every request is queued at the start,
            # and its latency counts from there
            self._results[r.rid] = Result(r.rid, r.key, r.nrhs, r.arrival if self.realtime else 0.0)
        pool = [threading.Thread(target=self._worker, args=(t0,), daemon=True)
                for _ in range(self.workers)]
        for th in pool:
            th.start()
        seen = set()
        for r in sorted(requests, key=lambda q: q.arrival):
            if self.realtime:
                delay = r.arrival - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            with self._lock:
                res = self._results[r.rid]
                res.cache_hit = r.key in seen
                seen.add(r.key)
                self._queue.setdefault(r.key, collections.deque()).append(r)
                self._lock.notify_all()
        with self._lock:
            self._arrivals_done = True
            self._lock.notify_all()
        for th in pool:
            th.join()
        wall = time.perf_counter() - t0
        for e in list(self._cache.values()):
            if e.handle is not None:
                self.backend.destroy(e.handle)
        self._cache.clear()
        results = [self._results[r.rid] for r in requests]
        return results, summarize(results, wall, self)


def summarize(results, wall, server=None):
    ok = [r for r in results if not r.status.startswith("failed")]
    lat = np.array([r.done - r.arrival for r in ok]) if ok else np.zeros(1)
    solves = sum(r.nrhs for r in ok)
    out = {
        "requests": len(results),
        "completed": len(ok),
        "failed": len(results) - len(ok),
        "solves": solves,
        "wall_s": wall,
        "solves_per_s": solves / wall if wall > 0 else 0.0,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "max_relres": float(max((r.relres.max() for r in ok if r.relres is not None), default=0.0)),
    }
    if server is not None:
        out.update({"factorizations": server.factorizations, "evictions": server.evictions,
                    "peak_bytes": server._peak, "budget_bytes": server.budget})
    return out
