"""Serving loop: solve requests on one GPU with continuous batching.

A request names a problem (a 2D or 3D grid Laplacian with jittered weights, built
on the device from its seed) and 1..8 right-hand sides.  The server:

* replays arrivals at their timestamps (a Poisson stream);
* admits a request when a slot is free and its HBM footprint fits the budget:
  requests that arrive while others run are admitted as slots and memory free up,
  and their kernels run concurrently (each slot builds inputs on its own HIP
  stream; each hierarchy solves on a stream of its own);
* keeps hierarchies resident (least recently used evicted first when memory is
  needed), so a request for a resident problem skips the setup;
* merges queued requests for the same problem: a slot that takes a request also
  takes the waiting requests with the same key, up to ``max_rhs`` right-hand sides
  in all, and solves them as one batch (``amg_solve_batch``), so their K-cycles --
  the latency-bound coarse levels above all -- share every launch;
* optionally (``group_n`` > 0) solves small problems -- n <= group_n, FP64 --
  through grouped launches: a slot that takes a small request also takes the
  waiting small requests of any problem, up to ``group_jobs`` right-hand sides,
  and solves all of them in ONE kernel launch (``amg_solve_group``: one workgroup
  per right-hand side runs the whole solve), so the small-level work of
  concurrent requests shares a dispatch;
* reports per-request latency (arrival to completion), p50/p99 and solves/s.

Every kernel of a solve reads and writes only that solve's hierarchy and vectors
and reduces in a fixed order, and every column of a batch iterates on its own
(it stops, confirms and restarts by its own residuals), so a request's result does
not depend on what else runs or what it was merged with: the same alone and in the
mix (a test checks this bit for bit).  A small request takes the grouped path
whether it is alone or not (the choice depends on its size only), and a grouped
job's result does not depend on the other jobs of its launch.
"""
from __future__ import annotations

import collections
import concurrent.futures
import math
import threading
import time
from dataclasses import dataclass, field

from . import amg, inputs


@dataclass
class Request:
    rid: int
    t_arrival: float   # seconds from the start of the stream
    dims: tuple        # interior grid sizes (2 or 3 axes)
    jitter_seed: int   # edge weights 1 + 0.1 (2u - 1), u from this seed
    rhs_seeds: tuple   # one seed per right-hand side (U[-1, 1] entries)

    @property
    def key(self):
        return (self.dims, self.jitter_seed)

    @property
    def n(self) -> int:
        return math.prod(self.dims)


@dataclass
class Result:
    rid: int
    status: int
    latency_ms: float  # arrival to completion
    service_ms: float  # taken by a slot to completion
    queue_ms: float    # waiting for memory / a busy hierarchy after being taken
    setup_ms: float
    solve_ms: float
    reused: bool
    iterations: list
    rel_residuals: list
    solution: object = None  # (nrhs, n) host array when kept
    merged: int = 1          # requests solved in the same batch
    grouped: bool = False    # solved by a grouped launch


def make_requests(count: int = 2000, rate: float = 200.0, seed: int = 6, reuse: float = 0.3,
                  n_range_2d=(1e4, 2e6), n_range_3d=(1e4, 4e6), max_rhs: int = 8, window: int = 16):
    """A seeded request stream.  Inter-arrival times are exponential with mean
    1/rate; a request reuses, with probability `reuse`, one of the last `window`
    distinct problems (uniformly), else draws a new one: dimension 2 or 3 with
    probability 1/2, n log-uniform in the range of that dimension, side
    round(n^(1/d)); 1..max_rhs right-hand sides.  Draw j of request k is
    u(seed, 8k + j) of the counter-based generator."""
    reqs, recent = [], []
    t = 0.0
    for k in range(count):
        u = inputs.uniform(seed, [8 * k + j for j in range(8)])
        t += -math.log(1.0 - u[0]) / rate
        if recent and u[1] < reuse:
            dims, jseed = recent[min(int(u[2] * len(recent)), len(recent) - 1)]
        else:
            d = 2 if u[3] < 0.5 else 3
            lo, hi = n_range_2d if d == 2 else n_range_3d
            n = math.exp(math.log(lo) + u[4] * (math.log(hi) - math.log(lo)))
            side = max(2, int(round(n ** (1.0 / d))))
            dims, jseed = (side,) * d, 1000 + k
            recent.append((dims, jseed))
            if len(recent) > window:
                recent.pop(0)
        nrhs = 1 + min(int(u[5] * max_rhs), max_rhs - 1)
        reqs.append(Request(k, t, dims, jseed, tuple(100000 * (k + 1) + j for j in range(nrhs))))
    return reqs


class Server:
    """Continuous-batching solve server over `slots` worker threads, one HIP stream
    each, within an HBM `budget` (bytes; default 0.8 of the free device memory)."""

    def __init__(self, slots: int = 4, budget: int | None = None, tol: float = 1e-8,
                 precision: int = amg.AMG_PREC_FP32_INNER, max_rhs: int = 16, keep_solutions: bool = False,
                 skip_ratio: float = 0.0, group_n: int = 0, group_jobs: int = 256):
        import torch
        self.torch = torch
        self.slots, self.tol, self.precision, self.max_rhs = slots, tol, precision, max_rhs
        self.skip_ratio = skip_ratio  # level skipping of the hierarchies (Sec. 3.3); 0: the plain method
        self.group_n, self.group_jobs = group_n, group_jobs
        self.keep = keep_solutions
        if budget is None:
            free, _ = torch.cuda.mem_get_info()
            budget = int(0.8 * free)
        self.budget = budget
        self.lock = threading.Condition()
        self.resident = collections.OrderedDict()  # key -> [hierarchy, bytes, in_use]
        self.resident_bytes = 0
        self.inflight_bytes = 0

    # bytes a request needs beyond its hierarchy: the CSR it is built from and its
    # right-hand sides / solutions
    @staticmethod
    def vector_bytes(req: Request) -> int:
        nnz = (2 * len(req.dims) + 1) * req.n
        return 12 * nnz + 4 * req.n + 16 * req.n * len(req.rhs_seeds)

    # a hierarchy's bytes before it exists: measured figures of this library are
    # about 110 bytes per unknown and 56 per stored entry with 8 right-hand sides,
    # plus an FP64 iterate per right-hand side on the levels of at least 100k rows
    # and up to 16 bytes per entry for the sliced copies of those levels
    @staticmethod
    def hierarchy_estimate(req: Request, max_rhs: int) -> int:
        nnz = (2 * len(req.dims) + 1) * req.n
        return 72 * nnz + (60 + 17 * max_rhs) * req.n + (64 << 20)

    def _evict(self, need: int):
        """Drop least recently used idle hierarchies until `need` more bytes fit."""
        for key in list(self.resident):
            if self.resident_bytes + self.inflight_bytes + need <= self.budget:
                return
            h, nb, in_use = self.resident[key]
            if in_use:
                continue
            del self.resident[key]
            self.resident_bytes -= nb
            h.close()

    def _ensure_free(self, need: int):
        """The budget is an account; the device also holds cached blocks (the
        library's and torch's).  When the memory actually free is short of `need`
        plus a margin, drop idle resident hierarchies and both caches (the cache
        releases synchronise the device: done only under pressure).  Caller holds
        self.lock."""
        torch = self.torch
        margin = 1 << 30
        if torch.cuda.mem_get_info()[0] >= need + margin:
            return
        for key in list(self.resident):
            h, nb, in_use = self.resident[key]
            if not in_use:
                del self.resident[key]
                self.resident_bytes -= nb
                h.close()
        amg.amg_release_cached_memory()
        torch.cuda.empty_cache()

    def _admit(self, group):
        """Block until a group of requests for one problem fits; returns (hierarchy or
        None, reserved bytes)."""
        req = group[0]
        with self.lock:
            while True:
                entry = self.resident.get(req.key)
                if entry is not None and entry[2]:  # the hierarchy is busy: wait for it
                    self.lock.wait()
                    continue
                need = sum(self.vector_bytes(q) for q in group) + \
                    (0 if entry else self.hierarchy_estimate(req, self.max_rhs))
                if self.resident_bytes + self.inflight_bytes + need > self.budget:
                    self._evict(need)
                self._ensure_free(need)
                if self.resident_bytes + self.inflight_bytes + need <= self.budget or \
                        (self.inflight_bytes == 0 and not any(e[2] for e in self.resident.values())):
                    self.inflight_bytes += need
                    if entry is not None:
                        entry[2] = True
                        self.resident.move_to_end(req.key)
                        return entry[0], need
                    return None, need
                self.lock.wait()

    def _admit_nowait(self, group):
        """As _admit, without waiting: (hierarchy or None, reserved bytes), or False
        when the problem's hierarchy is busy or the memory is not there now."""
        req = group[0]
        with self.lock:
            entry = self.resident.get(req.key)
            if entry is not None and entry[2]:
                return False
            need = sum(self.vector_bytes(q) for q in group) + \
                (0 if entry else self.hierarchy_estimate(req, self.max_rhs))
            if self.resident_bytes + self.inflight_bytes + need > self.budget:
                self._evict(need)
            self._ensure_free(need)
            alone = self.inflight_bytes == 0 and not any(e[2] for e in self.resident.values())
            if self.resident_bytes + self.inflight_bytes + need > self.budget and not alone:
                return False
            self.inflight_bytes += need
            if entry is not None:
                entry[2] = True
                self.resident.move_to_end(req.key)
                return entry[0], need
            return None, need

    def _groupable(self, req: Request) -> bool:
        return self.group_n > 0 and req.n <= self.group_n and self.precision == amg.AMG_PREC_FP64

    def _release(self, req: Request, h, reserved: int, new: bool):
        """Return a request's reservation; keep its hierarchy resident (h may be None
        when the setup failed)."""
        with self.lock:
            self.inflight_bytes -= reserved
            if h is not None:
                if new and req.key in self.resident:  # built twice concurrently: keep the first
                    h.close()
                elif new:
                    nb = h.memory_bytes
                    self.resident[req.key] = [h, nb, False]
                    self.resident_bytes += nb
                else:
                    self.resident[req.key][2] = False
                self.resident.move_to_end(req.key)
            self._evict(0)
            self.lock.notify_all()

    def _serve_group(self, group, stream, t0: float):
        """Solve the right-hand sides of a group of requests for one problem as one
        batch; returns one Result per request."""
        torch = self.torch
        req = group[0]
        t_start = time.perf_counter()
        h, reserved = self._admit(group)
        t_admit = time.perf_counter()
        new = h is None
        sp = stream.cuda_stream
        st, infos, sol = -1, [], None
        try:
            with torch.cuda.stream(stream):
                if new:
                    rp, ci, va = amg.device_grid_laplacian(req.dims, 0.1, req.jitter_seed, stream=sp)
                    # the hierarchy gets a stream of its own (the library's): a resident
                    # hierarchy is later used from other slots, and work of another slot
                    # on this slot's stream would mix with, or break, a graph this slot
                    # is capturing
                    # no lane-count autotuning: most requests bring a new shape, and the
                    # measurement would add to their latency
                    h = amg.Hierarchy(rp, ci, va, precision=self.precision, max_rhs=self.max_rhs, autotune=0,
                                      skip_ratio=self.skip_ratio)
                    del rp, ci, va
                seeds = [s for q in group for s in q.rhs_seeds]
                B = torch.empty((len(seeds), req.n), dtype=torch.float64, device="cuda")
                for j, s in enumerate(seeds):
                    amg.device_rhs(B[j], s, stream=sp)
                X = torch.zeros_like(B)
                stream.synchronize()  # the hierarchy's stream does not wait for this one
                st, infos = h.solve_batch(B, X, tol=self.tol, raise_on_error=False)
                sol = X.cpu().numpy() if self.keep else None
                del B, X
        finally:
            self._release(req, h, reserved, new)
        t_done = time.perf_counter()
        out, col = [], 0
        for q in group:
            k = len(q.rhs_seeds)
            mine = infos[col:col + k]
            out.append(Result(q.rid, st, 1e3 * (t_done - (t0 + q.t_arrival)), 1e3 * (t_done - t_start),
                              1e3 * (t_admit - t_start), mine[0].setup_ms if new else 0.0, mine[0].solve_ms,
                              not new or q is not req, [i.iterations for i in mine], [i.rel_residual for i in mine],
                              sol[col:col + k] if sol is not None else None, len(group)))
            col += k
        return out

    def _serve_small(self, group, stream, t0: float, requeue):
        """Solve small requests (of any problems) in one grouped launch; requests
        whose hierarchy is busy, or whose memory is not free now, go back to the
        queue.  Returns one Result per request solved."""
        torch = self.torch
        t_start = time.perf_counter()
        by_key = collections.OrderedDict()
        for q in group:
            by_key.setdefault(q.key, []).append(q)
        held, deferred = [], []
        for reqs in by_key.values():
            got = self._admit_nowait(reqs)
            if got is False:
                deferred += reqs
            else:
                held.append([reqs, got[0], got[1], got[0] is None])
        if deferred:
            requeue(deferred)
        if not held:
            with self.lock:
                self.lock.wait(0.01)  # a busy hierarchy or full memory: let others finish first
            return []
        t_admit = time.perf_counter()
        out = []
        try:
            sp = stream.cuda_stream

            def build(ent):  # a new problem's matrix and hierarchy, on a stream of its own
                req = ent[0][0]
                st = torch.cuda.Stream()
                with torch.cuda.stream(st):
                    rp, ci, va = amg.device_grid_laplacian(req.dims, 0.1, req.jitter_seed, stream=st.cuda_stream)
                    ent[1] = amg.Hierarchy(rp, ci, va, precision=self.precision, max_rhs=self.max_rhs, autotune=0,
                                           skip_ratio=self.skip_ratio)
                st.synchronize()

            # the setups of the group's new problems run side by side (host threads; the
            # library's calls release the interpreter while they wait on the device)
            fresh = [ent for ent in held if ent[3]]
            if len(fresh) > 1:
                with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(fresh))) as pool:
                    list(pool.map(build, fresh))
            elif fresh:
                build(fresh[0])
            with torch.cuda.stream(stream):
                jobs, spans = [], []
                for ent in held:
                    reqs, h, _, new = ent
                    req = reqs[0]
                    seeds = [s for q in reqs for s in q.rhs_seeds]
                    B = torch.empty((len(seeds), req.n), dtype=torch.float64, device="cuda")
                    for j, s in enumerate(seeds):
                        amg.device_rhs(B[j], s, stream=sp)
                    X = torch.zeros_like(B)
                    spans.append((len(jobs), B, X))
                    jobs += [(h, c, B[c], X[c]) for c in range(len(seeds))]
                stream.synchronize()
                st, status, infos = amg.solve_group(jobs, tol=self.tol, stream=sp, raise_on_error=False)
                t_done = time.perf_counter()
                for (reqs, h, _, new), (j0, B, X) in zip(held, spans):
                    sol = X.cpu().numpy() if self.keep else None
                    col = 0
                    for q in reqs:
                        k = len(q.rhs_seeds)
                        mine, ms = infos[j0 + col:j0 + col + k], status[j0 + col:j0 + col + k]
                        bad = [v for v in ms if v != amg.AMG_OK]
                        out.append(Result(q.rid, bad[0] if bad else amg.AMG_OK, 1e3 * (t_done - (t0 + q.t_arrival)),
                                          1e3 * (t_done - t_start), 1e3 * (t_admit - t_start),
                                          mine[0].setup_ms if new else 0.0, mine[0].solve_ms,
                                          not new or q is not reqs[0], [i.iterations for i in mine],
                                          [i.rel_residual for i in mine],
                                          sol[col:col + k] if sol is not None else None, len(group), True))
                        col += k
                del jobs, spans
        finally:
            for reqs, h, reserved, new in held:
                self._release(reqs[0], h, reserved, new)
        return out

    def _take(self, pending):
        """The oldest waiting request and the waiting requests for the same problem
        that fit in one batch with it; for a small request (grouped path), the
        waiting small requests of any problem, up to group_jobs right-hand sides and
        max_rhs per problem (caller holds the queue's lock)."""
        first = pending.popleft()
        if self._groupable(first):
            group, cols = [first], len(first.rhs_seeds)
            per_key = {first.key: cols}
            for q in list(pending):
                k = len(q.rhs_seeds)
                if not self._groupable(q) or cols + k > self.group_jobs or per_key.get(q.key, 0) + k > self.max_rhs:
                    continue
                pending.remove(q)
                group.append(q)
                cols += k
                per_key[q.key] = per_key.get(q.key, 0) + k
            return group
        group, cols = [first], len(first.rhs_seeds)
        for q in list(pending):
            if q.key == first.key and cols + len(q.rhs_seeds) <= self.max_rhs:
                pending.remove(q)
                group.append(q)
                cols += len(q.rhs_seeds)
        return group

    def run(self, requests, realtime: bool = True, progress=None):
        """Serve `requests` (sorted by arrival); returns (results by rid, stats).
        progress(done, total, result) is called after every completed request."""
        torch = self.torch
        pending = collections.deque()
        cv = threading.Condition()
        done_feeding = [False]
        results, errors = {}, []
        t0 = time.perf_counter()

        def requeue(reqs):
            with cv:
                for q in reversed(reqs):
                    pending.appendleft(q)
                cv.notify_all()

        def worker():
            stream = torch.cuda.Stream()
            while True:
                with cv:
                    while not pending and not done_feeding[0]:
                        cv.wait()
                    if not pending:
                        return
                    group = self._take(pending)
                try:
                    served = self._serve_small(group, stream, t0, requeue) if self._groupable(group[0]) \
                        else self._serve_group(group, stream, t0)
                    for res in served:
                        with cv:
                            results[res.rid] = res
                            done = len(results)
                        if progress:
                            progress(done, len(requests), res)
                except Exception as e:  # noqa: BLE001 - reported at once and by run()
                    req = group[0]
                    errors.append((req.rid, repr(e)))
                    print(f"[serve] requests {[q.rid for q in group]} {req.dims} failed: {e!r}", flush=True)

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.slots)]
        for t in threads:
            t.start()
        for req in requests:
            if realtime:
                delay = t0 + req.t_arrival - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            with cv:
                pending.append(req)
                cv.notify()
        with cv:
            done_feeding[0] = True
            cv.notify_all()
        for t in threads:
            t.join()
        wall = time.perf_counter() - t0
        if errors:
            raise RuntimeError(f"{len(errors)} requests failed, first: {errors[0]}")
        lat = sorted(r.latency_ms for r in results.values())
        svc = sorted(r.service_ms for r in results.values())
        pct = lambda q, v=lat: v[min(len(v) - 1, int(math.ceil(q * len(v))) - 1)]
        solves = sum(len(r.iterations) for r in results.values())
        stats = {"requests": len(results), "solves": solves, "wall_s": wall, "solves_per_s": solves / wall,
                 "requests_per_s": len(results) / wall, "p50_ms": pct(0.50), "p99_ms": pct(0.99),
                 "service_p50_ms": pct(0.50, svc), "service_p99_ms": pct(0.99, svc),
                 "max_ms": lat[-1], "reused": sum(r.reused for r in results.values()),
                 "merged": sum(r.merged > 1 for r in results.values()),
                 "grouped": sum(r.grouped for r in results.values()),
                 "failed": sum(r.status != amg.AMG_OK for r in results.values())}
        return results, stats

    def close(self):
        with self.lock:
            for h, _, _ in self.resident.values():
                h.close()
            self.resident.clear()
            self.resident_bytes = 0
