"""Served form: continuous batching of coarsening requests.

A request is one graph (host CSR) with its rating, k, stop size (20 k by
default, as in the experiments' 20 nodes per block) and balance tolerance.
Whenever a worker is free, the dispatcher takes the requests that have
arrived -- those with the oldest waiting request's rating and seed, in
arrival order -- until the batch's estimated device footprint reaches the
worker's budget or what is left of the device budget (batches in flight and
hierarchies kept resident count against it), or its union's weight sums
would leave 32 bits, and hands them over.  A worker (one host thread, one HIP
stream) uploads the batch's graphs, coarsens all of them together
(kappa_coarsen_graphs: the library lays out their union on the device), then
runs each request's way back up (stand-in partition, projection, cut and
balance) on its own hierarchy.  Workers run concurrently, so batches overlap
on the device; requests arriving meanwhile wait only for the next free worker
and for device memory.  Each result keeps its hierarchy resident on the
device when asked to, until BatchServer.release(result).

`LevelServer` batches at level granularity instead (the library's
kappa_server_*): every step advances all active requests of a rating by one
level in one batched pass, requests join at the next step after they arrive,
and each leaves as soon as its hierarchy ends.

`serve_plain` is the reference service: one request at a time, in arrival
order, through kappa_coarsen and kappa_uncoarsen.
"""
from __future__ import annotations

import queue
import threading
import time
from collections import deque
from dataclasses import dataclass
from typing import List, Optional, Sequence

from . import _lib as K


@dataclass
class Request:
    rid: int
    graph: object          # host CSR (workloads.CSR)
    rating: int
    k: int
    arrival: float = 0.0   # seconds after the start of the trace
    seed: int = 42
    stop_n: int = 0        # 0: 20 * k
    eps: tuple = (3, 100)
    part_seed: int = 1

    @property
    def stop(self) -> int:
        return self.stop_n if self.stop_n > 0 else 20 * self.k


@dataclass
class Result:
    rid: int
    levels: int
    stop_reason: int
    cut: tuple                  # level 0 cut/balance (kappa_cut_result fields)
    start: float                # when its batch started (trace clock)
    done: float                 # completion (trace clock)
    batch: float                # requests served together with it (itself included; the
                                # level-granular server: their mean over its steps)
    hierarchy: object = None    # the device-resident hierarchy (keep=True)

    def latency(self, arrival: float) -> float:
        return self.done - arrival


def footprint(g) -> int:
    """Estimated device bytes of one request inside a batch: input, matching
    and contraction scratch, and the hierarchy (about three times level 0)."""
    return 140 * int(g.n) + 44 * int(g.nnz) + (1 << 16)


def kept_bytes(g) -> int:
    """Estimated device bytes of one request's hierarchy kept resident
    (every level's c, offsets, mate, cmap and entries: about three times level 0)."""
    return 3 * (24 * int(g.n) + 8 * int(g.nnz)) + (1 << 12)


WEIGHT_CAP = (1 << 32) - 1   # the union's sum of w over E and sum of c over V


def weight_sums(g) -> tuple:
    """(sum of w over E, sum of c over V) of a host graph: a batch's union
    must keep both within 32 bits."""
    import numpy as np
    return int(np.asarray(g.ew, dtype=np.uint64).sum()) // 2, int(np.asarray(g.vw, dtype=np.uint64).sum())


def _finish(r: Request, H, t0: float, start: float, batch: int, keep: bool) -> Result:
    import torch
    n0 = int(H.info(0).n)
    part0 = torch.empty(max(n0, 1), dtype=torch.int32, device=H.device)
    _, res = K.kappa_uncoarsen(H, r.k, r.part_seed, r.eps[0], r.eps[1], part0=part0)
    levels = len(H)
    stop = int(H.info(levels - 1).stop_reason)
    return Result(r.rid, levels, stop, res[0].as_tuple(), start, time.perf_counter() - t0, batch,
                  H if keep else None)


def _wait_until(t0: float, at: float):
    d = at - (time.perf_counter() - t0)
    if d > 0:
        time.sleep(d)


def serve_plain(requests: Sequence[Request], device="cuda", keep: bool = False,
                t0: Optional[float] = None) -> List[Result]:
    """One request at a time, in arrival order."""
    import torch
    out = []
    t0 = time.perf_counter() if t0 is None else t0
    for r in sorted(requests, key=lambda q: q.arrival):
        _wait_until(t0, r.arrival)
        start = time.perf_counter() - t0
        dg = K.DeviceGraph.from_csr(r.graph, device)
        H = K.kappa_coarsen(dg, r.rating, r.seed, r.stop)
        out.append(_finish(r, H, t0, start, 1, keep))
    torch.cuda.synchronize()
    return out


def take_batch(arrived: Sequence[Request], budget: int, max_batch: int, sums: dict):
    """The next batch out of the arrived requests (in arrival order): those
    with the first one's rating and seed, as long as the estimated footprint
    stays within `budget`, the count within `max_batch` and the union's weight
    sums within 32 bits (the first request is always taken).  `sums` caches
    weight_sums per request id.  Returns (batch, the requests left)."""
    key = (arrived[0].rating, arrived[0].seed)
    batch, rest, used, uw, uc = [], [], 0, 0, 0
    for r in arrived:
        if r.rid not in sums:
            sums[r.rid] = weight_sums(r.graph)
        w, c = sums[r.rid]
        fp = footprint(r.graph)
        fits = (used + fp <= budget and uw + w <= WEIGHT_CAP and uc + c <= WEIGHT_CAP and
                len(batch) < max_batch)
        if (r.rating, r.seed) == key and (not batch or fits):
            batch.append(r)
            used += fp
            uw += w
            uc += c
        else:
            rest.append(r)
    return batch, rest


class BatchServer:
    """Continuous batching over `workers` concurrent workers."""

    def __init__(self, workers: int = 2, budget_bytes: int = 24 << 30, max_batch: int = 512,
                 device="cuda", hbm_budget: int = 200 << 30):
        self.workers = workers
        self.budget = budget_bytes        # per batch
        self.hbm_budget = hbm_budget      # batches in flight + kept hierarchies
        self.max_batch = max_batch
        self.device = device
        self._mem_lock = threading.Lock()
        self._kept = 0                    # bytes of kept hierarchies
        self._kept_of = {}                # request id -> its kept bytes
        self._inflight = 0                # bytes of batches being served

    def _run_batch(self, batch: List[Request], t0: float, keep: bool) -> List[Result]:
        start = time.perf_counter() - t0
        dgs = [K.DeviceGraph.from_csr(r.graph, self.device) for r in batch]
        B = K.kappa_coarsen_graphs(dgs, batch[0].rating, batch[0].seed, [r.stop for r in batch])
        del dgs
        return [_finish(r, B.hierarchy(i), t0, start, len(batch), keep)
                for i, r in enumerate(batch)]

    def release(self, result: Result):
        """Drops a kept hierarchy and returns its device memory to the budget."""
        if result.hierarchy is not None:
            result.hierarchy = None
            with self._mem_lock:
                self._kept -= self._kept_of.pop(result.rid, 0)

    def run(self, requests: Sequence[Request], keep: bool = False,
            t0: Optional[float] = None) -> List[Result]:
        import torch
        todo = deque(sorted(requests, key=lambda q: q.arrival))
        arrived: List[Request] = []
        jobs: "queue.Queue[Optional[List[Request]]]" = queue.Queue()
        free: "queue.Queue[int]" = queue.Queue()
        results: List[Result] = []
        errors: List[BaseException] = []
        sums = {}
        lock = threading.Lock()
        t0 = time.perf_counter() if t0 is None else t0

        def worker(wid: int):
            torch.cuda.set_device(torch.device(self.device).index or 0)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                while True:
                    batch = jobs.get()
                    if batch is None:
                        return
                    try:
                        res = self._run_batch(batch, t0, keep)
                        stream.synchronize()
                        with lock:
                            results.extend(res)
                        if keep:
                            with self._mem_lock:
                                for r in batch:
                                    self._kept_of[r.rid] = kept_bytes(r.graph)
                                    self._kept += self._kept_of[r.rid]
                    except BaseException as e:   # reported after the loop
                        with lock:
                            errors.append(e)
                    with self._mem_lock:
                        self._inflight -= sum(footprint(r.graph) for r in batch)
                    free.put(wid)

        threads = [threading.Thread(target=worker, args=(i,), daemon=True)
                   for i in range(self.workers)]
        for th in threads:
            th.start()
        idle = list(range(self.workers))
        while todo or arrived or len(idle) < self.workers:
            now = time.perf_counter() - t0
            while todo and todo[0].arrival <= now:
                arrived.append(todo.popleft())
            while True:   # collect finished workers
                try:
                    idle.append(free.get_nowait())
                except queue.Empty:
                    break
            if errors:
                break
            if arrived and idle:
                with self._mem_lock:
                    inflight, kept = self._inflight, self._kept
                room = self.hbm_budget - inflight - kept
                fp0 = footprint(arrived[0].graph)
                if fp0 <= room or (inflight == 0 and kept == 0):
                    batch, arrived = take_batch(arrived, min(self.budget, room), self.max_batch, sums)
                    with self._mem_lock:
                        self._inflight += sum(footprint(r.graph) for r in batch)
                    jobs.put(batch)
                    idle.pop()
                    continue
                if inflight == 0:   # only kept hierarchies stand in the way
                    errors.append(MemoryError(
                        f"request {arrived[0].rid} needs ~{fp0} device bytes; kept hierarchies "
                        f"hold {kept} of the {self.hbm_budget}-byte budget (release results)"))
                    break
            # nothing to hand out: wait for the next arrival or a free worker
            wait = (todo[0].arrival - now) if (todo and not arrived) else 0.05
            try:
                idle.append(free.get(timeout=max(wait, 1e-4)))
            except queue.Empty:
                pass
        for _ in threads:
            jobs.put(None)
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        torch.cuda.synchronize()
        return sorted(results, key=lambda q: q.rid)


class LevelServer:
    """Level-granular continuous batching over the library's servers
    (kappa_server_*: K.Server).

    Three kinds of host threads, each with its own HIP stream (a step runs
    level after level on the device until some request finishes or the
    uploaders interrupt it because a request of its class waits):
      * `uploaders` uploaders take requests in arrival order while the device
        budget allows (each is charged its estimated footprint until its
        result is recorded), copy the graph to the device and validate
        it there;
      * one engine per (rating, seed, size class) owns a server: it admits the
        uploaded requests of its class (trusted: validated already) while its
        active set stays within max_entries level-0 entries, then advances all
        of its active requests together, one batched pass per level; a
        request uploaded while a step runs joins at the next level boundary
        (at its level 0), and a request whose hierarchy ends leaves at once;
      * one finisher per engine runs the way back up (stand-in partition,
        projection, cut and balance) of each finished request on its own
        hierarchy and records the result, so that engines only step.
    Requests with more than split_entries level-0 entries step in engines of
    their own: a step lasts as long as its largest level, and small requests
    would otherwise wait on the large ones at every level.  Result.batch is
    the mean number of requests of the steps a request took part in."""

    def __init__(self, device="cuda", hbm_budget: int = 200 << 30, max_active: int = 4096,
                 max_entries: int = 1 << 27, split_entries: int = 1 << 18, uploaders: int = 2):
        self.device = device
        self.uploaders = uploaders
        self.hbm_budget = hbm_budget
        self.max_active = max_active
        self.max_entries = max_entries
        self.split_entries = split_entries
        self.profile = {}   # engine class -> {"steps", "step_s", "admit_s", "active_sum"}

    def _class(self, r: Request):
        return (r.rating, r.seed, int(r.graph.nnz) > self.split_entries)

    def run(self, requests: Sequence[Request], keep: bool = False,
            t0: Optional[float] = None) -> List[Result]:
        import torch
        t0 = time.perf_counter() if t0 is None else t0
        todo = sorted(requests, key=lambda q: q.arrival)
        classes = sorted({self._class(r) for r in todo})
        feeds = {c: queue.Queue() for c in classes}
        done_q = {c: queue.Queue() for c in classes}
        arrivals: queue.Queue = queue.Queue()
        results: List[Result] = []
        errors: List[BaseException] = []
        lock = threading.Lock()
        mem = threading.Condition()
        charged = [0]
        servers = {}   # class -> its engine's server, once created
        left = [self.uploaders]
        dev_index = torch.device(self.device).index or 0

        def fail(e):
            with lock:
                errors.append(e)
            with mem:
                mem.notify_all()

        def uploader():
            torch.cuda.set_device(dev_index)
            stream = torch.cuda.Stream()
            try:
                with torch.cuda.stream(stream):
                    while True:
                        r = arrivals.get()
                        if r is None:
                            break
                        fp = footprint(r.graph)
                        with mem:   # wait for device memory (a lone request always fits)
                            while not errors and charged[0] > 0 and charged[0] + fp > self.hbm_budget:
                                mem.wait()
                            charged[0] += fp
                        if errors:
                            break
                        dg = K.DeviceGraph.from_csr(r.graph, self.device)
                        st = K.kappa_validate(dg)
                        if st != K.OK:
                            raise K.KappaError("kappa_validate", st)
                        cls = self._class(r)
                        feeds[cls].put((r, dg))
                        srv = servers.get(cls)
                        if srv is not None:   # a running step ends at its next level boundary
                            srv.interrupt(True)
            except BaseException as e:
                fail(e)
            with lock:   # the last uploader to leave closes the feeds
                left[0] -= 1
                last = left[0] == 0
            if last:
                for c in classes:
                    feeds[c].put(None)

        def finisher(cls):
            torch.cuda.set_device(dev_index)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                while True:
                    item = done_q[cls].get()
                    if item is None:
                        break
                    r, H, start, sizes = item
                    try:
                        res = _finish(r, H, t0, start, 1, keep)
                        res.batch = float(sum(sizes)) / len(sizes)
                        with lock:
                            results.append(res)
                    except BaseException as e:
                        fail(e)
                    del H
                    with mem:
                        charged[0] -= footprint(r.graph)
                        mem.notify_all()

        def engine(cls):
            rating, seed, _ = cls
            torch.cuda.set_device(dev_index)
            stream = torch.cuda.Stream()
            prof = {"steps": 0, "step_s": 0.0, "admit_s": 0.0, "active_sum": 0}
            try:
                with torch.cuda.stream(stream):
                    srv = K.Server(rating, seed, trusted=True, device=self.device)
                    servers[cls] = srv
                    waiting: deque = deque()
                    live = {}        # server id -> (request, start, [step sizes])
                    entries = 0      # level-0 entries of the active set
                    ended = False
                    while not (ended and not waiting and not live) and not errors:
                        srv.interrupt(False)   # before looking: no arrival goes unseen
                        while not ended:   # uploaded requests (block only when idle)
                            try:
                                item = feeds[cls].get(block=not live and not waiting)
                            except queue.Empty:
                                break
                            if item is None:
                                ended = True
                            else:
                                waiting.append(item)
                        ta = time.perf_counter()
                        while waiting and len(live) < self.max_active:
                            r, dg = waiting[0]
                            if live and entries + int(r.graph.nnz) > self.max_entries:
                                break
                            waiting.popleft()
                            for t in (dg.xadj, dg.adj, dg.ew, dg.vw):
                                t.record_stream(stream)   # read by the admission copy
                            sid = srv.admit(dg, r.stop)
                            live[sid] = (r, time.perf_counter() - t0, [])
                            entries += int(r.graph.nnz)
                        prof["admit_s"] += time.perf_counter() - ta
                        if not live:
                            continue
                        size = len(live)
                        for v in live.values():
                            v[2].append(size)
                        ts = time.perf_counter()
                        fin = srv.step()
                        prof["step_s"] += time.perf_counter() - ts
                        prof["steps"] += 1
                        prof["active_sum"] += size
                        for sid in fin:
                            r, start, sizes = live.pop(sid)
                            entries -= int(r.graph.nnz)
                            done_q[cls].put((r, srv.take(sid), start, sizes))
                    stream.synchronize()
            except BaseException as e:
                fail(e)
            done_q[cls].put(None)
            with lock:
                self.profile[cls] = prof

        threads = [threading.Thread(target=uploader, daemon=True) for _ in range(self.uploaders)]
        threads += [threading.Thread(target=engine, args=(c,), daemon=True) for c in classes]
        threads += [threading.Thread(target=finisher, args=(c,), daemon=True) for c in classes]
        for th in threads:
            th.start()
        for r in todo:   # the dispatcher: hand each request over at its arrival
            _wait_until(t0, r.arrival)
            if errors:
                break
            arrivals.put(r)
        for _ in range(self.uploaders):
            arrivals.put(None)
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        torch.cuda.synchronize()
        return sorted(results, key=lambda q: q.rid)


def latency_stats(requests: Sequence[Request], results: Sequence[Result]) -> dict:
    """p50 / p99 latency (completion minus scheduled arrival, ms) and the
    aggregate edges/s (all edges over first arrival to last completion)."""
    import numpy as np
    arr = {r.rid: r.arrival for r in requests}
    lat = np.array([res.latency(arr[res.rid]) for res in results]) * 1e3
    edges = sum(int(r.graph.m) for r in requests)
    span = max(res.done for res in results) - min(arr.values())
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "edges_per_s": round(edges / span, 1), "span_s": round(span, 4),
            "requests": len(results),
            "mean_batch": round(float(np.mean([res.batch for res in results])), 2)}
