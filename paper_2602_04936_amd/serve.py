"""Continuous-batching serving loop over a resident index.

Requests (a block of 1..B queries sharing one k) arrive over time.  The index
stays resident in HBM; a fixed set of launch slots, one HIP stream each,
carries work to the GPU.  Whenever a slot is free, the scheduler packs the
oldest waiting requests that fit the slot's memory (query rows, k/offsets,
output entries) into one call of the index path, so requests that arrive
while others are on the GPU join the next launch and their work overlaps on
the device with launches already in flight.  Each query's answer does not
depend on which other queries share its launch (queries are independent and
the kernels are deterministic), so a request's result is the same alone and in
the mix.

The paper's sustained benchmark issues one top-1 query at a time (section 7,
Table "Sustained benchmark"; Appendix C); this loop is the batched, open-loop
form of that measurement: latency = completion time - arrival time, reported
as p50/p99 next to the achieved queries/s.

`Scheduler` is pure host logic and is tested on the CPU with a fake executor;
`GpuExecutor` is the only part that touches the device.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Deque, List, Optional

import numpy as np

__all__ = ["Request", "Scheduler", "GpuExecutor", "run_loop", "latency_report", "slot_capacities",
           "requests_from_schedule", "run_served", "run_synchronous"]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    queries: np.ndarray     # [b, L] tokens
    k: int
    done: float = -1.0      # completion time (seconds since start)
    ids: Optional[np.ndarray] = None   # [b, k]
    lcps: Optional[np.ndarray] = None  # [b, k]

    @property
    def b(self) -> int:
        return int(self.queries.shape[0])


class Scheduler:
    """FIFO admission into launch slots bounded by per-slot capacities.

    cap_queries : query rows per launch
    cap_entries : output entries (sum of k over the launch's queries) per launch
    A request larger than a whole slot is rejected at submit time.
    """

    def __init__(self, cap_queries: int, cap_entries: int):
        if cap_queries < 1 or cap_entries < 1:
            raise ValueError("capacities must be positive")
        self.cap_queries = cap_queries
        self.cap_entries = cap_entries
        self.pending: Deque[Request] = collections.deque()

    def submit(self, req: Request):
        if req.b > self.cap_queries or req.b * req.k > self.cap_entries:
            raise ValueError(f"request {req.rid} ({req.b} queries, k={req.k}) exceeds one launch slot")
        self.pending.append(req)

    def next_batch(self) -> List[Request]:
        """Oldest pending requests that fit one slot (possibly empty)."""
        batch: List[Request] = []
        nq = ne = 0
        while self.pending:
            r = self.pending[0]
            if nq + r.b > self.cap_queries or ne + r.b * r.k > self.cap_entries:
                break
            batch.append(self.pending.popleft())
            nq += r.b
            ne += r.b * r.k
        return batch

    def __len__(self):
        return len(self.pending)


def slot_capacities(budget_bytes: int, n_slots: int, row_bytes: int, k_max: int = 100):
    """Split a device-memory budget over the slots: each query row costs its
    tokens + k and offset words, each output entry 8 bytes (id + LCP)."""
    per_slot = budget_bytes // n_slots
    per_query = row_bytes + 4 + 8 + 8 * k_max
    cap_q = max(1, per_slot // per_query)
    return int(cap_q), int(cap_q * k_max)


class GpuExecutor:
    """Launch slots on separate HIP streams; outputs come back to pinned host memory."""

    def __init__(self, index, n_slots: int, cap_queries: int, cap_entries: int, scan: bool = False):
        import torch
        self.torch = torch
        self.index = index
        self.scan = scan
        dev = index.device
        L, tb = index.L, index.token_bytes
        qdt = torch.uint8 if tb == 1 else torch.int16
        self.slots = []
        for _ in range(n_slots):
            s = {
                "stream": torch.cuda.Stream(device=dev),
                "q_host": torch.empty((cap_queries, L), dtype=qdt, pin_memory=True),
                "k_host": torch.empty(cap_queries, dtype=torch.int32, pin_memory=True),
                "off_host": torch.empty(cap_queries + 1, dtype=torch.int64, pin_memory=True),
                "q_dev": torch.empty((cap_queries, L), dtype=qdt, device=dev),
                "k_dev": torch.empty(cap_queries, dtype=torch.int32, device=dev),
                "off_dev": torch.empty(cap_queries + 1, dtype=torch.int64, device=dev),
                "ids_dev": torch.empty(cap_entries, dtype=torch.int32, device=dev),
                "lcp_dev": torch.empty(cap_entries, dtype=torch.int32, device=dev),
                "ids_host": torch.empty(cap_entries, dtype=torch.int32, pin_memory=True),
                "lcp_host": torch.empty(cap_entries, dtype=torch.int32, pin_memory=True),
                "event": torch.cuda.Event(),
                "batch": None,
            }
            self.slots.append(s)

    def warmup(self, sample: np.ndarray, ks=(1,), max_batch: int = 1):
        """Launches on every slot before timing starts, one per k in `ks` and
        one of `max_batch` queries: the first use of a stream allocates its
        per-stream scratch, and the first launch of each kernel variant (they
        differ by the batch's largest k) loads it."""
        mb = max(1, int(max_batch))  # within the slots' capacity
        sizes = sorted({min(b, mb) for b in (1, 9, 17, mb)})  # the scan's queries per wave change at 9 and 17
        for k in ks:
            for b in sizes:
                reps = -(-b // sample.shape[0])
                rows = np.concatenate([sample] * reps, axis=0)[:b]
                for s in self.slots:
                    self.launch(s, [Request(-1, 0.0, rows, int(k))])
                self.torch.cuda.synchronize()
                for s in self.slots:
                    s["batch"] = None

    def free_slot(self):
        for s in self.slots:
            if s["batch"] is None:
                return s
        return None

    def launch(self, slot, batch: List[Request]):
        torch = self.torch
        nq = sum(r.b for r in batch)
        q_np = slot["q_host"].numpy()
        k_np = slot["k_host"].numpy()
        off_np = slot["off_host"].numpy()
        row = 0
        kmax = 1
        for r in batch:
            qs = r.queries if r.queries.dtype != np.uint16 else r.queries.view(np.int16)
            q_np[row:row + r.b] = qs
            k_np[row:row + r.b] = r.k
            kmax = max(kmax, r.k)
            row += r.b
        off_np[0] = 0
        np.cumsum(k_np[:nq], out=off_np[1:nq + 1])
        total = int(off_np[nq])
        st = slot["stream"]
        with torch.cuda.stream(st):
            slot["q_dev"][:nq].copy_(slot["q_host"][:nq], non_blocking=True)
            slot["k_dev"][:nq].copy_(slot["k_host"][:nq], non_blocking=True)
            slot["off_dev"][:nq + 1].copy_(slot["off_host"][:nq + 1], non_blocking=True)
            self.index.topk_dev(slot["q_dev"][:nq], slot["k_dev"], slot["off_dev"], kmax, slot["ids_dev"],
                                slot["lcp_dev"], stream=st, scan=self.scan)
            slot["ids_host"][:total].copy_(slot["ids_dev"][:total], non_blocking=True)
            slot["lcp_host"][:total].copy_(slot["lcp_dev"][:total], non_blocking=True)
            slot["event"].record(st)
        slot["batch"] = batch
        slot["nq"] = nq

    def poll(self, now_fn) -> List[Request]:
        done: List[Request] = []
        for s in self.slots:
            if s["batch"] is not None and s["event"].query():
                t = now_fn()
                ids = s["ids_host"].numpy()
                lcps = s["lcp_host"].numpy()
                pos = 0
                for r in s["batch"]:
                    n = r.b * r.k
                    r.ids = ids[pos:pos + n].reshape(r.b, r.k).copy()
                    r.lcps = lcps[pos:pos + n].reshape(r.b, r.k).copy()
                    r.done = t
                    pos += n
                    done.append(r)
                s["batch"] = None
        return done

    def busy(self) -> bool:
        return any(s["batch"] is not None for s in self.slots)


def run_loop(requests: List[Request], scheduler: Scheduler, executor, clock=None, max_wall_s: float = 600.0):
    """Open-loop driver: requests are released at their arrival times; free
    slots are refilled as soon as they drain.  Returns the completed requests.

    `clock` is a callable giving seconds since the start (real time by default);
    a fake executor may supply a virtual clock that jumps between events.
    """
    if clock is None:
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
    order = sorted(requests, key=lambda r: (r.arrival, r.rid))
    i = 0
    finished: List[Request] = []
    start = clock()
    while i < len(order) or len(scheduler) or executor.busy():
        now = clock()
        while i < len(order) and order[i].arrival <= now:
            scheduler.submit(order[i])
            i += 1
        while len(scheduler):
            slot = executor.free_slot()
            if slot is None:
                break
            batch = scheduler.next_batch()
            if not batch:
                break
            executor.launch(slot, batch)
        finished.extend(executor.poll(clock))
        if clock() - start > max_wall_s:
            raise RuntimeError("serving loop exceeded its wall-time limit")
        if hasattr(executor, "advance"):
            executor.advance(order[i].arrival if i < len(order) else None)
    return finished


def latency_report(done: List[Request], duration_s: float) -> dict:
    lat = np.array([(r.done - r.arrival) * 1e3 for r in done])
    nq = sum(r.b for r in done)
    span = max(r.done for r in done) if done else 0.0
    return {
        "requests": len(done),
        "queries": int(nq),
        "offered_s": round(duration_s, 3),
        "achieved_qps": round(nq / max(span, 1e-9), 1),
        "p50_ms": round(float(np.percentile(lat, 50)), 4) if len(lat) else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 4) if len(lat) else None,
        "max_ms": round(float(lat.max()), 4) if len(lat) else None,
    }


def requests_from_schedule(query_pool: np.ndarray, arrival_s, batch_sizes, ks) -> List[Request]:
    """Requests for an arrival schedule; request i takes the next batch_sizes[i]
    rows of the query pool (cycling)."""
    reqs = []
    pos = 0
    n = query_pool.shape[0]
    for i in range(len(arrival_s)):
        b = int(batch_sizes[i])
        sel = (np.arange(b) + pos) % n
        pos = (pos + b) % n
        reqs.append(Request(i, float(arrival_s[i]), query_pool[sel], int(ks[i])))
    return reqs


def _variant_ks(requests) -> List[int]:
    """The largest k of each kernel variant the requests use (the per-query
    list grows at k = 65, 129 and 257; a launch with the largest k of a
    variant also sizes per-stream scratch for every smaller one)."""
    best = {}
    for r in requests:
        v = 0 if r.k <= 64 else 1 if r.k <= 128 else 2 if r.k <= 256 else 3
        best[v] = max(best.get(v, 1), int(r.k))
    return [best[v] for v in sorted(best)]


def _without_gc(fn):
    """Run fn with Python's cyclic garbage collector paused (a collection in
    the middle of a timed loop shows up as a latency spike)."""
    import gc
    was = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        return fn()
    finally:
        if was:
            gc.enable()


def run_served(index, requests: List[Request], n_slots: int = 3, budget_bytes: int = 1 << 30,
               cap_queries: int = 8192, scan: bool = False) -> dict:
    """Continuous batching over `n_slots` streams under a device-memory budget;
    returns the latency report (requests are filled in with their answers)."""
    row_bytes = index.L * index.token_bytes
    kmax = max((r.k for r in requests), default=1)
    cq, ce = slot_capacities(budget_bytes, n_slots, row_bytes, k_max=max(kmax, 1))
    cq = min(cq, cap_queries)
    ce = min(ce, cq * kmax)
    ex = GpuExecutor(index, n_slots, cq, ce, scan=scan)
    if requests:
        bmax = min(max(r.b for r in requests), cq, ce // max(kmax, 1))
        ex.warmup(requests[0].queries, ks=_variant_ks(requests), max_batch=bmax)
    sched = Scheduler(cq, ce)
    duration = max((r.arrival for r in requests), default=0.0)
    done = _without_gc(lambda: run_loop(requests, sched, ex))
    rep = latency_report(done, duration)
    rep["slots"] = n_slots
    rep["path"] = "scan" if scan else "index"
    rep["mode"] = "continuous batching"
    return rep


def run_synchronous(index, requests: List[Request], scan: bool = True, max_wall_s: float = 120.0) -> dict:
    """Baseline: one request per call, each call waited for before the next
    (no batching, no overlap).  Requests that arrive while a call runs queue."""
    import torch
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0  # noqa: E731
    done = []
    fn = index.scan_topk if scan else index.topk
    if requests:  # the same warm-up as the batched executor gets: every kernel variant and batch shape
        bmax = max(r.b for r in requests)
        sample = requests[0].queries
        for kk in _variant_ks(requests):
            for b in sorted({1, min(9, bmax), min(17, bmax), bmax}):
                rows = np.concatenate([sample] * (-(-b // sample.shape[0])), axis=0)[:b]
                fn(rows, kk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()

    def loop():
        for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
            while clock() < r.arrival:
                pass
            res = fn(r.queries, r.k)
            torch.cuda.synchronize()
            r.ids = res.ids.cpu().numpy().reshape(r.b, r.k)
            r.lcps = res.lcps.cpu().numpy().reshape(r.b, r.k)
            r.done = clock()
            done.append(r)
            if clock() > max_wall_s:
                break

    loop()
    duration = max((r.arrival for r in requests), default=0.0)
    rep = latency_report(done, duration)
    rep["path"] = "scan" if scan else "index"
    rep["mode"] = "synchronous, one request per call"
    rep["completed_fraction"] = round(len(done) / max(len(requests), 1), 4)
    return rep


def run_step_stream(index, steps, rate_hz: float, k: int, append_every: int = 0, append=None,
                    max_wall_s: float = 120.0, keep=None) -> dict:
    """Paced stream of query batches (the GNC loop of section 7, Table "GNC
    benchmark": each step queries the current readings of every sensor).

    steps        : iterable of [S, L] token arrays, one batch per step
    rate_hz      : target step rate; step t is released at t / rate_hz (None or
                   0: unpaced, each step released when the previous one is done)
    append_every : every that many steps, `append(index, batch)` is called with
                   the step's batch and must return the index to use next
                   (rows join the database with the next ids)
    keep         : optional predicate on the step number; the answers of the
                   steps it accepts are returned under "answers" as
                   {t: (ids [S, k], lcps [S, k])} (copied after the step's
                   latency is taken)
    Returns the achieved step rate and step latency percentiles (latency =
    completion - release time, so a late step also delays the next ones).
    """
    import torch
    dev = index.device
    lat = []
    appends_ms = []
    kept = {}
    buf = {}
    t0 = time.perf_counter()
    n = 0
    for t, batch in enumerate(steps):
        if rate_hz:
            release = t / rate_hz
            while time.perf_counter() - t0 < release:
                pass
        else:  # unpaced: each step is released when the previous one is done
            release = time.perf_counter() - t0
        raw = np.ascontiguousarray(batch if batch.dtype != np.uint16 else batch.view(np.int16))
        if buf.get("shape") != raw.shape:  # pinned staging and outputs, reused across steps
            qdt = torch.uint8 if raw.dtype == np.uint8 else torch.int16
            buf = {"shape": raw.shape,
                   "qh": torch.empty(raw.shape, dtype=qdt, pin_memory=True),
                   "qd": torch.empty(raw.shape, dtype=qdt, device=dev),
                   "ids": torch.empty(raw.shape[0] * k, dtype=torch.int32, device=dev),
                   "lcp": torch.empty(raw.shape[0] * k, dtype=torch.int32, device=dev),
                   "ids_h": torch.empty(raw.shape[0] * k, dtype=torch.int32, pin_memory=True),
                   "lcp_h": torch.empty(raw.shape[0] * k, dtype=torch.int32, pin_memory=True)}
        buf["qh"].numpy()[:] = raw
        buf["qd"].copy_(buf["qh"], non_blocking=True)
        index.topk(buf["qd"], k, out=(buf["ids"], buf["lcp"]))
        buf["ids_h"].copy_(buf["ids"], non_blocking=True)
        buf["lcp_h"].copy_(buf["lcp"], non_blocking=True)
        torch.cuda.current_stream().synchronize()
        done = time.perf_counter() - t0
        lat.append((done - release) * 1e3)
        n += 1
        if keep is not None and keep(t):
            kept[t] = (buf["ids_h"].numpy().reshape(-1, k).copy(), buf["lcp_h"].numpy().reshape(-1, k).copy())
        if append_every and append is not None and (t + 1) % append_every == 0:
            a0 = time.perf_counter()
            index = append(index, batch)
            torch.cuda.synchronize()
            appends_ms.append((time.perf_counter() - a0) * 1e3)
        if done > max_wall_s:
            break
    wall = time.perf_counter() - t0
    lat = np.asarray(lat)
    return {
        "steps": n,
        "target_hz": rate_hz,
        "achieved_hz": round(n / wall, 1),
        "p50_step_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_step_ms": round(float(np.percentile(lat, 99)), 4),
        "max_step_ms": round(float(lat.max()), 4),
        "appends": len(appends_ms),
        "append_ms_mean": round(float(np.mean(appends_ms)), 3) if appends_ms else None,
        "append_ms": [round(x, 3) for x in appends_ms],
        "index": index,
        **({"answers": kept} if keep is not None else {}),
    }
