"""Uneven query batches in one HIP-graph-captured launch.

A batch mixes queries of different k (and, through the data, tied blocks of
very different lengths).  `CapturedLaunch` captures one device-counted
index-path launch (`lcp_topk_persistent`: the batch size is read on the
device) into a HIP graph over fixed buffers; each batch is copied into those
buffers and the graph is replayed, so a launch costs one graph replay whatever
its size (up to the capacity) and its mix of k.  By default the captured grid
has one wave per query of the capacity; a smaller persistent grid, whose waves
loop over queries from a device work counter, can be chosen instead.

`tune_launch` is the autotuner: it times the plain launch, the one-wave-per-
query counted launch and persistent grids of several sizes, each with the
queries in their own order and with the largest k first, on a sample batch,
and returns the fastest shape.

Query order.  Every query's answer goes to its own offset, so a batch may be
launched in any order of its queries without moving the answers: staging the
queries, their k and their offsets in the same permuted order leaves the
output layout as it is.  With the largest k first, the longest waves start
first and the short ones fill the device at the end of the launch (longest-
processing-time-first order).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import torch

__all__ = ["CapturedLaunch", "LaunchShape", "tune_launch", "split_by_k"]


@dataclasses.dataclass
class LaunchShape:
    mode: str          # "plain", "counted" (one wave per query) or "persistent" (waves loop)
    blocks: int = 0    # grid size in blocks of 4 waves (0 = one wave per query)
    ms: float = float("nan")
    order: str = "given"  # "given" or "k_desc" (largest k first)


def launch_order(k, n: int, order: str) -> Optional[np.ndarray]:
    """The permutation a shape launches the batch in (None: as given).
    Stable, so equal k keep their relative order."""
    if order == "given":
        return None
    if order != "k_desc":
        raise ValueError(f"unknown query order {order!r}")
    ks = np.broadcast_to(np.asarray(k, dtype=np.int32), (n,))
    return np.argsort(-ks, kind="stable")


class CapturedLaunch:
    """Device-counted index-path launch captured once, replayed per batch.

    cap_queries : largest batch; k_max : largest k any batch may use;
    blocks : 0 for one wave per query of the capacity, else a persistent grid.
    The object owns its stream; replays run on that stream in order.  The graph
    holds the index's arrays as they were at capture, so `run` refuses to
    replay it once the index has been appended to (its generation changed).  Per-batch
    k, offsets and size go up in one copy from one of two pinned staging
    buffers, so the host fills the next batch while the previous one runs.
    """

    def __init__(self, index, cap_queries: int, k_max: int, blocks: int = 0):
        self.index = index
        self.cap = int(cap_queries)
        self.k_max = int(k_max)
        dev = index.device
        qdt = torch.uint8 if index.token_bytes == 1 else torch.int16
        self.stream = torch.cuda.Stream(device=dev)
        self.q = torch.zeros((self.cap, index.L), dtype=qdt, device=dev)
        # staging layout (bytes): [count int64][off int64 x (cap+1)][k int32 x cap]
        self._nbytes = 8 + 8 * (self.cap + 1) + 4 * self.cap
        self.dbuf = torch.zeros(self._nbytes, dtype=torch.uint8, device=dev)
        self.count, self.off, self.k = self._views(self.dbuf)
        self.k.fill_(1)
        self.hbufs = [torch.zeros(self._nbytes, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.hviews = [self._views(h) for h in self.hbufs]
        self.staged = [torch.cuda.Event(), torch.cuda.Event()]  # copy out of pinned buffer i done
        for e in self.staged:
            e.record(torch.cuda.current_stream(dev))
        self.turn = 0
        self.ids = torch.empty(self.cap * self.k_max, dtype=torch.int32, device=dev)
        self.lcps = torch.empty(self.cap * self.k_max, dtype=torch.int32, device=dev)
        self.blocks = int(blocks)
        torch.cuda.synchronize(dev)
        with torch.cuda.stream(self.stream):  # first call on the stream sets up its work counter
            self._launch()
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        self.generation = index.generation()  # the index's arrays are baked into the graph
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._launch()
        self.stream.synchronize()

    def _views(self, buf):
        c = 8 + 8 * (self.cap + 1)
        return buf[0:8].view(torch.int64), buf[8:c].view(torch.int64), buf[c:c + 4 * self.cap].view(torch.int32)

    def _launch(self):
        self.index.topk_persistent(self.q, self.count, self.k, self.off, self.k_max, self.ids, self.lcps,
                                   blocks=self.blocks, stream=self.stream)

    def stage(self, k, n: int, order: Optional[np.ndarray] = None) -> np.ndarray:
        """Put a batch's size, offsets and k into the device buffers ahead of a
        replay (for producers that prepare batches before they are due);
        returns the offsets of the answers (in the batch's own order).  The
        queries go into the first n rows of `self.q`; with `order`, row j
        holds query order[j] and the answers still land at the batch's own
        offsets."""
        if self.index.generation() != self.generation:
            raise RuntimeError("the index has been appended to since this launch was captured; capture it again")
        n = int(n)
        if n > self.cap:
            raise ValueError(f"batch of {n} exceeds the captured capacity {self.cap}")
        ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
        if n and (ks.min() < 1 or ks.max() > self.k_max):
            raise ValueError(f"k must lie in [1, {self.k_max}]")
        off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(ks, out=off[1:])
        host = torch.zeros(self._nbytes, dtype=torch.uint8)
        hc, ho, hk = (v.numpy() for v in self._views(host))
        hc[0] = n
        if order is None:
            ho[:n + 1] = off
            hk[:n] = ks
        else:
            ho[:n] = off[:n][order]
            ho[n] = off[n]
            hk[:n] = ks[order]
        with torch.cuda.stream(self.stream):
            self.dbuf.copy_(host.to(self.dbuf.device))
        self.stream.synchronize()
        return off

    def replay(self, events=None):
        """Replay the captured launch on the batch already staged (see `stage`)."""
        if self.index.generation() != self.generation:
            raise RuntimeError("the index has been appended to since this launch was captured; capture it again")
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            if events is not None:
                events[0].record(self.stream)
            self.graph.replay()
            if events is not None:
                events[1].record(self.stream)
        cur.wait_stream(self.stream)

    def run(self, queries: Optional[torch.Tensor], k, n: Optional[int] = None,
            events=None, order: Optional[np.ndarray] = None) -> "tuple[torch.Tensor, torch.Tensor, np.ndarray]":
        """Answer `queries` (device [n, L]) with per-query k (host); returns
        (ids, lcps, offsets) views valid until the next run, in the batch's
        own order.  With queries None the first n rows of `self.q`, filled
        by the caller, are used (row j holding query order[j] when an order
        is given).  With `order` the queries are launched in that order (see
        `launch_order`).  `events` = (start, end) are recorded around the
        device work."""
        if self.index.generation() != self.generation:
            raise RuntimeError("the index has been appended to since this launch was captured; capture it again")
        n = int(queries.shape[0]) if queries is not None else int(n)
        if n > self.cap:
            raise ValueError(f"batch of {n} exceeds the captured capacity {self.cap}")
        ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
        if n and (ks.min() < 1 or ks.max() > self.k_max):
            raise ValueError(f"k must lie in [1, {self.k_max}]")
        t = self.turn
        self.turn ^= 1
        self.staged[t].synchronize()  # the copy of two runs ago has left this buffer
        hc, ho, hk = (v.numpy() for v in self.hviews[t])
        hc[0] = n
        ho[0] = 0
        np.cumsum(ks, out=ho[1:n + 1])
        hk[:n] = ks
        answer_off = ho[:n + 1].copy()
        if order is not None:
            ho[:n] = answer_off[:n][order]
            hk[:n] = ks[order]
            if queries is not None:
                queries = queries[torch.from_numpy(np.asarray(order)).to(queries.device)]
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)  # the queries were produced on the caller's stream
        with torch.cuda.stream(self.stream):
            if events is not None:
                events[0].record(self.stream)
            if n and queries is not None:
                self.q[:n].copy_(queries, non_blocking=True)
            self.dbuf.copy_(self.hbufs[t], non_blocking=True)
            self.staged[t].record(self.stream)
            self.graph.replay()
            if events is not None:
                events[1].record(self.stream)
        cur.wait_stream(self.stream)
        total = int(answer_off[n])
        return self.ids[:total], self.lcps[:total], answer_off


def _time_ms(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def shape_inputs(queries: torch.Tensor, k, order: str):
    """(queries, k, offsets) on the device as a shape launches them: in the
    shape's query order, each query's offset still its place in the batch's
    own answer layout."""
    n = int(queries.shape[0])
    ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(ks, out=off[1:])
    perm = launch_order(ks, n, order)
    dev = queries.device
    if perm is None:
        return queries, torch.from_numpy(ks).to(dev), torch.from_numpy(off).to(dev)
    po = np.append(off[:n][perm], off[n])
    pt = torch.from_numpy(perm).to(dev)
    return queries[pt].contiguous(), torch.from_numpy(ks[perm].copy()).to(dev), torch.from_numpy(po).to(dev)


def run_shape(index, sh: LaunchShape, inputs, kmax: int, ids: torch.Tensor, lcps: torch.Tensor,
              count: torch.Tensor) -> None:
    """One launch of shape `sh` on `shape_inputs(...)` for its order."""
    q, k_dev, off_dev = inputs
    if sh.mode == "plain":
        index.topk_dev(q, k_dev, off_dev, kmax, ids, lcps)
    else:
        index.topk_persistent(q, count, k_dev, off_dev, kmax, ids, lcps, blocks=sh.blocks)


def tune_launch(index, queries: torch.Tensor, k, reps: int = 7, cus: Optional[int] = None) -> Dict:
    """Time the plain launch, the one-wave-per-query counted launch and
    persistent grids of 1, 2 and 4 blocks per CU on one batch, each with the
    queries in their given order and with the largest k first; return
    {"best": LaunchShape, "tried": [LaunchShape, ...]}."""
    n = int(queries.shape[0])
    ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
    kmax = int(ks.max())
    dev = index.device
    count = torch.tensor([n], dtype=torch.int64, device=dev)
    ids = torch.empty(int(ks.sum()), dtype=torch.int32, device=dev)
    lcps = torch.empty_like(ids)
    if cus is None:
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
    shapes = [LaunchShape("plain", 0), LaunchShape("counted", 0)]
    shapes += [LaunchShape("persistent", cus * m) for m in (1, 2, 4) if 4 * cus * m < n]  # larger: the counted launch
    tried: List[LaunchShape] = []
    for order in ("given", "k_desc"):
        inputs = shape_inputs(queries, ks, order)
        for base in shapes:
            sh = LaunchShape(base.mode, base.blocks, order=order)
            sh.ms = _time_ms(lambda: run_shape(index, sh, inputs, kmax, ids, lcps, count), reps)
            tried.append(sh)
    best = min(tried, key=lambda s: s.ms)
    return {"best": best, "tried": tried}


def split_by_k(ks: np.ndarray) -> Dict[int, np.ndarray]:
    """Query indices grouped by k (for per-bucket launches)."""
    out = {}
    for kv in np.unique(ks):
        out[int(kv)] = np.nonzero(ks == kv)[0]
    return out
