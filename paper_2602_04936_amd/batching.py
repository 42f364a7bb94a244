"""Uneven query batches in one persistent, HIP-graph-captured launch.

A batch mixes queries of different k (and, through the data, tied blocks of
very different lengths).  `CapturedLaunch` captures one persistent index-path
launch (`lcp_topk_persistent`: a grid that fills the device, waves taking
queries from a device counter, the batch size read on the device) into a HIP
graph over fixed buffers; each batch is copied into those buffers and the graph
is replayed, so a launch costs one graph replay whatever its size (up to the
capacity) and its mix of k.

`tune_launch` is the autotuner: it times the plain launch (one wave per query)
and persistent launches of several grid sizes on a sample batch and returns
the fastest shape.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import torch

__all__ = ["CapturedLaunch", "LaunchShape", "tune_launch", "split_by_k"]


@dataclasses.dataclass
class LaunchShape:
    mode: str          # "plain" (one wave per query) or "persistent"
    blocks: int = 0    # persistent grid size (0 = library default)
    ms: float = float("nan")


class CapturedLaunch:
    """Persistent index-path launch captured once, replayed per batch.

    cap_queries : largest batch; k_max : largest k any batch may use.
    The object owns its stream; replays run on that stream and must not
    overlap each other (they share the device work counter).
    """

    def __init__(self, index, cap_queries: int, k_max: int, blocks: int = 0):
        self.index = index
        self.cap = int(cap_queries)
        self.k_max = int(k_max)
        dev = index.device
        qdt = torch.uint8 if index.token_bytes == 1 else torch.int16
        self.stream = torch.cuda.Stream(device=dev)
        self.q = torch.zeros((self.cap, index.L), dtype=qdt, device=dev)
        self.k = torch.ones(self.cap, dtype=torch.int32, device=dev)
        self.off = torch.zeros(self.cap + 1, dtype=torch.int64, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ids = torch.empty(self.cap * self.k_max, dtype=torch.int32, device=dev)
        self.lcps = torch.empty(self.cap * self.k_max, dtype=torch.int32, device=dev)
        self.k_host = torch.empty(self.cap, dtype=torch.int32, pin_memory=True)
        self.off_host = torch.empty(self.cap + 1, dtype=torch.int64, pin_memory=True)
        self.count_host = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.blocks = int(blocks)
        self.staged = torch.cuda.Event()  # the last run's copies out of the pinned staging have run
        self.staged.record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize(dev)
        with torch.cuda.stream(self.stream):  # first call on the stream sets up its work counter
            self._launch()
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._launch()
        self.stream.synchronize()

    def _launch(self):
        self.index.topk_persistent(self.q, self.count, self.k, self.off, self.k_max, self.ids, self.lcps,
                                   blocks=self.blocks, stream=self.stream)

    def run(self, queries: torch.Tensor, k) -> "tuple[torch.Tensor, torch.Tensor, np.ndarray]":
        """Answer `queries` (device [n, L]) with per-query k (host); returns
        (ids, lcps, offsets) views valid until the next run."""
        n = int(queries.shape[0])
        if n > self.cap:
            raise ValueError(f"batch of {n} exceeds the captured capacity {self.cap}")
        ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
        if n and (ks.min() < 1 or ks.max() > self.k_max):
            raise ValueError(f"k must lie in [1, {self.k_max}]")
        self.staged.synchronize()  # the previous run may still be reading the pinned staging
        kh = self.k_host.numpy()
        oh = self.off_host.numpy()
        kh[:n] = ks
        oh[0] = 0
        np.cumsum(ks, out=oh[1:n + 1])
        self.count_host.numpy()[0] = n
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)  # the queries were produced on the caller's stream
        with torch.cuda.stream(self.stream):
            if n:
                self.q[:n].copy_(queries, non_blocking=True)
                self.k[:n].copy_(self.k_host[:n], non_blocking=True)
                self.off[:n + 1].copy_(self.off_host[:n + 1], non_blocking=True)
            self.count.copy_(self.count_host, non_blocking=True)
            self.staged.record(self.stream)
            self.graph.replay()
        cur.wait_stream(self.stream)
        total = int(oh[n])
        return self.ids[:total], self.lcps[:total], oh[:n + 1].copy()


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


def tune_launch(index, queries: torch.Tensor, k, reps: int = 7, cus: Optional[int] = None) -> Dict:
    """Time the plain launch and persistent launches of several grid sizes on
    one batch; return {"best": LaunchShape, "tried": [LaunchShape, ...]}."""
    n = int(queries.shape[0])
    ks = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
    kmax = int(ks.max())
    dev = index.device
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(ks, out=off[1:])
    k_dev = torch.from_numpy(ks).to(dev)
    off_dev = torch.from_numpy(off).to(dev)
    count = torch.tensor([n], dtype=torch.int64, device=dev)
    ids = torch.empty(int(off[-1]), dtype=torch.int32, device=dev)
    lcps = torch.empty_like(ids)
    if cus is None:
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
    tried: List[LaunchShape] = []
    tried.append(LaunchShape("plain", 0, _time_ms(
        lambda: index.topk_dev(queries, k_dev, off_dev, kmax, ids, lcps), reps)))
    for mult in (1, 2, 4, 6):
        b = cus * mult
        tried.append(LaunchShape("persistent", b, _time_ms(
            lambda: index.topk_persistent(queries, count, k_dev, off_dev, kmax, ids, lcps, blocks=b), reps)))
    best = min(tried, key=lambda s: s.ms)
    return {"best": best, "tried": tried}


def split_by_k(ks: np.ndarray) -> Dict[int, np.ndarray]:
    """Query indices grouped by k (for per-bucket launches)."""
    out = {}
    for kv in np.unique(ks):
        out[int(kv)] = np.nonzero(ks == kv)[0]
    return out
