"""Seeded synthetic workloads for exact top-k LCP retrieval.

This module only draws random token sequences, query sets, per-query k values
and request arrival schedules.  It contains none of the retrieval arithmetic
(no prefix comparison, no ordering, no selection), so both the CPU oracle and
the GPU path can take their inputs from it without sharing any method code.

The paper evaluates on synthetic data only and does not give a distribution
(Appendix "Availability and Reproducibility"); the five workloads below follow
the shapes of its experiments (section 7: OOM wall at N=500K, the 2M-candidate
sustained load, the GNC sensor-fusion stream) with the concrete recipes stated
in each function's docstring.

Every generator is a pure function of its seed: the random streams come from
``numpy.random.SeedSequence(base_seed).spawn(...)`` and are consumed in a fixed
order, so the arrays are byte-identical across runs of the same NumPy version.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Iterator

import numpy as np

__all__ = [
    "Workload",
    "prototype_rows",
    "c1_tiny",
    "c2_oom_boundary",
    "c3_hierarchy",
    "c3_like",
    "serving_schedule",
    "SensorStream",
    "c5_sensor",
    "random_rows",
    "sha256_of",
    "uneven_k",
    "long_ties",
]


@dataclasses.dataclass
class Workload:
    """A database, a query batch and per-query k (all host NumPy arrays).

    db      : [N, L] uint8 or uint16 token matrix; row i has id i.
    queries : [Q, L] same dtype.
    k       : [Q] int32, each >= 1.
    V       : vocabulary size; every db token is < V.
    """

    name: str
    db: np.ndarray
    queries: np.ndarray
    k: np.ndarray
    V: int
    extras: dict = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.db.shape[0])

    @property
    def L(self) -> int:
        return int(self.db.shape[1])

    @property
    def Q(self) -> int:
        return int(self.queries.shape[0])


def sha256_of(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _streams(base_seed: int, n: int = 4):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(base_seed).spawn(n)]


def _dtype_for(V: int):
    return np.uint8 if V <= 256 else np.uint16


def prototype_rows(rng: np.random.Generator, protos: np.ndarray, n: int, p: float, V: int) -> np.ndarray:
    """Rows that copy a random prototype's first m tokens, m = min(G, L).

    G ~ Geometric(p) on {0, 1, 2, ...}; the remaining L - m tokens are uniform
    in [0, V).  Draw order: prototype pick, m, fill tokens.
    """
    P, L = protos.shape
    pick = rng.integers(0, P, size=n)
    m = np.minimum(rng.geometric(p, size=n) - 1, L)
    fill = rng.integers(0, V, size=(n, L), dtype=np.int64).astype(protos.dtype)
    keep = np.arange(L)[None, :] < m[:, None]
    return np.where(keep, protos[pick], fill)


def _prototype_workload(name, seed, N, L, V, n_protos, p, n_gen, n_copies, k):
    r_db, r_q, r_k, _ = _streams(seed)
    dt = _dtype_for(V)
    protos = r_db.integers(0, V, size=(n_protos, L), dtype=np.int64).astype(dt)
    db = prototype_rows(r_db, protos, N, p, V)
    gen = prototype_rows(r_q, protos, n_gen, p, V)
    copy_ids = r_q.choice(N, size=n_copies, replace=False)
    queries = np.concatenate([gen, db[copy_ids]], axis=0)
    kk = np.full(queries.shape[0], k, dtype=np.int32)
    return Workload(name, np.ascontiguousarray(db), np.ascontiguousarray(queries), kk, V,
                    {"copy_ids": copy_ids.astype(np.int64), "n_generated": n_gen})


def c1_tiny(seed: int = 1001) -> Workload:
    """N=10,000, L=16 uint8, V=16; 64 prototypes, Geometric(0.15);
    1,000 generated queries + 100 exact copies of database rows; k=10."""
    return _prototype_workload("c1_tiny", seed, 10_000, 16, 16, 64, 0.15, 1000, 100, 10)


def c2_oom_boundary(seed: int = 1002, n_gen: int = 9000, n_copies: int = 1000) -> Workload:
    """N=500,000, L=64 uint8, V=256; 4,096 prototypes, Geometric(0.05);
    9,000 generated queries + 1,000 copies (10%); k=10."""
    return _prototype_workload("c2_oom_boundary", seed, 500_000, 64, 256, 4096, 0.05,
                               n_gen, n_copies, 10)


def _zipf_cdf(V: int, s: float) -> np.ndarray:
    w = 1.0 / np.arange(1, V + 1, dtype=np.float64) ** s
    return np.cumsum(w) / w.sum()


class _Hierarchy:
    """3-level random tree (branching b0/b1/b2) over the first three positions,
    then i.i.d. bounded Zipf(s) tokens (rank r -> token r-1) at the others.
    Sibling labels are distinct uniform draws from [0, V)."""

    def __init__(self, rng, V=4096, branching=(16, 16, 16), s=1.1):
        b0, b1, b2 = branching
        self.V = V
        self.branching = branching
        self.l0 = rng.choice(V, size=b0, replace=False)
        self.l1 = np.stack([rng.choice(V, size=b1, replace=False) for _ in range(b0)])
        self.l2 = np.stack([np.stack([rng.choice(V, size=b2, replace=False) for _ in range(b1)])
                            for _ in range(b0)])
        self.cdf = _zipf_cdf(V, s)

    def rows(self, rng, n, L=32):
        b0, b1, b2 = self.branching
        out = np.empty((n, L), dtype=_dtype_for(self.V))
        path = np.stack([rng.integers(0, b0, n), rng.integers(0, b1, n), rng.integers(0, b2, n)], 1)
        out[:, 0] = self.l0[path[:, 0]]
        out[:, 1] = self.l1[path[:, 0], path[:, 1]]
        out[:, 2] = self.l2[path[:, 0], path[:, 1], path[:, 2]]
        # inverse-CDF sampling in slabs to bound the float64 temporary
        slab = 1 << 18
        for s0 in range(0, n, slab):
            u = rng.random((min(slab, n - s0), L - 3))
            t = np.searchsorted(self.cdf, u, side="right")
            out[s0:s0 + u.shape[0], 3:] = np.minimum(t, self.V - 1)
        return out


def c3_like(N: int, Q: int, seed: int = 1003, k_choices=(1, 10, 100), k_fixed: int | None = None,
            L: int = 32, V: int = 4096, branching=(16, 16, 16)) -> Workload:
    """The 3-level hierarchy workload at an arbitrary size (same recipe as c3)."""
    r_db, r_q, r_k, _ = _streams(seed)
    h = _Hierarchy(r_db, V=V, branching=branching)
    db = h.rows(r_db, N, L)
    queries = h.rows(r_q, Q, L)
    if k_fixed is not None:
        kk = np.full(Q, k_fixed, dtype=np.int32)
    else:
        kk = np.asarray(k_choices, dtype=np.int32)[r_k.integers(0, len(k_choices), Q)]
    return Workload(f"c3_like_N{N}", db, queries, kk, V, {"hierarchy": h})


def c3_hierarchy(seed: int = 1003, Q: int = 8192, k_fixed: int | None = None) -> Workload:
    """N=2,000,000, L=32 uint16, V=4,096: 16/16/16 random hierarchy over
    positions 0-2, Zipf(s=1.1) tokens after; 8,192 queries from the same
    generator with k uniform on {1, 10, 100} (or k_fixed for every query)."""
    w = c3_like(2_000_000, Q, seed=seed, k_fixed=k_fixed)
    w.name = "c3_hierarchy"
    return w


def serving_schedule(rate_qps: float, duration_s: float, seed: int = 1004,
                     k_mode: str = "uniform", k_fixed: int = 10, max_batch: int = 256):
    """Poisson request arrivals for the serving loop.

    Batch size b = floor(exp(U * ln(max_batch + 1))) in [1, max_batch]
    (log-uniform); request rate = rate_qps / E[b]; k uniform on [1, 100] per
    request (k_mode="uniform") or k_fixed.  Returns (arrival_s, batch, k).
    """
    _, _, r_k, r_a = _streams(seed)
    lnb = math.log(max_batch + 1)
    # E[floor(exp(U ln(B+1)))] computed exactly over the integer support
    support = np.arange(1, max_batch + 1)
    probs = (np.log(support + 1) - np.log(support)) / lnb
    eb = float((support * probs).sum())
    lam = rate_qps / eb
    n_est = int(lam * duration_s * 1.2) + 16
    gaps = r_a.exponential(1.0 / lam, size=n_est)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    n = t.shape[0]
    b = np.floor(np.exp(r_a.random(n) * lnb)).astype(np.int64)
    b = np.clip(b, 1, max_batch)
    if k_mode == "uniform":
        k = r_k.integers(1, 101, size=n).astype(np.int32)
    else:
        k = np.full(n, k_fixed, dtype=np.int32)
    return t, b, k


class SensorStream:
    """GNC sensor-fusion stream: 1,000 sensors, L=24 uint8 tokens, V=16.

    Row layout: [type (8 values), subsystem hi (sub >> 4), subsystem lo
    (sub & 15), 21 quantised channel values (16 levels)].  Each channel starts
    uniform in [0,16) and moves by clamp(v + d, 0, 15) with d uniform in
    {-1, 0, +1} at every step.  Row id of sensor s at step t is t*S + s.
    """

    L = 24
    V = 16

    def __init__(self, seed: int = 1005, sensors: int = 1000, channels: int = 21):
        r_static, r_walk, _, _ = _streams(seed)
        self.S = sensors
        self.C = channels
        self.type = r_static.integers(0, 8, sensors)
        self.sub = r_static.integers(0, 128, sensors)
        self.vals = r_static.integers(0, 16, (sensors, channels))
        self._rng = r_walk
        self.t = 0

    def step(self) -> np.ndarray:
        """Readings at the current step (then advance the random walk)."""
        rows = np.empty((self.S, self.L), dtype=np.uint8)
        rows[:, 0] = self.type
        rows[:, 1] = self.sub >> 4
        rows[:, 2] = self.sub & 15
        rows[:, 3:] = self.vals
        d = self._rng.integers(-1, 2, (self.S, self.C))
        self.vals = np.clip(self.vals + d, 0, 15)
        self.t += 1
        return rows

    def steps(self, n: int) -> Iterator[np.ndarray]:
        for _ in range(n):
            yield self.step()


def c5_sensor(seed: int = 1005, history_steps: int = 1000, sensors: int = 1000,
              query_steps: int = 1) -> Workload:
    """History of `history_steps` steps (N = steps * sensors rows, id = t*S+s),
    queries = the readings of the next `query_steps` steps, k = 5."""
    st = SensorStream(seed, sensors)
    hist = np.concatenate(list(st.steps(history_steps)), axis=0)
    qs = np.concatenate(list(st.steps(query_steps)), axis=0)
    kk = np.full(qs.shape[0], 5, dtype=np.int32)
    return Workload("c5_sensor", hist, qs, kk, SensorStream.V, {"stream": st})


def random_rows(rng: np.random.Generator, n: int, L: int, V: int, dtype=None) -> np.ndarray:
    """Uniform tokens in [0, V)."""
    dt = dtype or _dtype_for(V)
    return rng.integers(0, V, size=(n, L), dtype=np.int64).astype(dt)


def uneven_k(Q: int, seed: int = 1013, choices=(1, 10, 100)) -> np.ndarray:
    """Per-query k drawn uniformly from `choices` (the uneven-batch workload)."""
    rng = np.random.default_rng(seed)
    return np.asarray(choices, dtype=np.int32)[rng.integers(0, len(choices), Q)]


def long_ties(seed: int = 1021, N: int = 400_000, L: int = 8, Q: int = 512,
              probs=(0.80, 0.15, 0.002, 0.048), k_choices=(1, 10, 54, 100, 250)) -> Workload:
    """Heavily duplicated rows, so that the rows tied at the cutoff LCP number
    in the thousands to hundreds of thousands.

    Every db token is i.i.d. over V=4 symbols with probabilities `probs`
    (symbol 0 dominant).  Queries, in this order: Q/8 all-zero rows; Q/8 rows
    0^(L-1) 2 (few exact matches, with the rows of last token 3 sorted after
    them and those of tokens 0 and 1 before, so rows tied one level up sit on
    both sides of them); Q/4 rows 0^j x
    then zeros, j uniform in [0, L), x uniform in {1, 2, 3}; Q/4 copies of
    random db rows; the rest fresh draws from the db distribution.  k uniform
    on `k_choices`.
    """
    r_db, r_q, r_k, _ = _streams(seed)
    db = r_db.choice(4, size=(N, L), p=np.asarray(probs)).astype(np.uint8)
    n8, n4 = Q // 8, Q // 4
    zeros = np.zeros((n8, L), dtype=np.uint8)
    both = np.zeros((n8, L), dtype=np.uint8)
    both[:, L - 1] = 2
    step = np.zeros((n4, L), dtype=np.uint8)
    j = r_q.integers(0, L, n4)
    step[np.arange(n4), j] = r_q.integers(1, 4, n4)
    copies = db[r_q.choice(N, size=n4, replace=False)]
    fresh = r_q.choice(4, size=(Q - 2 * n8 - 2 * n4, L), p=np.asarray(probs)).astype(np.uint8)
    queries = np.ascontiguousarray(np.concatenate([zeros, both, step, copies, fresh], axis=0))
    kk = np.asarray(k_choices, dtype=np.int32)[r_k.integers(0, len(k_choices), Q)]
    return Workload("long_ties", np.ascontiguousarray(db), queries, kk, 4)
