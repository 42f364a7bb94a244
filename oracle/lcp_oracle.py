"""Plain CPU oracle for exact top-k retrieval under LCP similarity.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only the test-suite, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the GPU implementation.

Everything here is written straight from the paper's definitions, favouring
"obviously correct" over fast:

* LCP similarity (section 2.1, Definition "LCP Similarity"): the length of the
  longest common prefix of two length-L sequences; 0 when the first symbols
  already differ, L when the sequences are equal.
* Top-k LCP retrieval (section 2.1, Definition "Top-k LCP Retrieval"): the k
  items of highest LCP with the query, ties broken by index.  Readings taken
  where the paper is silent: ids are 0-based row positions, ties go to the
  *lower* id, results are listed in rank order (LCP descending, id
  ascending), and when k exceeds N the list is padded with (-1, -1).
* The sorted dataset that the TAL range scan searches (Appendix D.1,
  TALRangeScan) and the trie's leaf order (section 5.2, Algorithm 1, posting
  lists kept in insertion order): rows in lexicographic order, tokens compared
  as unsigned integers with position 0 most significant, equal rows by id.
* Prefix buckets (section 6.2, Definition "Prefix Bucket"): the rows sharing a
  given length-d prefix, which form a contiguous range of the sorted order.
* The bucket range scan (section 6.2, Definition "Thermal-Aware Logic";
  Appendix D.1, TALRangeScan): a query scans only the rows of its own
  depth-d bucket, and its answer is the top-k of those rows alone.  Reading
  taken: rank order and ids as in the top-k definition, and (-1, -1) past the
  bucket's size (an empty bucket gives k pads).

All arithmetic is integer; results are exact.
"""
from __future__ import annotations

import bisect

import numpy as np

__all__ = [
    "lcp",
    "lcp_against",
    "topk",
    "topk_batch",
    "sorted_permutation",
    "adjacent_lcp",
    "lower_bound",
    "prefix_bucket",
    "bucket_topk",
    "bucket_topk_batch",
    "csr_offsets",
]


def lcp(s, t) -> int:
    """LCP similarity of two equal-length sequences (section 2.1)."""
    n = 0
    for a, b in zip(s, t):
        if int(a) != int(b):
            break
        n += 1
    return n


def lcp_against(db: np.ndarray, q: np.ndarray) -> np.ndarray:
    """LCP(q, s_i) for every row s_i of db, as int32 (section 2.1).

    The first position where row and query differ is the LCP; a row equal to
    the query has LCP = L.
    """
    db = np.asarray(db)
    q = np.asarray(q)
    L = db.shape[1]
    eq = db == q[None, :]
    first_diff = np.argmin(eq, axis=1)          # index of the first False
    return np.where(eq.all(axis=1), L, first_diff).astype(np.int32)


def topk(db: np.ndarray, q: np.ndarray, k: int):
    """Top-k LCP retrieval for one query (section 2.1).

    Returns (ids, lcps) as int32 arrays of length k: rank order by LCP
    descending then id ascending; positions past N are (-1, -1).
    """
    if k < 1:
        raise ValueError("k must be >= 1")
    v = lcp_against(db, q)
    ids = np.arange(db.shape[0], dtype=np.int64)
    order = np.lexsort((ids, -v.astype(np.int64)))   # primary: -lcp, then id
    take = order[:k]
    out_ids = np.full(k, -1, dtype=np.int32)
    out_lcp = np.full(k, -1, dtype=np.int32)
    out_ids[: take.shape[0]] = take
    out_lcp[: take.shape[0]] = v[take]
    return out_ids, out_lcp


def csr_offsets(ks) -> np.ndarray:
    ks = np.asarray(ks, dtype=np.int64)
    off = np.zeros(ks.shape[0] + 1, dtype=np.int64)
    np.cumsum(ks, out=off[1:])
    return off


def topk_batch(db: np.ndarray, queries: np.ndarray, ks):
    """Top-k for a batch; outputs concatenated in query order (CSR by k)."""
    ks = np.broadcast_to(np.asarray(ks, dtype=np.int64), (queries.shape[0],))
    off = csr_offsets(ks)
    ids = np.empty(off[-1], dtype=np.int32)
    lcps = np.empty(off[-1], dtype=np.int32)
    for i in range(queries.shape[0]):
        a, b = topk(db, queries[i], int(ks[i]))
        ids[off[i]:off[i + 1]] = a
        lcps[off[i]:off[i + 1]] = b
    return ids, lcps, off


def sorted_permutation(db: np.ndarray) -> np.ndarray:
    """Ids of db in lexicographic row order, equal rows by ascending id.

    numpy.lexsort sorts by its *last* key first and is stable, so passing the
    columns last-to-first makes column 0 the most significant position.
    """
    db = np.asarray(db)
    L = db.shape[1]
    keys = tuple(db[:, j].astype(np.int64) for j in range(L - 1, -1, -1))
    return np.lexsort(keys).astype(np.int32)


def adjacent_lcp(db: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """A[i] = LCP(T[i-1], T[i]) over the sorted rows T = db[perm]; A[0] = 0."""
    t = np.asarray(db)[np.asarray(perm)]
    n, L = t.shape
    a = np.zeros(n, dtype=np.int32)
    if n > 1:
        eq = t[1:] == t[:-1]
        a[1:] = np.where(eq.all(axis=1), L, np.argmin(eq, axis=1))
    return a


def lower_bound(db: np.ndarray, perm: np.ndarray, q) -> int:
    """Number of rows lexicographically smaller than q (its insertion point
    in the sorted order)."""
    rows = [tuple(int(x) for x in r) for r in np.asarray(db)[np.asarray(perm)]]
    return bisect.bisect_left(rows, tuple(int(x) for x in q))


def prefix_bucket(db: np.ndarray, perm: np.ndarray, q, d: int):
    """[lo, hi) of the sorted rows whose first d tokens equal q's (section 6.2)."""
    t = np.asarray(db)[np.asarray(perm)]
    if d == 0:
        return 0, t.shape[0]
    match = (t[:, :d] == np.asarray(q)[None, :d]).all(axis=1)
    idx = np.nonzero(match)[0]
    if idx.size == 0:
        p = lower_bound(db, perm, q)
        return p, p
    return int(idx[0]), int(idx[-1]) + 1


def bucket_topk(db: np.ndarray, q: np.ndarray, k: int, d: int):
    """Top-k of the query's depth-d prefix bucket alone (section 6.2,
    Definitions "Prefix Bucket" and "Thermal-Aware Logic").

    The bucket is every row whose first d tokens equal q's (d = 0: every row);
    its rows are ranked as in topk (LCP descending, id ascending, ids of the
    whole database) and the first k returned, padded with (-1, -1).
    """
    if k < 1:
        raise ValueError("k must be >= 1")
    db = np.asarray(db)
    q = np.asarray(q)
    member = (db[:, :d] == q[None, :d]).all(axis=1)
    ids = np.nonzero(member)[0].astype(np.int64)
    v = lcp_against(db[ids], q)
    order = np.lexsort((ids, -v.astype(np.int64)))[:k]
    out_ids = np.full(k, -1, dtype=np.int32)
    out_lcp = np.full(k, -1, dtype=np.int32)
    out_ids[: order.shape[0]] = ids[order]
    out_lcp[: order.shape[0]] = v[order]
    return out_ids, out_lcp


def bucket_topk_batch(db: np.ndarray, queries: np.ndarray, ks, d: int):
    """bucket_topk for a batch; outputs concatenated in query order (CSR by k)."""
    ks = np.broadcast_to(np.asarray(ks, dtype=np.int64), (queries.shape[0],))
    off = csr_offsets(ks)
    ids = np.empty(off[-1], dtype=np.int32)
    lcps = np.empty(off[-1], dtype=np.int32)
    for i in range(queries.shape[0]):
        a, b = bucket_topk(db, queries[i], int(ks[i]), d)
        ids[off[i]:off[i + 1]] = a
        lcps[off[i]:off[i + 1]] = b
    return ids, lcps, off
