"""Checks that pin the CPU oracle to facts other than its own formulas.

Each check takes the oracle functions as arguments so that the mutation tests
can hand it deliberately broken versions and confirm that it fails them.

Independent facts used (none re-types the oracle's arithmetic):

* Exhaustive enumeration of tiny databases, compared with a second
  formulation of the definition (section 2.1): LCP through the library routine
  ``os.path.commonprefix`` and the ranking built level by level (all ids at
  LCP = L in ascending order, then LCP = L-1, ...).
* The defining optimality property of a top-k answer: every returned row
  ranks above every row left out, under (LCP descending, id ascending).
* ``heapq.nsmallest`` on (L - LCP, id) as a library selection routine.
* Hand-derived values in tests/golden/handworked_acgt.json.
* Sortedness of the permutation checked pairwise with Python tuple order;
  the range-minimum identity LCP(T[i], T[j]) = min(A[i+1..j]), which follows
  from the ultrametric property (section 2.1, Theorem "Ultrametric Property")
  and sorted order, checked against brute-force pairwise LCPs; the insertion
  point checked against its counting definition.
* The bucket range scan (section 6.2): a row is in the query's depth-d bucket
  exactly when its LCP with the query is at least d, so the bucket's answer is
  the level ranking cut off below level d; and whenever the k-th best LCP over
  all rows is at least d the bucket holds every row that can rank, so its
  answer equals the full top-k (Theorem "Range Scan Complexity").
"""
from __future__ import annotations

import heapq
import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ref_lcp(a, b) -> int:
    return len(os.path.commonprefix([[int(x) for x in a], [int(x) for x in b]]))


def level_ranking(db, q, k):
    """Second formulation: concatenate ids level by level from LCP=L down to 0."""
    L = len(q)
    lv = [ref_lcp(r, q) for r in db]
    ids, lcps = [], []
    for c in range(L, -1, -1):
        for i, v in enumerate(lv):
            if v == c:
                ids.append(i)
                lcps.append(c)
    ids, lcps = ids[:k], lcps[:k]
    ids += [-1] * (k - len(ids))
    lcps += [-1] * (k - len(lcps))
    return ids, lcps


def check_exhaustive(topk_fn, V=2, L_values=(1, 2, 3), N_max=3, k_extra=2):
    """Every database of N <= N_max rows over Sigma^L, every query in Sigma^L,
    every k in 1..N+k_extra."""
    for L in L_values:
        alphabet_rows = [np.array(r, dtype=np.uint8) for r in itertools.product(range(V), repeat=L)]
        for N in range(1, N_max + 1):
            for rows in itertools.product(range(len(alphabet_rows)), repeat=N):
                db = np.stack([alphabet_rows[i] for i in rows])
                for q in alphabet_rows:
                    for k in range(1, N + k_extra + 1):
                        ids, lcps = topk_fn(db, q, k)
                        want_ids, want_lcps = level_ranking(db, q, k)
                        assert list(map(int, ids)) == want_ids, (db.tolist(), q.tolist(), k)
                        assert list(map(int, lcps)) == want_lcps, (db.tolist(), q.tolist(), k)


def check_valid_answer(db, q, k, ids, lcps):
    """The defining property of a top-k answer (section 2.1)."""
    N = db.shape[0]
    ids = [int(x) for x in ids]
    lcps = [int(x) for x in lcps]
    assert len(ids) == k and len(lcps) == k
    kp = min(k, N)
    assert ids[kp:] == [-1] * (k - kp) and lcps[kp:] == [-1] * (k - kp)
    got = ids[:kp]
    assert len(set(got)) == kp and all(0 <= i < N for i in got)
    true = [ref_lcp(db[i], q) for i in range(N)]
    assert [true[i] for i in got] == lcps[:kp]
    ranks = [(-true[i], i) for i in got]
    assert ranks == sorted(ranks)
    if kp < N:
        worst = ranks[-1]
        chosen = set(got)
        for i in range(N):
            if i not in chosen:
                assert (-true[i], i) > worst, (i, true[i], worst)


def check_heapq(topk_fn, db, q, k):
    L = db.shape[1]
    cand = heapq.nsmallest(k, ((L - ref_lcp(r, q), i) for i, r in enumerate(db)))
    ids, lcps = topk_fn(db, q, k)
    n = len(cand)
    assert [int(x) for x in ids[:n]] == [i for _, i in cand]
    assert [int(x) for x in lcps[:n]] == [L - d for d, _ in cand]


def load_golden(name="handworked_acgt.json"):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def check_golden(topk_fn, sorted_fn, adj_fn, lb_fn):
    g = load_golden()
    db = np.array(g["db"], dtype=np.uint8)
    for case in g["queries"]:
        q = np.array(case["q"], dtype=np.uint8)
        ids, lcps = topk_fn(db, q, case["k"])
        assert list(map(int, ids)) == case["ids"], case
        assert list(map(int, lcps)) == case["lcps"], case
    perm = sorted_fn(db)
    assert list(map(int, perm)) == g["perm"]
    assert list(map(int, adj_fn(db, perm))) == g["adjacent_lcp"]
    for case in g["lower_bound"]:
        assert lb_fn(db, perm, np.array(case["q"], dtype=np.uint8)) == case["p"], case


def check_sorted(sorted_fn, db):
    perm = [int(x) for x in sorted_fn(db)]
    N = db.shape[0]
    assert sorted(perm) == list(range(N))
    rows = [tuple(int(x) for x in db[i]) for i in perm]
    for i in range(1, N):
        assert rows[i - 1] < rows[i] or (rows[i - 1] == rows[i] and perm[i - 1] < perm[i]), i


def check_range_min(sorted_fn, adj_fn, db):
    perm = sorted_fn(db)
    A = [int(x) for x in adj_fn(db, perm)]
    t = db[np.asarray(perm)]
    N = t.shape[0]
    assert A[0] == 0
    for i in range(N):
        for j in range(i + 1, N):
            assert ref_lcp(t[i], t[j]) == min(A[i + 1:j + 1]), (i, j)


def check_lower_bound(sorted_fn, lb_fn, db, q):
    perm = sorted_fn(db)
    want = sum(1 for r in db if tuple(int(x) for x in r) < tuple(int(x) for x in q))
    assert lb_fn(db, perm, q) == want


def bucket_level_ranking(db, q, k, d):
    """Second formulation of the bucket scan: levels L, L-1, ..., d of the
    level ranking (rows below level d are outside the bucket)."""
    L = len(q)
    lv = [ref_lcp(r, q) for r in db]
    ids, lcps = [], []
    for c in range(L, d - 1, -1):
        for i, v in enumerate(lv):
            if v == c:
                ids.append(i)
                lcps.append(c)
    ids, lcps = ids[:k], lcps[:k]
    return ids + [-1] * (k - len(ids)), lcps + [-1] * (k - len(lcps))


def check_bucket_exhaustive(bucket_fn, V=2, L_values=(1, 2, 3), N_max=3, k_extra=2):
    """Every database of N <= N_max rows over Sigma^L, every query, every depth
    0..L and every k in 1..N+k_extra."""
    for L in L_values:
        alphabet_rows = [np.array(r, dtype=np.uint8) for r in itertools.product(range(V), repeat=L)]
        for N in range(1, N_max + 1):
            for rows in itertools.product(range(len(alphabet_rows)), repeat=N):
                db = np.stack([alphabet_rows[i] for i in rows])
                for q in alphabet_rows:
                    for d in range(L + 1):
                        for k in range(1, N + k_extra + 1):
                            ids, lcps = bucket_fn(db, q, k, d)
                            want = bucket_level_ranking(db, q, k, d)
                            got = (list(map(int, ids)), list(map(int, lcps)))
                            assert got == want, (db.tolist(), q.tolist(), d, k)


def check_bucket_golden(bucket_fn):
    g = load_golden()
    db = np.array(g["db"], dtype=np.uint8)
    for case in g["bucket_scan"]:
        q = np.array(case["q"], dtype=np.uint8)
        ids, lcps = bucket_fn(db, q, case["k"], case["d"])
        assert list(map(int, ids)) == case["ids"], case
        assert list(map(int, lcps)) == case["lcps"], case


def check_bucket_theorem(bucket_fn, topk_fn, db, q, k, d):
    """When the k-th best LCP over all rows is >= d (and N >= k) the bucket
    answer is the full answer; otherwise it is the full ranking's prefix of
    rows with LCP >= d, then pads."""
    full_ids, full_lcps = topk_fn(db, q, db.shape[0])
    ids, lcps = bucket_fn(db, q, k, d)
    ids, lcps = list(map(int, ids)), list(map(int, lcps))
    keep = [(int(i), int(v)) for i, v in zip(full_ids, full_lcps) if v >= d][:k]
    want_ids = [i for i, _ in keep] + [-1] * (k - len(keep))
    want_lcps = [v for _, v in keep] + [-1] * (k - len(keep))
    assert (ids, lcps) == (want_ids, want_lcps), (q.tolist(), k, d)
    if k <= db.shape[0] and int(full_lcps[k - 1]) >= d:
        a, b = topk_fn(db, q, k)
        assert ids == list(map(int, a)) and lcps == list(map(int, b))
