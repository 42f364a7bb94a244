"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pin checks reject every one of them."""
import bisect

import numpy as np
import pytest

import synth
from oracle import lcp_oracle as O

import pins


def _topk_from_lcp(lcp_fn, order_fn, pad=-1):
    def topk(db, q, k):
        v = lcp_fn(db, q)
        ids = np.arange(db.shape[0])
        order = order_fn(ids, v)[:k]
        out_i = np.full(k, pad, dtype=np.int32)
        out_l = np.full(k, pad, dtype=np.int32)
        out_i[: order.shape[0]] = order
        out_l[: order.shape[0]] = v[order]
        return out_i, out_l
    return topk


good_order = lambda ids, v: np.lexsort((ids, -v.astype(np.int64)))


def lcp_off_by_one(db, q):
    return np.minimum(O.lcp_against(db, q) + 1, db.shape[1]).astype(np.int32)


def lcp_count_matches(db, q):
    return (db == q[None, :]).sum(axis=1).astype(np.int32)


def lcp_suffix(db, q):
    return O.lcp_against(db[:, ::-1], q[::-1])


TOPK_MUTANTS = {
    "tie_break_id_descending": _topk_from_lcp(O.lcp_against, lambda ids, v: np.lexsort((-ids, -v.astype(np.int64)))),
    "lowest_lcp_first": _topk_from_lcp(O.lcp_against, lambda ids, v: np.lexsort((ids, v))),
    "lcp_off_by_one": _topk_from_lcp(lcp_off_by_one, good_order),
    "lcp_counts_matches": _topk_from_lcp(lcp_count_matches, good_order),
    "lcp_from_the_end": _topk_from_lcp(lcp_suffix, good_order),
    "pad_with_zero": _topk_from_lcp(O.lcp_against, good_order, pad=0),
    "ties_by_lexicographic_order": None,  # filled below
}


def _lex_tie_topk(db, q, k):
    # Algorithm 4 taken literally: equal-LCP rows in sorted (leaf) order
    v = O.lcp_against(db, q)
    perm = O.sorted_permutation(db)
    rank_in_sorted = np.empty_like(perm)
    rank_in_sorted[perm] = np.arange(perm.shape[0])
    order = np.lexsort((rank_in_sorted, -v.astype(np.int64)))[:k]
    out_i = np.full(k, -1, dtype=np.int32)
    out_l = np.full(k, -1, dtype=np.int32)
    out_i[: order.shape[0]] = order
    out_l[: order.shape[0]] = v[order]
    return out_i, out_l


TOPK_MUTANTS["ties_by_lexicographic_order"] = _lex_tie_topk


def _fails(check, *args):
    try:
        check(*args)
    except AssertionError:
        return True
    return False


def _topk_pin_suite_fails(topk_fn):
    if _fails(pins.check_golden, topk_fn, O.sorted_permutation, O.adjacent_lcp, O.lower_bound):
        return True
    if _fails(pins.check_exhaustive, topk_fn, 2, (1, 2, 3), 3):
        return True
    rng = np.random.default_rng(0)
    db = synth.random_rows(rng, 40, 5, 3)
    for _ in range(20):
        q = db[rng.integers(0, 40)]
        k = int(rng.integers(1, 45))
        ids, lcps = topk_fn(db, q, k)
        if _fails(pins.check_valid_answer, db, q, k, ids, lcps):
            return True
    return False


@pytest.mark.parametrize("name", sorted(TOPK_MUTANTS))
def test_topk_mutant_is_caught(name):
    assert _topk_pin_suite_fails(TOPK_MUTANTS[name]), name


def test_unmutated_topk_passes_suite():
    assert not _topk_pin_suite_fails(O.topk)


def sorted_last_column_first(db):
    L = db.shape[1]
    return np.lexsort(tuple(db[:, j].astype(np.int64) for j in range(L))).astype(np.int32)


def sorted_unstable_ties(db):
    perm = O.sorted_permutation(db)
    # equal rows in descending id order
    out = perm.copy()
    i = 0
    t = db[perm]
    while i < len(perm):
        j = i
        while j + 1 < len(perm) and (t[j + 1] == t[i]).all():
            j += 1
        out[i:j + 1] = perm[i:j + 1][::-1]
        i = j + 1
    return out


def adj_shifted(db, perm):
    a = O.adjacent_lcp(db, perm)
    return np.concatenate([a[1:], [0]]).astype(np.int32)


def adj_off_by_one(db, perm):
    a = O.adjacent_lcp(db, perm).copy()
    a[1:] = np.minimum(a[1:] + 1, db.shape[1])
    return a


def lb_bisect_right(db, perm, q):
    rows = [tuple(int(x) for x in r) for r in db[perm]]
    return bisect.bisect_right(rows, tuple(int(x) for x in q))


def _structure_suite_fails(sorted_fn, adj_fn, lb_fn):
    if _fails(pins.check_golden, O.topk, sorted_fn, adj_fn, lb_fn):
        return True
    rng = np.random.default_rng(3)
    for _ in range(5):
        db = synth.random_rows(rng, 30, 4, 3)
        if _fails(pins.check_sorted, sorted_fn, db) or _fails(pins.check_range_min, sorted_fn, adj_fn, db):
            return True
        for _ in range(5):
            q = db[rng.integers(0, 30)]
            if _fails(pins.check_lower_bound, sorted_fn, lb_fn, db, q):
                return True
    return False


@pytest.mark.parametrize("mut", ["sorted_last_column_first", "sorted_unstable_ties", "adj_shifted",
                                 "adj_off_by_one", "lb_bisect_right"])
def test_structure_mutant_is_caught(mut):
    fns = {"sorted": O.sorted_permutation, "adj": O.adjacent_lcp, "lb": O.lower_bound}
    m = globals()[mut]
    key = mut.split("_")[0]
    fns[{"sorted": "sorted", "adj": "adj", "lb": "lb"}[key]] = m
    assert _structure_suite_fails(fns["sorted"], fns["adj"], fns["lb"])


def test_unmutated_structure_passes_suite():
    assert not _structure_suite_fails(O.sorted_permutation, O.adjacent_lcp, O.lower_bound)


# ---- bucket range scan (section 6.2)

def _bucket_depth_minus_one(db, q, k, d):
    return O.bucket_topk(db, q, k, max(d - 1, 0))


def _bucket_depth_plus_one(db, q, k, d):
    return O.bucket_topk(db, q, k, min(d + 1, db.shape[1]))


def _bucket_by_last_tokens(db, q, k, d):
    L = db.shape[1]
    member = (db[:, L - d:] == q[None, L - d:]).all(axis=1) if d else np.ones(db.shape[0], bool)
    ids = np.nonzero(member)[0]
    v = O.lcp_against(db[ids], q)
    order = np.lexsort((ids, -v.astype(np.int64)))[:k]
    out_i = np.full(k, -1, np.int32)
    out_l = np.full(k, -1, np.int32)
    out_i[:len(order)] = ids[order]
    out_l[:len(order)] = v[order]
    return out_i, out_l


def _bucket_ignored(db, q, k, d):
    return O.topk(db, q, k)


def _bucket_local_ids(db, q, k, d):
    member = (db[:, :d] == q[None, :d]).all(axis=1)
    sub = db[member]
    return O.topk(sub, q, k) if sub.shape[0] else (np.full(k, -1, np.int32), np.full(k, -1, np.int32))


def _bucket_ties_by_sorted_position(db, q, k, d):
    perm = O.sorted_permutation(db)
    t = db[perm]
    member = (t[:, :d] == q[None, :d]).all(axis=1)
    pos = np.nonzero(member)[0]
    v = O.lcp_against(t[pos], q)
    order = np.lexsort((pos, -v.astype(np.int64)))[:k]
    out_i = np.full(k, -1, np.int32)
    out_l = np.full(k, -1, np.int32)
    out_i[:len(order)] = perm[pos[order]]
    out_l[:len(order)] = v[order]
    return out_i, out_l


BUCKET_MUTANTS = {
    "depth_minus_one": _bucket_depth_minus_one,
    "depth_plus_one": _bucket_depth_plus_one,
    "bucket_by_last_tokens": _bucket_by_last_tokens,
    "bucket_ignored": _bucket_ignored,
    "ids_local_to_bucket": _bucket_local_ids,
    "ties_by_sorted_position": _bucket_ties_by_sorted_position,
}


def _bucket_pin_suite_fails(fn):
    if _fails(pins.check_bucket_golden, fn):
        return True
    if _fails(pins.check_bucket_exhaustive, fn, 2, (1, 2, 3), 3):
        return True
    rng = np.random.default_rng(0)
    db = synth.random_rows(rng, 60, 5, 3)
    for _ in range(10):
        q = db[rng.integers(0, 60)]
        k = int(rng.integers(1, 65))
        for d in range(6):
            if _fails(pins.check_bucket_theorem, fn, O.topk, db, q, k, d):
                return True
    return False


@pytest.mark.parametrize("name", sorted(BUCKET_MUTANTS))
def test_bucket_mutant_is_caught(name):
    assert _bucket_pin_suite_fails(BUCKET_MUTANTS[name]), name


def test_unmutated_bucket_passes_suite():
    assert not _bucket_pin_suite_fails(O.bucket_topk)
