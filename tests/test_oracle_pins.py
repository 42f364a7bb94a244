"""Pins of the CPU oracle (no GPU needed)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import lcp_oracle as O

import pins


def test_golden_handworked():
    pins.check_golden(O.topk, O.sorted_permutation, O.adjacent_lcp, O.lower_bound)


def test_exhaustive_tiny_V2():
    pins.check_exhaustive(O.topk, V=2, L_values=(1, 2, 3), N_max=4)


def test_exhaustive_tiny_V3_L2():
    pins.check_exhaustive(O.topk, V=3, L_values=(2,), N_max=3)


@pytest.mark.parametrize("seed", range(6))
def test_validity_and_heapq_random(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 60))
    L = int(rng.integers(1, 7))
    V = int(rng.integers(2, 5))
    db = synth.random_rows(rng, N, L, V)
    for _ in range(20):
        # half the queries are database rows, so long LCPs and duplicates occur
        q = db[rng.integers(0, N)] if rng.random() < 0.5 else synth.random_rows(rng, 1, L, V)[0]
        k = int(rng.integers(1, N + 5))
        ids, lcps = O.topk(db, q, k)
        pins.check_valid_answer(db, q, k, ids, lcps)
        pins.check_heapq(O.topk, db, q, k)


def test_lcp_invariants():
    """LCP(q,q)=L, symmetry, and the strong triangle inequality (section 2.1,
    Theorem 'Ultrametric Property') on random triples."""
    rng = np.random.default_rng(7)
    for _ in range(500):
        L = int(rng.integers(1, 9))
        s, t, u = synth.random_rows(rng, 3, L, 3)
        assert O.lcp(s, s) == L
        assert O.lcp(s, t) == O.lcp(t, s) == pins.ref_lcp(s, t)
        assert O.lcp(s, u) >= min(O.lcp(s, t), O.lcp(t, u))
        v = O.lcp_against(np.stack([t, u]), s)
        assert list(v) == [pins.ref_lcp(s, t), pins.ref_lcp(s, u)]


def test_duplicate_member_top1():
    """A query equal to a database row gets, at rank 1, the lowest id among
    the rows equal to it, at LCP = L."""
    rng = np.random.default_rng(11)
    db = synth.random_rows(rng, 300, 5, 2)
    for i in rng.integers(0, 300, 40):
        ids, lcps = O.topk(db, db[i], 1)
        dup = [j for j in range(300) if (db[j] == db[i]).all()]
        assert ids[0] == min(dup) and lcps[0] == 5


@pytest.mark.parametrize("seed", range(4))
def test_structure_oracles(seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(1, 40))
    L = int(rng.integers(1, 6))
    db = synth.random_rows(rng, N, L, 3)
    pins.check_sorted(O.sorted_permutation, db)
    pins.check_range_min(O.sorted_permutation, O.adjacent_lcp, db)
    for _ in range(10):
        q = synth.random_rows(rng, 1, L, 4)[0]
        pins.check_lower_bound(O.sorted_permutation, O.lower_bound, db, q)


def test_prefix_bucket_matches_definition():
    """Prefix bucket (section 6.2): the rows sharing q's first d tokens are a
    contiguous sorted range."""
    rng = np.random.default_rng(5)
    db = synth.random_rows(rng, 200, 4, 3)
    perm = O.sorted_permutation(db)
    t = db[perm]
    for _ in range(30):
        q = synth.random_rows(rng, 1, 4, 3)[0]
        for d in range(5):
            lo, hi = O.prefix_bucket(db, perm, q, d)
            members = [i for i in range(200) if pins.ref_lcp(t[i], q) >= d]
            if members:
                assert members == list(range(lo, hi))
            else:
                assert lo == hi


def test_bucket_scan_golden_handworked():
    """Hand-derived bucket answers and bounds (section 6.2, Appendix D.1)."""
    pins.check_bucket_golden(O.bucket_topk)
    g = pins.load_golden()
    db = np.array(g["db"], dtype=np.uint8)
    perm = O.sorted_permutation(db)
    for case in g["bucket_scan"]:
        assert list(O.prefix_bucket(db, perm, np.array(case["q"]), case["d"])) == case["bounds"], case


def test_bucket_scan_exhaustive_tiny():
    pins.check_bucket_exhaustive(O.bucket_topk, V=2, L_values=(1, 2, 3), N_max=3)


@pytest.mark.parametrize("seed", range(4))
def test_bucket_scan_reduces_to_full_answer(seed):
    """Theorem "Range Scan Complexity": the bucket holds every row that can rank
    once the k-th best LCP reaches d; d = 0 is the full scan."""
    rng = np.random.default_rng(100 + seed)
    db = synth.random_rows(rng, 120, 6, 3)
    for _ in range(12):
        q = db[rng.integers(0, 120)].copy() if rng.random() < 0.5 else synth.random_rows(rng, 1, 6, 3)[0]
        k = int(rng.integers(1, 130))
        for d in range(7):
            pins.check_bucket_theorem(O.bucket_topk, O.topk, db, q, k, d)
        a, b = O.bucket_topk(db, q, k, 0)
        c, e = O.topk(db, q, k)
        assert (a == c).all() and (b == e).all()


def test_c_oracle_matches_numpy_oracle_c1():
    w = synth.c1_tiny()
    ids, lcps, off = oracle.c_topk(w.db, w.queries, w.k)
    nids, nlcps, noff = O.topk_batch(w.db, w.queries, w.k)
    assert (off == noff).all()
    assert (ids == nids).all() and (lcps == nlcps).all()


@pytest.mark.parametrize("seed", range(5))
def test_c_oracle_random_uint16_and_padding(seed):
    rng = np.random.default_rng(200 + seed)
    N = int(rng.integers(1, 80))
    L = int(rng.integers(1, 9))
    V = int(rng.choice([2, 3, 300, 65536]))
    db = synth.random_rows(rng, N, L, V, dtype=np.uint16)
    qs = np.concatenate([synth.random_rows(rng, 10, L, V, dtype=np.uint16), db[: min(N, 5)]])
    ks = rng.integers(1, N + 6, qs.shape[0]).astype(np.int32)
    ids, lcps, off = oracle.c_topk(db, qs, ks)
    nids, nlcps, _ = O.topk_batch(db, qs, ks)
    assert (ids == nids).all() and (lcps == nlcps).all()
    for i in range(qs.shape[0]):
        pins.check_valid_answer(db, qs[i], int(ks[i]), ids[off[i]:off[i + 1]], lcps[off[i]:off[i + 1]])


def test_c_oracle_exhaustive_tiny():
    def c_topk_one(db, q, k):
        ids, lcps, _ = oracle.c_topk(db, q[None, :], [k])
        return ids, lcps
    pins.check_exhaustive(c_topk_one, V=2, L_values=(1, 2), N_max=3)


def test_dense_matrix_remark_arithmetic():
    """The pairwise fp16 matrix that the paper reports as out of memory at
    N=500K (section 7, Table 'OOM wall') is N^2 * 2 bytes = 465.66 GiB."""
    assert round(500_000 ** 2 * 2 / 2 ** 30, 2) == 465.66
    assert round(100_000 ** 2 * 2 / 2 ** 30, 2) == 18.63
