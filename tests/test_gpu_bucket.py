"""GPU parity of the prefix-bucket range scan (lcp_bucket_scan_topk, section
6.2) against the CPU oracle's bucket_topk and prefix_bucket: ids, LCPs and
bucket bounds bit-exact (all integer; no tolerance)."""
import numpy as np
import pytest

import pins
import synth
from oracle import lcp_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2602_04936_amd as P
    torch.cuda.init()
    return P


def _run(idx, qs, ks, d):
    import torch
    r, b = idx.bucket_scan_topk(qs, ks, d, bounds=True)
    torch.cuda.synchronize()
    return r.ids.cpu().numpy(), r.lcps.cpu().numpy(), r.offsets, b.cpu().numpy()


def _assert_equal(got_ids, got_lcp, want_ids, want_lcp, off, what):
    if (got_ids == want_ids).all() and (got_lcp == want_lcp).all():
        return
    bad = np.nonzero((got_ids != want_ids) | (got_lcp != want_lcp))[0][0]
    qi = int(np.searchsorted(off, bad, side="right") - 1)
    a, b = off[qi], off[qi + 1]
    raise AssertionError(f"{what}: query {qi} differs\n got ids {got_ids[a:b]}\n want    {want_ids[a:b]}\n"
                         f" got lcp {got_lcp[a:b]}\n want    {want_lcp[a:b]}")


def _check_index(idx, db, qs, ks, depths, what, check_bounds=True):
    ks = np.broadcast_to(np.asarray(ks, dtype=np.int32), (qs.shape[0],)).copy()
    perm = O.sorted_permutation(db) if check_bounds else None
    for d in depths:
        gi, gl, off, gb = _run(idx, qs, ks, d)
        wi, wl, woff = O.bucket_topk_batch(db, qs, ks, d)
        assert (off == woff).all()
        _assert_equal(gi, gl, wi, wl, off, f"{what} depth {d}")
        if check_bounds:
            for i in range(qs.shape[0]):
                assert tuple(int(x) for x in gb[i]) == O.prefix_bucket(db, perm, qs[i], d), (what, d, i)


def _check(P, db, qs, ks, V, depths, what):
    with P.Index(db, V) as idx:
        _check_index(idx, db, qs, ks, depths, what)


def test_golden_handworked(P):
    g = pins.load_golden()
    db = np.array(g["db"], dtype=np.uint8)
    with P.Index(db, g["V"]) as idx:
        for case in g["bucket_scan"]:
            q = np.array([case["q"]], dtype=np.uint8)
            gi, gl, _, gb = _run(idx, q, [case["k"]], case["d"])
            assert gi.tolist() == case["ids"] and gl.tolist() == case["lcps"], case
            assert gb[0].tolist() == case["bounds"], case


@pytest.mark.parametrize("V,L", [(4, 6), (16, 24), (300, 9), (65536, 3), (2, 40), (256, 1)])
def test_random_depths_and_widths(P, V, L):
    """One- and two-byte tokens, rows of one to ten key words, every depth class:
    0 (every row), shallow, deep, L; queries copied from rows (deep buckets)
    and drawn at random (often empty buckets); k on both sides of every list size."""
    rng = np.random.default_rng(V * 31 + L)
    N = 4000
    protos = synth.random_rows(rng, 40, L, V)
    db = np.where(rng.random((N, L)) < 0.15, synth.random_rows(rng, N, L, V), protos[rng.integers(0, 40, N)])
    qs = np.concatenate([db[rng.integers(0, N, 24)], synth.random_rows(rng, 16, L, V)])
    ks = rng.choice([1, 5, 10, 64, 65, 100, 200, 1024], qs.shape[0]).astype(np.int32)
    depths = sorted({0, 1, min(2, L), min(3, L), L // 2, L})
    _check(P, db, qs, ks, V, depths, f"V={V} L={L}")


def test_c1_workload(P):
    w = synth.c1_tiny()
    qs, ks = w.queries[:96], w.k[:96]
    _check(P, w.db, qs, ks, w.V, [0, 1, 2, 3, 5], "c1")


def test_edge_cases(P):
    rng = np.random.default_rng(9)
    # N = 1: bucket of one row or none
    db = np.array([[3, 1, 2]], dtype=np.uint8)
    _check(P, db, np.array([[3, 1, 2], [3, 0, 0], [0, 0, 0]], np.uint8), [1, 3, 2], 4, [0, 1, 2, 3], "N=1")
    # all rows identical: every bucket that is not empty is all N rows, tied on id
    db = np.tile(np.array([[7, 7, 7, 7]], np.uint8), (3000, 1))
    qs = np.array([[7, 7, 7, 7], [7, 7, 1, 0], [0, 7, 7, 7]], np.uint8)
    _check(P, db, qs, [1, 100, 1024], 8, [0, 1, 2, 4], "identical rows")
    # buckets smaller than k, and k = K_MAX
    db = synth.random_rows(rng, 700, 5, 3)
    qs = synth.random_rows(rng, 8, 5, 3)
    _check(P, db, qs, [1024, 700, 699, 701, 1, 64, 128, 256], 3, [0, 1, 2, 5], "large k")


def test_bucket_larger_than_a_wave_round(P):
    """Buckets of tens of thousands of rows (many scan steps per wave) with long
    ties at the cutoff: c3-shaped rows, depth 1 and 2."""
    w = synth.c3_like(60_000, 48, seed=77, k_choices=(1, 10, 100))
    with P.Index(w.db, w.V) as idx:
        _check_index(idx, w.db, w.queries, w.k, [0, 1, 2], "c3_like 60k", check_bounds=False)


def test_depth_out_of_range_is_rejected(P):
    db = synth.random_rows(np.random.default_rng(2), 50, 4, 5)
    with P.Index(db, 5) as idx:
        for d in (-1, 5):
            with pytest.raises(Exception):
                idx.bucket_scan_topk(db[:2], 3, d)


def test_after_append_and_reserve(P):
    """The sorted prefixes follow the index through appends and a reserve."""
    rng = np.random.default_rng(41)
    L, V = 10, 6
    a = synth.random_rows(rng, 2500, L, V)
    b = np.concatenate([synth.random_rows(rng, 400, L, V), a[:30]])
    c = synth.random_rows(rng, 90, L, V)
    qs = np.concatenate([synth.random_rows(rng, 20, L, V), a[rng.integers(0, 2500, 12)], b[:6]])
    ks = rng.integers(1, 70, qs.shape[0]).astype(np.int32)
    with P.Index(a, V) as idx:
        _check_index(idx, a, qs, ks, [0, 2, 4], "before append")
        idx.append(b)
        ab = np.concatenate([a, b])
        _check_index(idx, ab, qs, ks, [0, 2, 4], "after one append")
        idx.reserve(10_000)
        idx.append(c)
        _check_index(idx, np.concatenate([ab, c]), qs, ks, [1, 3, L], "after reserve and append")


def test_c3_full_size_sampled_and_against_the_index_path(P):
    """c3 in full (N = 2,000,000, 8,192 queries) in the configuration the
    benchmark times (one call over the batch, k = 10) at depths 1 and 2: a
    spread sample of queries against the oracle one by one, and for every
    query the range-scan theorem against the index path (whose answers the
    c3 parity test checks): where the k-th best LCP is at least d the two
    answers agree; elsewhere the bucket holds exactly the index path's rows of
    LCP >= d, and its answer is those rows followed by pads."""
    import torch
    w = synth.c3_hierarchy()
    k = 10
    sample = np.linspace(0, w.Q - 1, 48).astype(np.int64)
    with P.Index(w.db, w.V) as idx:
        full = idx.topk(w.queries, k)
        torch.cuda.synchronize()
        fi = full.ids.cpu().numpy().reshape(w.Q, k)
        fl = full.lcps.cpu().numpy().reshape(w.Q, k)
        for d in (1, 2):
            print(f"bucket scan c3 N={w.N} depth={d}", flush=True)
            gi, gl, _, gb = _run(idx, w.queries, np.full(w.Q, k, np.int32), d)
            gi, gl = gi.reshape(w.Q, k), gl.reshape(w.Q, k)
            for i in sample:
                wi, wl = O.bucket_topk(w.db, w.queries[i], k, d)
                assert (gi[i] == wi).all() and (gl[i] == wl).all(), (d, int(i))
            size = gb[:, 1] - gb[:, 0]
            full_inside = fl[:, k - 1] >= d
            assert (gi[full_inside] == fi[full_inside]).all() and (gl[full_inside] == fl[full_inside]).all()
            for i in np.nonzero(~full_inside)[0]:
                # the k-th best LCP is below d: every row of the bucket is in the
                # index path's answer, and the bucket answer is those rows, then pads
                m = int((fl[i] >= d).sum())
                assert int(size[i]) == m, (d, int(i))
                assert (gi[i, :m] == fi[i, :m]).all() and (gl[i, :m] == fl[i, :m]).all(), (d, int(i))
                assert (gi[i, m:] == -1).all() and (gl[i, m:] == -1).all(), (d, int(i))


def test_query_tokens_beyond_the_vocabulary(P):
    """Query tokens >= V compare as integers (their bucket is empty, or shorter
    than d when the token comes later)."""
    rng = np.random.default_rng(23)
    for V, L in ((16, 10), (300, 6)):
        db = synth.random_rows(rng, 3000, L, V)
        qs = db[rng.integers(0, 3000, 24)].copy()
        big = np.iinfo(qs.dtype).max
        qs[::3, 0] = big          # empty bucket at every depth >= 1
        qs[1::3, L // 2] = big    # the bucket is the rows' own up to L/2
        _check(P, db, qs, rng.integers(1, 40, qs.shape[0]).astype(np.int32), V, [0, 1, L // 2, L // 2 + 1, L],
               f"tokens >= V, V={V}")


def test_two_streams_share_the_sorted_planes(P):
    """Calls on two streams after an append: the first call that needs a plane
    lays it out and waits, later calls on either stream read it."""
    import torch
    rng = np.random.default_rng(31)
    L, V = 12, 8
    a = synth.random_rows(rng, 4000, L, V)
    b = synth.random_rows(rng, 500, L, V)
    qs = np.concatenate([a[rng.integers(0, 4000, 30)], synth.random_rows(rng, 10, L, V)])
    ks = rng.integers(1, 50, qs.shape[0]).astype(np.int32)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    with P.Index(a, V) as idx:
        idx.append(b)
        db = np.concatenate([a, b])
        q = P.to_device_tokens(qs, torch.device("cuda:0"))
        outs = []
        for i, d in enumerate((0, 5, 2, 9, 0, 5)):
            outs.append((d, idx.bucket_scan_topk(q, ks, d, stream=streams[i % 2])))
        torch.cuda.synchronize()
        for d, r in outs:
            wi, wl, _ = O.bucket_topk_batch(db, qs, ks, d)
            _assert_equal(r.ids.cpu().numpy(), r.lcps.cpu().numpy(), wi, wl, r.offsets, f"two streams depth {d}")
