"""GPU parity: the HIP index path and full-scan path against the CPU oracle,
bit-exact on ids and LCPs (all integer; no tolerance)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import lcp_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2602_04936_amd as P
    torch.cuda.init()
    return P


def _both(P, idx, queries, ks):
    import torch
    a = idx.topk(queries, ks)
    b = idx.scan_topk(queries, ks)
    torch.cuda.synchronize()
    return (a.ids.cpu().numpy(), a.lcps.cpu().numpy(), b.ids.cpu().numpy(), b.lcps.cpu().numpy(), a.offsets)


def _assert_equal(got_ids, got_lcp, want_ids, want_lcp, off, what):
    if (got_ids == want_ids).all() and (got_lcp == want_lcp).all():
        return
    bad = np.nonzero((got_ids != want_ids) | (got_lcp != want_lcp))[0][0]
    qi = int(np.searchsorted(off, bad, side="right") - 1)
    a, b = off[qi], off[qi + 1]
    raise AssertionError(f"{what}: query {qi} differs\n got ids {got_ids[a:b]}\n want    {want_ids[a:b]}\n"
                         f" got lcp {got_lcp[a:b]}\n want    {want_lcp[a:b]}")


def check_against_oracle(P, db, queries, ks, V, what, use_c=True):
    ks = np.broadcast_to(np.asarray(ks, dtype=np.int32), (queries.shape[0],)).copy()
    with P.Index(db, V) as idx:
        gi, gl, si, sl, off = _both(P, idx, queries, ks)
    if use_c:
        wi, wl, woff = oracle.c_topk(db, queries, ks)
    else:
        wi, wl, woff = O.topk_batch(db, queries, ks)
    assert (off == woff).all()
    _assert_equal(gi, gl, wi, wl, off, f"{what} index path")
    _assert_equal(si, sl, wi, wl, off, f"{what} scan path")


def test_structure_c1(P):
    import torch
    w = synth.c1_tiny()
    with P.Index(w.db, w.V) as idx:
        v = idx.views()
        torch.cuda.synchronize()
        perm = v["perm"].cpu().numpy()
        A = v["adj_lcp"].cpu().numpy().astype(np.int32)
    want = O.sorted_permutation(w.db)
    assert (perm == want).all()
    assert (A == O.adjacent_lcp(w.db, want)).all()


@pytest.mark.parametrize("V,L", [(16, 16), (256, 13), (4096, 7), (2, 40), (65536, 3)])
def test_structure_random(P, V, L):
    import torch
    rng = np.random.default_rng(V + L)
    db = synth.random_rows(rng, 5000, L, V)
    db[100:200] = db[50]  # duplicates must come out by ascending id
    with P.Index(db, V) as idx:
        v = idx.views()
        torch.cuda.synchronize()
        perm = v["perm"].cpu().numpy()
        A = v["adj_lcp"].cpu().numpy().astype(np.int32)
    want = O.sorted_permutation(db)
    assert (perm == want).all()
    assert (A == O.adjacent_lcp(db, want)).all()


def test_c1_full_numpy_oracle(P):
    w = synth.c1_tiny()
    check_against_oracle(P, w.db, w.queries, w.k, w.V, "c1", use_c=False)


@pytest.mark.parametrize("seed", range(12))
def test_random_small(P, seed):
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.choice([1, 2, 3, 63, 64, 65, 129, 500, 4097, 20000]))
    L = int(rng.choice([1, 2, 3, 5, 8, 16, 24, 31, 64, 100]))
    V = int(rng.choice([2, 3, 16, 256, 300, 4096, 65536]))
    db = synth.random_rows(rng, N, L, V)
    nq = 64
    qs = synth.random_rows(rng, nq, L, V)
    # half the queries share long prefixes with database rows
    src = db[rng.integers(0, N, nq)]
    cut = rng.integers(0, L + 1, nq)
    mix = np.where(np.arange(L)[None, :] < cut[:, None], src, qs)
    queries = np.concatenate([mix, db[rng.integers(0, N, 16)]])
    ks = rng.integers(1, min(N + 5, 150), queries.shape[0]).astype(np.int32)
    check_against_oracle(P, db, queries, ks, V, f"random N={N} L={L} V={V}")


def test_edge_cases(P):
    rng = np.random.default_rng(5)
    # N = 1
    db = np.array([[3, 1, 2]], dtype=np.uint8)
    check_against_oracle(P, db, np.array([[3, 1, 2], [3, 0, 0], [0, 0, 0]], np.uint8), [1, 3, 2], 4, "N=1")
    # L = 1
    db = synth.random_rows(rng, 300, 1, 5)
    check_against_oracle(P, db, synth.random_rows(rng, 20, 1, 6), 7, 5, "L=1")
    # all rows identical: one tied block of N rows
    db = np.tile(np.array([[7, 7, 7, 7]], np.uint8), (3000, 1))
    qs = np.array([[7, 7, 7, 7], [7, 7, 1, 0], [0, 7, 7, 7]], np.uint8)
    check_against_oracle(P, db, qs, [1, 10, 100], 8, "identical rows")
    # a query sharing no first token with any row (cutoff 0, id walk)
    db = synth.random_rows(rng, 5000, 6, 4)
    qs = np.full((4, 6), 9, np.uint8)
    check_against_oracle(P, db, qs, [1, 64, 65, 200], 16, "no shared first token")
    # k = K_MAX and k > N
    db = synth.random_rows(rng, 700, 4, 3)
    qs = synth.random_rows(rng, 8, 4, 3)
    check_against_oracle(P, db, qs, [1024, 700, 699, 701, 1, 64, 128, 256], 3, "large k")


def test_c2_subset(P):
    w = synth.c2_oom_boundary(n_gen=900, n_copies=100)
    check_against_oracle(P, w.db, w.queries, w.k, w.V, "c2 subset")


def test_c3_sampled_and_paths_agree(P):
    import torch
    w = synth.c3_hierarchy()
    with P.Index(w.db, w.V) as idx:
        gi, gl, si, sl, off = _both(P, idx, w.queries, w.k)
    _assert_equal(gi, gl, si, sl, off, "c3 index vs scan")
    sample = np.arange(0, w.Q, 32)
    wi, wl, woff = oracle.c_topk(w.db, w.queries[sample], w.k[sample])
    for j, qi in enumerate(sample):
        a, b = off[qi], off[qi + 1]
        assert (gi[a:b] == wi[woff[j]:woff[j + 1]]).all(), qi
        assert (gl[a:b] == wl[woff[j]:woff[j + 1]]).all(), qi


def test_c5_sensor(P):
    w = synth.c5_sensor()
    check_against_oracle(P, w.db, w.queries, w.k, w.V, "c5")


def test_determinism_and_batch_invariance(P):
    import torch
    w = synth.c3_like(200_000, 600, seed=77)
    with P.Index(w.db, w.V) as idx:
        r1 = idx.topk(w.queries, w.k)
        r2 = idx.topk(w.queries, w.k)
        s1 = idx.scan_topk(w.queries, w.k)
        sel = np.array([5, 17, 400, 3])
        r3 = idx.topk(w.queries[sel], w.k[sel])
        s3 = idx.scan_topk(w.queries[sel], w.k[sel])
        torch.cuda.synchronize()
        assert torch.equal(r1.ids, r2.ids) and torch.equal(r1.lcps, r2.lcps)
        assert torch.equal(r1.ids, s1.ids) and torch.equal(r1.lcps, s1.lcps)
        for j, qi in enumerate(sel):
            a, b = r1.query(int(qi))
            c, d = r3.query(j)
            e, f = s3.query(j)
            assert torch.equal(a, c) and torch.equal(b, d)
            assert torch.equal(a, e) and torch.equal(b, f)


def test_errors(P):
    import torch
    db = np.zeros((10, 4), np.uint8)
    with pytest.raises(P.LcpError) as e:
        P.Index(db + 5, 5)
    assert e.value.status == -4
    with pytest.raises(P.LcpError):
        P.Index(db, 0)
    idx = P.Index(db, 5)
    q = np.zeros((2, 4), np.uint8)
    with pytest.raises(P.LcpError):
        idx.topk(q, [1, 0])
    with pytest.raises(P.LcpError):
        idx.topk(q, [1, 1025])
    r = idx.topk(q[:0], 1)
    assert r.ids.numel() == 0
    idx.close()
    torch.cuda.synchronize()


def test_uniform_and_mixed_k_agree(P):
    """Uniform k (offsets computed on the device) and per-query k (staged
    offsets) give the same per-query answers."""
    import torch
    w = synth.c3_like(100_000, 300, seed=9)
    with P.Index(w.db, w.V) as idx:
        for kval in (1, 10, 64, 65, 100):
            a = idx.topk(w.queries, kval)
            ks = np.full(w.Q, kval, np.int32)
            ks[0] = 1 if kval != 1 else 2  # force the staged path
            b = idx.topk(w.queries, ks)
            s = idx.scan_topk(w.queries, kval)
            torch.cuda.synchronize()
            assert torch.equal(a.ids, s.ids) and torch.equal(a.lcps, s.lcps)
            for qi in range(1, w.Q):
                x, y = a.query(qi)
                u, v = b.query(qi)
                assert torch.equal(x, u) and torch.equal(y, v)
        wi, wl, _ = oracle.c_topk(w.db, w.queries, 10)
        a = idx.topk(w.queries, 10)
        torch.cuda.synchronize()
        assert (a.ids.cpu().numpy() == wi).all() and (a.lcps.cpu().numpy() == wl).all()


def test_device_k_entry_points(P):
    import torch
    w = synth.c1_tiny()
    rng = np.random.default_rng(3)
    ks = rng.integers(1, 80, w.Q).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    wi, wl, _ = O.topk_batch(w.db, w.queries, ks)
    with P.Index(w.db, w.V) as idx:
        q = P.to_device_tokens(w.queries)
        kd = torch.from_numpy(ks).cuda()
        od = torch.from_numpy(off).cuda()
        for scan in (False, True):
            ids = torch.full((int(off[-1]),), -7, dtype=torch.int32, device="cuda")
            lcps = torch.full_like(ids, -7)
            idx.topk_dev(q, kd, od, int(ks.max()), ids, lcps, scan=scan)
            torch.cuda.synchronize()
            assert (ids.cpu().numpy() == wi).all() and (lcps.cpu().numpy() == wl).all()


def test_groups_far_beyond_the_staged_window(P):
    """Skewed data: 90% of rows share a 12-token prefix, so the groups around
    most queries span tens of thousands of sorted positions."""
    rng = np.random.default_rng(21)
    N, L = 120_000, 24
    db = synth.random_rows(rng, N, L, 4)
    hot = rng.random(N) < 0.9
    db[hot, :12] = 1
    qs = synth.random_rows(rng, 40, L, 4)
    qs[:30, :12] = 1
    qs[10:20, 12:] = db[hot][:10, 12:]
    ks = np.array([1, 10, 100, 1000] * 10, dtype=np.int32)
    check_against_oracle(P, db, qs, ks, 4, "skewed long groups")


def test_served_results_equal_alone(P):
    """Continuous batching on the GPU: every request's answer equals the
    oracle's answer for that request alone."""
    from paper_2602_04936_amd import serve
    w = synth.c3_like(200_000, 2000, seed=4)
    t, b, k = synth.serving_schedule(20000, 0.5, seed=5, k_mode="uniform")
    with P.Index(w.db, w.V) as idx:
        reqs = serve.requests_from_schedule(w.queries, t, b, k)
        rep = serve.run_served(idx, reqs, n_slots=3)
    assert rep["requests"] == len(reqs)
    for r in reqs[:: max(1, len(reqs) // 60)]:
        wi, wl, _ = oracle.c_topk(w.db, r.queries, r.k)
        assert (r.ids.reshape(-1) == wi).all() and (r.lcps.reshape(-1) == wl).all(), r.rid
