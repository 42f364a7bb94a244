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


def test_c2_full(P):
    """c2 in full: N = 500,000, 10,000 queries (10% copies of rows), k = 10."""
    w = synth.c2_oom_boundary()
    assert w.Q == 10_000
    check_against_oracle(P, w.db, w.queries, w.k, w.V, "c2")


def test_c3_full_and_paths_agree(P):
    """c3 in full: N = 2,000,000, 8,192 queries with k uniform on {1, 10, 100};
    both paths against the C oracle for every query."""
    w = synth.c3_hierarchy()
    check_against_oracle(P, w.db, w.queries, w.k, w.V, "c3")


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


def _tie_shape(db, q, k):
    """(c, rows above c, tied rows at c) for one query, from the oracle's LCPs."""
    lc = O.lcp_against(db, q)
    G = np.cumsum(np.bincount(lc, minlength=db.shape[1] + 2)[::-1])[::-1]  # G[d] = rows with LCP >= d
    kp = min(int(k), db.shape[0])
    c = max(d for d in range(db.shape[1] + 1) if G[d] >= kp)
    return c, int(G[c + 1]), int(G[c] - G[c + 1])


def test_long_tied_blocks(P):
    """Rows tied at the cutoff number in the thousands to hundreds of
    thousands (V=4, one dominant symbol): the index kernel prunes them with the
    per-64-position id minima.  Both paths and the persistent launch against
    the oracle; the workload must reach the pruned selection (m <= 256 and at
    least 256*max(m, 8) tied rows), also with rows above the cutoff."""
    import torch
    w = synth.long_ties()
    pruned = with_inner = 0
    for qi in range(w.Q):
        c, n_gt, tn = _tie_shape(w.db, w.queries[qi], w.k[qi])
        m = min(int(w.k[qi]), w.N) - n_gt
        if c >= 1 and m <= 256 and tn >= 256 * max(m, 8):
            pruned += 1
            with_inner += n_gt > 0
    assert pruned >= 100 and with_inner >= 5, (pruned, with_inner)
    check_against_oracle(P, w.db, w.queries, w.k, w.V, "long tied blocks")
    qd = P.to_device_tokens(w.queries)
    with P.Index(w.db, w.V) as idx:
        ref = idx.topk(qd, w.k)
        kd = torch.from_numpy(w.k).cuda()
        od = torch.from_numpy(ref.offsets).cuda()
        cnt = torch.tensor([w.Q], dtype=torch.int64, device="cuda")
        for blocks in (0, 8):  # one wave per query; 32 looping waves
            ids = torch.full_like(ref.ids, -9)
            lcps = torch.full_like(ref.lcps, -9)
            idx.topk_persistent(qd, cnt, kd, od, int(w.k.max()), ids, lcps, blocks=blocks)
            torch.cuda.synchronize()
            assert torch.equal(ids, ref.ids) and torch.equal(lcps, ref.lcps), blocks


def _tie_case(rng, T, n_gt, n_other=300, L=6):
    """Rows for query 1 5 5 5 5 5 with exactly n_gt rows of LCP >= 2 (LCPs 2..6
    mixed), T rows of LCP exactly 1 and n_other of LCP 0, ids shuffled."""
    q = np.array([1, 5, 5, 5, 5, 5], np.uint8)[:L]
    inner = np.tile(q, (n_gt, 1))
    for i in range(n_gt):  # break the match at a random position >= 2 (or never)
        d = int(rng.integers(2, L + 1))
        if d < L:
            inner[i, d] = rng.choice([0, 2, 3, 4, 6, 7])
            inner[i, d + 1:] = rng.integers(0, 8, L - d - 1)
    tied = rng.integers(0, 8, (T, L)).astype(np.uint8)
    tied[:, 0] = 1
    tied[:, 1] = rng.choice(np.array([0, 2, 3, 4, 6, 7], np.uint8), T)
    other = rng.integers(0, 8, (n_other, L)).astype(np.uint8)
    other[:, 0] = rng.choice(np.array([0, 2, 3], np.uint8), n_other)
    db = np.concatenate([inner, tied, other])
    return db[rng.permutation(db.shape[0])], q[None, :]


@pytest.mark.parametrize("T,n_gt,k", [
    (512, 0, 16), (512, 0, 17), (512, 3, 259), (513, 0, 17), (512, 0, 257), (64, 0, 64),
    (3000, 2, 12), (20000, 5, 200), (60000, 5, 200), (200, 127, 128), (200, 63, 64), (200, 64, 66),
    (511, 120, 128), (64, 0, 16), (65, 2, 16), (128, 0, 10), (129, 3, 12),
    (513, 0, 1), (600, 0, 10), (640, 3, 16), (640, 0, 200), (641, 0, 10), (641, 2, 17)])
def test_tie_selection_boundaries(P, T, n_gt, k):
    """Each tie-selection path at its limits: wave minima (m <= 16, <= 512
    tied rows, also at 64 and 128 rows), bisection select (m <= 256 from at
    most 640 rows, and m <= 16 from 513 to 640 rows), pruned by block minima
    (long ranges), the sorted list otherwise; inner groups of up to 127 rows
    ranked by counting."""
    rng = np.random.default_rng(T * 1000 + n_gt * 7 + k)
    db, q = _tie_case(rng, T, n_gt)
    c, above, tn = _tie_shape(db, q[0], k)
    assert c == 1 and above == n_gt and tn == T, (c, above, tn)
    qs = np.repeat(q, 4, axis=0)
    check_against_oracle(P, db, qs, [k, 1, k, max(1, k - 1)], 8, f"ties T={T} n_gt={n_gt} k={k}")


@pytest.mark.parametrize("N,k", [(20000, 10), (300000, 1), (300000, 10), (300000, 16), (300000, 17)])
def test_scan_merge_paths(P, N, k):
    """Nearly every row ties with the query on its first L-1 tokens and a
    quarter match it exactly, so every scan chunk keeps k entries: partial
    lists of a few hundred to several thousand entries per query.  That covers
    each merge path: the few-answer passes (k <= 16, one pass up to 512
    entries, several passes up to 4,096) and the sorted list (k > 16, or more
    than 4,096 entries)."""
    rng = np.random.default_rng(N * 31 + k)
    L = 8
    q = rng.integers(0, 4, L).astype(np.uint8)
    db = np.tile(q, (N, 1))
    db[:, L - 1] = rng.integers(0, 4, N)
    early = rng.choice(N, N // 10, replace=False)  # some rows leave the query's prefix earlier
    db[early, 3] = (q[3] + 1 + rng.integers(0, 3, early.size)) % 4
    other = q.copy()
    other[0] = (q[0] + 1) % 4
    qs = np.stack([q, q, q, other])
    check_against_oracle(P, db, qs, [k, k, 1, k], 4, f"merge paths N={N} k={k}")


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


@pytest.mark.parametrize("seed", range(3))
def test_append_equals_build_over_concatenation(P, seed):
    """Appending rows (ids N, N+1, ...) yields the index a build over the
    concatenated rows would give: same order, adjacent LCP, id-order rows and
    answers; equal rows across batches keep ascending ids."""
    import torch
    rng = np.random.default_rng(300 + seed)
    L, V = [(6, 4), (24, 16), (9, 300)][seed]
    a = synth.random_rows(rng, 3000, L, V)
    b = np.concatenate([synth.random_rows(rng, 500, L, V), a[:50]])      # duplicates of old rows
    c = np.concatenate([b[10:20], synth.random_rows(rng, 37, L, V)])     # duplicates of appended rows
    whole = np.concatenate([a, b, c])
    qs = np.concatenate([synth.random_rows(rng, 40, L, V), whole[rng.integers(0, len(whole), 24)]])
    ks = rng.integers(1, 80, qs.shape[0]).astype(np.int32)
    with P.Index(a, V) as idx:
        idx.append(b)
        idx.append(c)
        assert idx.N == len(whole)
        va = {k: v.cpu().numpy() for k, v in idx.views().items()}
        ra = idx.topk(qs, ks)
        torch.cuda.synchronize()
        got = (ra.ids.cpu().numpy(), ra.lcps.cpu().numpy())
    with P.Index(whole, V) as ref:
        vb = {k: v.cpu().numpy() for k, v in ref.views().items()}
    for key in ("perm", "adj_lcp", "sorted_keys", "id_keys"):
        assert (va[key] == vb[key]).all(), key
    want = O.sorted_permutation(whole)
    assert (va["perm"] == want).all()
    wi, wl, _ = oracle.c_topk(whole, qs, ks)
    assert (got[0] == wi).all() and (got[1] == wl).all()


def test_append_rejects_out_of_range_and_keeps_index(P):
    import torch
    db = np.zeros((100, 4), np.uint8)
    with P.Index(db, 5) as idx:
        with pytest.raises(P.LcpError) as e:
            idx.append(np.full((3, 4), 9, np.uint8))
        assert e.value.status == -4 and idx.N == 100
        idx.append(np.ones((2, 4), np.uint8))
        r = idx.topk(np.ones((1, 4), np.uint8), 3)
        torch.cuda.synchronize()
        assert r.ids.cpu().tolist() == [100, 101, 0] and r.lcps.cpu().tolist() == [4, 4, 0]


def test_sensor_stream_with_appends(P):
    """The paced step loop: every step's answers equal the oracle's over the
    rows appended so far (including the steps right after each append)."""
    from paper_2602_04936_amd import serve
    st = synth.SensorStream(seed=77, sensors=200)
    hist = np.concatenate(list(st.steps(50)), axis=0)
    steps = list(st.steps(60))
    db = [hist]
    seen = []

    def append(index, batch):
        db.append(batch)
        index.append(batch)
        return index

    idx = P.Index(hist, 16)
    captured = []
    orig_topk = idx.topk

    def topk_and_keep(q, k, out=None, stream=None):
        r = orig_topk(q, k, out=out, stream=stream)
        captured.append((np.concatenate(db, axis=0).shape[0], r.ids[: q.shape[0] * k].cpu().numpy().copy(),
                         r.lcps[: q.shape[0] * k].cpu().numpy().copy()))
        return r

    idx.topk = topk_and_keep
    rep = serve.run_step_stream(idx, iter(steps), rate_hz=2000.0, k=5, append_every=20, append=append)
    rep.pop("index").close()
    assert rep["steps"] == 60 and rep["appends"] == 3
    whole = np.concatenate(db, axis=0)
    for t, (n_rows, ids, lcps) in enumerate(captured):
        wi, wl, _ = oracle.c_topk(whole[:n_rows], steps[t], 5)
        assert (ids == wi).all() and (lcps == wl).all(), t


def test_captured_persistent_launch_replays(P):
    """One persistent launch captured in a HIP graph, replayed for batches of
    different sizes and uneven k, with eager work and syncs in between: every
    replay equals the eager index path, and that equals the oracle for every query."""
    import torch
    from paper_2602_04936_amd import batching
    w = synth.c3_like(300_000, 3000, seed=12)
    qd = P.to_device_tokens(w.queries)
    with P.Index(w.db, w.V) as idx:
        ref = idx.topk(qd, w.k)
        torch.cuda.synchronize()
        ref_ids, ref_lcp = ref.ids.cpu().numpy(), ref.lcps.cpu().numpy()
        for blocks in (0, 16):  # one wave per query; a 64-wave grid whose waves loop
            cl = batching.CapturedLaunch(idx, cap_queries=3000, k_max=100, blocks=blocks)
            for n in (3000, 1000, 1, 0, 2999, 3000):
                ids, lcps, off = cl.run(qd[:n], w.k[:n])
                torch.cuda.synchronize()
                gi, gl = ids.cpu().numpy(), lcps.cpu().numpy()
                assert gi.shape[0] == int(w.k[:n].sum())
                assert (gi == ref_ids[: gi.shape[0]]).all() and (gl == ref_lcp[: gl.shape[0]]).all(), (blocks, n)
                idx.topk(qd[:7], 3)  # eager work between replays
                torch.cuda.synchronize()
            # back-to-back replays without a host sync in between (alternating staging buffers)
            outs = [tuple(t.clone() for t in cl.run(qd[:m], w.k[:m])[:2]) for m in (2000, 3000, 500)]
            torch.cuda.synchronize()
            for (gi, gl), m in zip(outs, (2000, 3000, 500)):
                tot = int(w.k[:m].sum())
                assert (gi.cpu().numpy() == ref_ids[:tot]).all() and (gl.cpu().numpy() == ref_lcp[:tot]).all()
        # the eager answers every replay was compared with, against the oracle for all 3,000 queries
        wi, wl, woff = oracle.c_topk(w.db, w.queries, w.k)
        assert (woff == ref.offsets).all()
        assert (ref_ids == wi).all() and (ref_lcp == wl).all()


def test_autotuned_shapes_agree(P):
    import torch
    from paper_2602_04936_amd import batching
    w = synth.c3_like(200_000, 1500, seed=13)
    qd = P.to_device_tokens(w.queries)
    with P.Index(w.db, w.V) as idx:
        res = batching.tune_launch(idx, qd, w.k, reps=2)
        assert res["best"].ms == min(s.ms for s in res["tried"])
        ref = idx.topk(qd, w.k)
        cnt = torch.tensor([w.Q], dtype=torch.int64, device="cuda")
        assert {s.order for s in res["tried"]} == {"given", "k_desc"}
        for shape in res["tried"]:
            ids = torch.full_like(ref.ids, -9)
            lcps = torch.full_like(ref.lcps, -9)
            batching.run_shape(idx, shape, batching.shape_inputs(qd, w.k, shape.order), 100, ids, lcps, cnt)
            torch.cuda.synchronize()
            assert torch.equal(ids, ref.ids) and torch.equal(lcps, ref.lcps), shape
        wi, wl, woff = oracle.c_topk(w.db, w.queries, w.k)
        assert (ref.ids.cpu().numpy() == wi).all() and (ref.lcps.cpu().numpy() == wl).all()


def test_captured_launch_in_largest_k_first_order(P):
    """A captured launch fed its batch with the largest k first (queries, k
    and offsets permuted together, by run and by stage + replay) answers in
    the batch's own layout, equal to the oracle for every query."""
    import torch
    from paper_2602_04936_amd import batching
    w = synth.c3_like(200_000, 2000, seed=14)
    qd = P.to_device_tokens(w.queries)
    wi, wl, woff = oracle.c_topk(w.db, w.queries, w.k)
    with P.Index(w.db, w.V) as idx:
        cl = batching.CapturedLaunch(idx, cap_queries=2000, k_max=100)
        for n in (2000, 777):
            order = batching.launch_order(w.k[:n], n, "k_desc")
            assert (np.diff(w.k[:n][order]) <= 0).all()
            ids, lcps, off = cl.run(qd[:n], w.k[:n], order=order)
            torch.cuda.synchronize()
            tot = int(w.k[:n].sum())
            assert (off == woff[:n + 1]).all()
            assert (ids.cpu().numpy() == wi[:tot]).all() and (lcps.cpu().numpy() == wl[:tot]).all(), n
        order = batching.launch_order(w.k, 2000, "k_desc")
        cl.q.copy_(qd[torch.from_numpy(order).cuda()])
        cl.stage(w.k, 2000, order=order)
        cl.replay()
        torch.cuda.synchronize()
        assert (cl.ids[:woff[-1]].cpu().numpy() == wi).all() and (cl.lcps[:woff[-1]].cpu().numpy() == wl).all()


def test_append_large_batch_and_after_a_rejected_one(P):
    """An append of more than 8,192 rows (radix-sorted on its own), then a
    rejected append (token >= V), then a small one: the index equals a build
    over the accepted rows at every point."""
    import torch
    rng = np.random.default_rng(77)
    L, V = 12, 16
    a = synth.random_rows(rng, 20000, L, V)
    b = np.concatenate([synth.random_rows(rng, 12000, L, V), a[:300]])
    c = synth.random_rows(rng, 50, L, V)
    qs = np.concatenate([synth.random_rows(rng, 30, L, V), a[:10], b[-10:], c[:5]])
    ks = rng.integers(1, 120, qs.shape[0]).astype(np.int32)
    with P.Index(a, V) as idx:
        g0 = idx.generation()
        idx.append(b)
        assert idx.generation() == g0 + 1
        bad = c.copy()
        bad[7, 3] = V
        with pytest.raises(P.LcpError) as e:
            idx.append(bad)
        assert e.value.status == -4 and idx.N == len(a) + len(b) and idx.generation() == g0 + 1
        for rows in ((a, b), (a, b, c)):
            whole = np.concatenate(rows)
            if len(rows) == 3:
                idx.append(c)
            va = {k: v.cpu().numpy() for k, v in idx.views().items()}
            r = idx.topk(qs, ks)
            torch.cuda.synchronize()
            with P.Index(whole, V) as ref:
                vb = {k: v.cpu().numpy() for k, v in ref.views().items()}
            for key in ("perm", "adj_lcp", "sorted_keys", "id_keys"):
                assert (va[key] == vb[key]).all(), (len(rows), key)
            wi, wl, _ = oracle.c_topk(whole, qs, ks)
            assert (r.ids.cpu().numpy() == wi).all() and (r.lcps.cpu().numpy() == wl).all()


def test_captured_launch_refuses_replay_after_append(P):
    """A graph captured before an append holds the old arrays: replaying it is
    refused on the host (nothing stale is launched); a new capture works."""
    import torch
    from paper_2602_04936_amd import batching
    w = synth.c3_like(50_000, 200, seed=15)
    qd = P.to_device_tokens(w.queries)
    with P.Index(w.db, w.V) as idx:
        cl = batching.CapturedLaunch(idx, cap_queries=200, k_max=100)
        cl.run(qd, w.k)
        torch.cuda.synchronize()
        idx.append(w.queries[:20])
        with pytest.raises(RuntimeError):
            cl.run(qd, w.k)
        cl2 = batching.CapturedLaunch(idx, cap_queries=200, k_max=100)
        gi, gl, _ = cl2.run(qd, w.k)
        ref = idx.topk(qd, w.k)
        torch.cuda.synchronize()
        assert torch.equal(gi, ref.ids) and torch.equal(gl, ref.lcps)
        wi, wl, _ = oracle.c_topk(np.concatenate([w.db, w.queries[:20]]), w.queries, w.k)
        assert (gi.cpu().numpy() == wi).all() and (gl.cpu().numpy() == wl).all()


@pytest.mark.parametrize("name", ["c1", "long_ties", "c3_like"])
def test_work_stats_match_the_oracle(P, name):
    """lcp_topk_stats: the cutoff c, the rows above it and the rows tied at it,
    per query, equal what the oracle's LCPs give; the answers equal lcp_topk."""
    import torch
    if name == "c1":
        w = synth.c1_tiny()
        sel = np.arange(w.Q)
    elif name == "long_ties":
        w = synth.long_ties()
        sel = np.arange(0, w.Q, 4)
    else:
        w = synth.c3_like(100_000, 300, seed=16)
        sel = np.arange(w.Q)
    qs, ks = w.queries[sel], w.k[sel]
    with P.Index(w.db, w.V) as idx:
        r, st = idx.topk_stats(qs, ks)
        ref = idx.topk(qs, ks)
        torch.cuda.synchronize()
        assert torch.equal(r.ids, ref.ids) and torch.equal(r.lcps, ref.lcps)
        st = st.cpu().numpy()
    for j in range(len(sel)):
        c, n_gt, tied = _tie_shape(w.db, qs[j], ks[j])
        assert tuple(st[j, :3]) == (c, n_gt, tied), (name, j)
        m = min(int(ks[j]), w.N) - n_gt
        assert (st[j, 3] == 0) == (m == 0) and (st[j, 3] == 1) == (m > 0 and c == 0)


@pytest.mark.parametrize("case", ["c1", "c2_like", "c3_like", "random_v2", "random_v300", "random_v65536",
                                  "tokens_beyond_v", "sparse_first_tokens"])
def test_first_token_directory_search(P, case):
    """Both insertion-point searches (65-ary tables, first-token directory)
    give the oracle's answers, also for query first tokens no row has and
    tokens >= V; switching the search bumps the generation."""
    import torch
    rng = np.random.default_rng(sum(map(ord, case)))
    if case == "c1":
        w = synth.c1_tiny()
        db, qs, ks, V = w.db, w.queries, w.k, w.V
    elif case == "c2_like":
        db = synth.prototype_rows(rng, synth.random_rows(rng, 512, 64, 256), 60000, 0.05, 256)
        qs = np.concatenate([synth.prototype_rows(rng, db[:512], 200, 0.05, 256), db[:50]])
        ks, V = rng.integers(1, 100, qs.shape[0]).astype(np.int32), 256
    elif case == "c3_like":
        w = synth.c3_like(150_000, 400, seed=19)
        db, qs, ks, V = w.db, w.queries, w.k, w.V
    elif case.startswith("random_v"):
        V = int(case[len("random_v"):])
        L = 9
        db = synth.random_rows(rng, 30000, L, V)
        qs = np.concatenate([synth.random_rows(rng, 100, L, V), db[rng.integers(0, 30000, 40)]])
        ks = rng.integers(1, 300, qs.shape[0]).astype(np.int32)
    elif case == "tokens_beyond_v":
        V = 300
        db = synth.random_rows(rng, 20000, 6, V)
        qs = synth.random_rows(rng, 64, 6, 65536)  # first tokens mostly >= V
        qs[:8, 0] = 299
        qs[8:16, 0] = 0
        ks = rng.integers(1, 40, 64).astype(np.int32)
    else:  # first tokens drawn from 5 of 4,096 values: most queries fall in empty buckets
        V = 4096
        db = synth.random_rows(rng, 20000, 5, V)
        db[:, 0] = rng.choice(np.array([3, 700, 701, 2048, 4095], np.uint16), 20000)
        qs = synth.random_rows(rng, 80, 5, V)
        qs[:40, 0] = db[rng.integers(0, 20000, 40), 0]
        ks = rng.integers(1, 70, 80).astype(np.int32)
    wi, wl, _ = oracle.c_topk(db, qs, ks)
    with P.Index(db, V) as idx:
        g0 = idx.generation()
        switches, cur = 0, idx.search_mode()
        for mode in (0, 1, 0):
            idx.set_search(mode)
            switches += mode != cur
            cur = mode
            assert idx.search_mode() == mode
            r = idx.topk(qs, ks)
            torch.cuda.synchronize()
            assert (r.ids.cpu().numpy() == wi).all() and (r.lcps.cpu().numpy() == wl).all(), (case, mode)
        assert idx.generation() == g0 + switches


def test_reserve_then_appends_equal_a_rebuild(P):
    """After lcp_index_reserve, appends up to the reserved size leave an index
    equal to a build over all rows; the generation counts the reserve and
    every append."""
    import torch
    st = synth.SensorStream(seed=91, sensors=300)
    hist = np.concatenate(list(st.steps(40)), axis=0)
    with P.Index(hist, 16) as idx:
        g0 = idx.generation()
        idx.reserve(idx.N + 5 * 300)
        assert idx.generation() == g0 + 1
        rows = [hist]
        for _ in range(5):
            b = st.step()
            idx.append(b)
            rows.append(b)
        assert idx.generation() == g0 + 6
        whole = np.concatenate(rows)
        va = {k: v.cpu().numpy() for k, v in idx.views().items()}
        qs = st.step()
        r = idx.topk(qs, 5)
        torch.cuda.synchronize()
    with P.Index(whole, 16) as ref:
        vb = {k: v.cpu().numpy() for k, v in ref.views().items()}
    for key in ("perm", "adj_lcp", "sorted_keys", "id_keys"):
        assert (va[key] == vb[key]).all(), key
    wi, wl, _ = oracle.c_topk(whole, qs, 5)
    assert (r.ids.cpu().numpy() == wi).all() and (r.lcps.cpu().numpy() == wl).all()


def test_build_picks_the_search_with_fewer_steps(P):
    """c2-like rows (first tokens spread over 256 values, buckets of about
    2,000 rows) take the directory; the c3 hierarchy (16 first tokens, buckets
    of 125,000 rows) keeps the search tables."""
    rng = np.random.default_rng(5)
    db = synth.prototype_rows(rng, synth.random_rows(rng, 4096, 64, 256), 500_000, 0.05, 256)
    with P.Index(db, 256) as idx:
        assert idx.search_mode() == 1
    w = synth.c3_like(2_000_000, 8, seed=20)
    with P.Index(w.db, w.V) as idx:
        assert idx.search_mode() == 0


@pytest.mark.parametrize("L,V", [(12, 16), (9, 300)])
def test_append_rows_equal_in_their_first_bytes(P, L, V):
    """Appended rows that agree on their first 8 bytes and differ later, and
    exact duplicates within the batch and of old rows, sort as a rebuild
    does (ties by id)."""
    import torch
    rng = np.random.default_rng(L * 1000 + V)
    old = synth.random_rows(rng, 4000, L, V)
    base = synth.random_rows(rng, 1, L, V)
    same_head = np.repeat(base, 600, axis=0)
    same_head[:, L - 3:] = synth.random_rows(rng, 600, 3, V)  # only the last 3 tokens differ
    batch = np.concatenate([same_head, same_head[:50], old[:40], same_head[::7]])
    batch = batch[rng.permutation(batch.shape[0])]
    whole = np.concatenate([old, batch])
    with P.Index(old, V) as idx:
        idx.append(batch)
        va = {k: v.cpu().numpy() for k, v in idx.views().items()}
    with P.Index(whole, V) as ref:
        vb = {k: v.cpu().numpy() for k, v in ref.views().items()}
    for key in ("perm", "adj_lcp", "sorted_keys", "id_keys"):
        assert (va[key] == vb[key]).all(), key
    assert (va["perm"] == O.sorted_permutation(whole)).all()


@pytest.mark.parametrize("k", [1, 10, 64, 65, 200, 300])
def test_scan_every_launch_shape(P, k):
    """The full scan splits a batch into query groups whose size and test
    (one query at a time, or the hashed pre-filter) depend on the batch size
    and k: batch sizes around each group-size boundary cover every compiled
    shape, each against the C oracle, bit-exact."""
    w = synth.c3_like(200_000, 256, seed=1031, k_fixed=k)
    seen = set()
    with P.Index(w.db, w.V) as idx:
        for Q in (1, 2, 5, 8, 12, 13, 16, 17, 32, 33, 64, 65, 200):
            qs = w.queries[:Q]
            seen.add(idx.scan_info(Q, k)[0] / Q)
            b = idx.scan_topk(qs, k)
            gi, gl = b.ids.cpu().numpy(), b.lcps.cpu().numpy()
            wi, wl, woff = oracle.c_topk(w.db, qs, k)
            _assert_equal(gi, gl, wi, wl, woff, f"scan Q={Q} k={k}")
    # shapes compiled per list size: k <= 64 six, k <= 128 three, k <= 256 two, above one
    assert len(seen) >= (4 if k <= 64 else 2 if k <= 256 else 1), seen
