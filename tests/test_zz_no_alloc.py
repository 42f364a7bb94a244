"""The allocation-free full scan (lcp_scan_topk_dev_noalloc, fixed device
scratch) against the allocating one (lcp_scan_topk_dev): bit-identical ids
and LCPs on two calls in a row, the second with a smaller batch and smaller
k, and both against the CPU oracle.  A batch too large for the fixed scratch
is rejected on the host, before anything is launched."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2602_04936_amd as P
    torch.cuda.init()
    return P


def _run(P, idx, qd, ks, noalloc):
    import torch
    off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    kd = torch.from_numpy(ks).cuda()
    od = torch.from_numpy(off).cuda()
    ids = torch.full((int(off[-1]),), -7, dtype=torch.int32, device="cuda")
    lcps = torch.full_like(ids, -7)
    idx.topk_dev(qd, kd, od, int(ks.max()), ids, lcps, scan=True, noalloc=noalloc)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), lcps.cpu().numpy()


def test_noalloc_scan_equals_allocating_scan_twice(P):
    w = synth.c3_like(300_000, 2048, seed=31)  # k uniform on {1, 10, 100}
    rng = np.random.default_rng(32)
    with P.Index(w.db, w.V) as idx:
        # first call: 2,048 queries, k up to 100; second: 300 queries, k up to 40
        for n, kmax in ((2048, 100), (300, 40)):
            sel = rng.choice(w.Q, n, replace=False)
            qs = w.queries[sel]
            ks = w.k[sel] if kmax == 100 else rng.integers(1, kmax + 1, n).astype(np.int32)
            qd = P.to_device_tokens(qs)
            want = _run(P, idx, qd, ks, noalloc=False)
            got = _run(P, idx, qd, ks, noalloc=True)
            assert (got[0] == want[0]).all() and (got[1] == want[1]).all(), (n, kmax)
            wi, wl, _ = oracle.c_topk(w.db, qs, ks)
            assert (got[0] == wi).all() and (got[1] == wl).all(), (n, kmax)


def test_noalloc_rejects_batches_beyond_the_scratch(P):
    import torch
    w = synth.c3_like(20_000, 64, seed=33)
    with P.Index(w.db, w.V) as idx:
        # 65,536 queries at k = 1024 need about 1 GiB of partial lists
        Q = 65536
        qd = torch.zeros((Q, w.L), dtype=torch.int16, device="cuda")
        kd = torch.full((Q,), 1024, dtype=torch.int32, device="cuda")
        od = torch.arange(Q + 1, dtype=torch.int64, device="cuda") * 1024
        out = torch.empty(1, dtype=torch.int32, device="cuda")  # never written: nothing is launched
        with pytest.raises(P.LcpError) as e:
            idx.topk_dev(qd, kd, od, 1024, out, out, scan=True, noalloc=True)
        assert e.value.status == -1 and "fixed scratch" in str(e.value)
        torch.cuda.synchronize()
