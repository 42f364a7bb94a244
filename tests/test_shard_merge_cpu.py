"""The exchange step a sharded deployment would use (each shard returns its
local top-k over an id range; one merge by (LCP desc, id asc)) gives the
global answer exactly.  Checked with the CPU oracle only; no device code."""
import numpy as np
import pytest

import synth
from oracle import lcp_oracle as O


def merge_shard_answers(answers, k):
    """answers: list of (ids, lcps) per shard (global ids, -1 padding)."""
    cand = [(-int(l), int(i)) for ids, lcps in answers for i, l in zip(ids, lcps) if i >= 0]
    cand.sort()
    ids = [i for _, i in cand[:k]] + [-1] * max(0, k - len(cand))
    lcps = [-d for d, _ in cand[:k]] + [-1] * max(0, k - len(cand))
    return np.array(ids), np.array(lcps)


@pytest.mark.parametrize("seed", range(5))
def test_union_of_local_topk_is_exact(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(50, 400))
    db = synth.random_rows(rng, N, 5, 3)
    cuts = np.sort(rng.choice(np.arange(1, N), size=int(rng.integers(1, 6)), replace=False))
    bounds = [0, *cuts.tolist(), N]
    for _ in range(15):
        q = db[rng.integers(0, N)] if rng.random() < 0.5 else synth.random_rows(rng, 1, 5, 3)[0]
        k = int(rng.integers(1, N + 3))
        answers = []
        for a, b in zip(bounds[:-1], bounds[1:]):
            ids, lcps = O.topk(db[a:b], q, k)
            answers.append((np.where(ids >= 0, ids + a, -1), lcps))
        got_ids, got_lcps = merge_shard_answers(answers, k)
        want_ids, want_lcps = O.topk(db, q, k)
        assert (got_ids == want_ids).all() and (got_lcps == want_lcps).all()
