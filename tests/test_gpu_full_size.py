"""GPU parity of the two loop workloads at their full sizes, every answer
against the C oracle, bit-exact:

  - the serving loop on the 2,000,000-row hierarchy database (L = 32 uint16,
    V = 4,096), Poisson arrivals at 10,000 queries/s for 2 s, 1-256 queries
    per request (log-uniform), k uniform on [1, 100]: every served request;
  - the sensor-fusion stream: 1,000 sensors, 1,000,000 history rows (L = 24
    uint8, V = 16), 1,050 steps of 1,000 queries at k = 5, step 999's
    readings appended after it: every step after the append and every tenth
    step before it.
"""
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


def test_served_full_size_k_uniform(P):
    from paper_2602_04936_amd import serve
    w = synth.c3_hierarchy()
    t, b, k = synth.serving_schedule(10000.0, 2.0, seed=1004, k_mode="uniform")
    print(f"served: N={w.N} requests={len(t)} queries={int(b.sum())}", flush=True)
    with P.Index(w.db, w.V) as idx:
        reqs = serve.requests_from_schedule(w.queries, t, b, k)
        rep = serve.run_served(idx, reqs, n_slots=3)
    assert rep["requests"] == len(reqs)
    qs = np.concatenate([r.queries for r in reqs])
    ks = np.concatenate([np.full(r.b, r.k, np.int32) for r in reqs])
    wi, wl, _ = oracle.c_topk(w.db, qs, ks)
    gi = np.concatenate([r.ids.reshape(-1) for r in reqs])
    gl = np.concatenate([r.lcps.reshape(-1) for r in reqs])
    if not ((gi == wi).all() and (gl == wl).all()):
        bad = int(np.nonzero((gi != wi) | (gl != wl))[0][0])
        pos = np.cumsum([0] + [r.b * r.k for r in reqs])
        rid = int(np.searchsorted(pos, bad, side="right") - 1)
        raise AssertionError(f"served request {reqs[rid].rid} differs from the oracle")


def test_sensor_stream_full_size_with_append(P):
    from paper_2602_04936_amd import serve
    st = synth.SensorStream(seed=1005)
    hist = np.concatenate(list(st.steps(1000)), axis=0)
    steps = list(st.steps(1050))
    assert hist.shape == (1_000_000, 24)

    def checked(t):
        return t >= 999 or t % 10 == 0

    def append(index, batch):
        index.append(batch)
        return index

    idx = P.Index(hist, synth.SensorStream.V)
    rep = serve.run_step_stream(idx, iter(steps), rate_hz=4000.0, k=5, append_every=1000, append=append,
                                keep=checked)
    rep.pop("index").close()
    assert rep["steps"] == 1050 and rep["appends"] == 1
    got = rep["answers"]
    assert sorted(got) == [t for t in range(1050) if checked(t)]
    print(f"sensor stream: {len(got)} steps checked, p99 step {rep['p99_step_ms']} ms", flush=True)
    # steps up to 999 see the history; later ones also the appended step 999
    for db, ts in ((hist, [t for t in got if t <= 999]),
                   (np.concatenate([hist, steps[999]]), [t for t in got if t >= 1000])):
        qs = np.concatenate([steps[t] for t in ts])
        wi, wl, _ = oracle.c_topk(db, qs, 5)
        wi = wi.reshape(len(ts), -1, 5)
        wl = wl.reshape(len(ts), -1, 5)
        for j, t in enumerate(ts):
            assert (got[t][0] == wi[j]).all() and (got[t][1] == wl[j]).all(), t
