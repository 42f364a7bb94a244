"""The energy sampler on the GPU: it returns a finite, positive J/query for a
short sustained run of the index path, or says why no figure is available."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_energy_sampler_on_the_gpu():
    import torch
    import paper_2602_04936_amd as P
    from paper_2602_04936_amd import energy
    dev = torch.device("cuda:0")
    meter, why = energy.try_meter(dev)
    if meter is None:
        assert isinstance(why, str) and why
        pytest.skip(f"no energy figure on this box: {why}")
    w = synth.c3_like(200_000, 2048, seed=18, k_fixed=10)
    with P.Index(w.db, w.V) as idx:
        q = P.to_device_tokens(w.queries)
        out = (torch.empty(w.Q * 10, dtype=torch.int32, device=dev), torch.empty(w.Q * 10, dtype=torch.int32, device=dev))

        def run():
            idx.topk(q, 10, out=out)
            return w.Q

        rep = meter.measure(run, 1.5, sync_every=16)
    meter.close()
    if rep.get("j_per_query") is None:
        assert rep.get("reason") or rep.get("error"), rep
        pytest.skip(f"no energy figure: {rep}")
    j = rep["j_per_query"]
    assert math.isfinite(j) and j > 0, rep
    assert rep["queries_per_s"] > 0 and rep["watts"] > 0, rep
