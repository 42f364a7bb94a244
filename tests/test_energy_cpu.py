"""Energy sampler without a GPU driver: it reports why no figure is available
instead of failing the caller."""
import pytest


def test_energy_meter_reports_unavailable_without_driver():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; tests/test_energy_gpu.py exercises the sampler there")
    from paper_2602_04936_amd import energy
    meter, why = energy.try_meter("cuda:0")
    assert meter is None
    assert isinstance(why, str) and why
