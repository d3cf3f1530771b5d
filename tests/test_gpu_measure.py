"""The atomic-rate measurement kernel: every FP64 add lands (the table sums
to the number of adds of both launches), in both tally patterns, and the
invalid arguments are refused before any launch."""
import pytest

from paper_1401_5469_amd import smc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scattered", [False, True], ids=["window", "scattered"])
def test_every_add_lands(scattered):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    table = torch.zeros(64 * 1000 + 64, dtype=torch.float64, device="cuda")
    rounds = 8
    rate = smc.measure_atomic_rate(table, rounds, scattered=scattered)
    assert rate > 0.0
    # two launches of 8 * n_cu workgroups of 256 lanes, `rounds` adds of 1.0 each
    assert float(table.sum().item()) == 2.0 * 8 * n_cu * 256 * rounds
    assert float(table.min().item()) >= 0.0
    if not scattered:
        # a wavefront adds to all 64 doubles of a window at once: each window
        # holds one count in all its entries
        rows = table.view(-1, 64)
        assert bool((rows == rows[:, :1]).all().item())


def test_invalid_arguments_are_refused():
    import torch
    table = torch.zeros(32, dtype=torch.float64, device="cuda")
    with pytest.raises(smc.SmcError):
        smc.measure_atomic_rate(table, 8)
    table = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(smc.SmcError):
        smc.measure_atomic_rate(table, 0)
