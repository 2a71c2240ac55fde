"""The random-gather probe behind the bench line's gather peak: every thread
reads `iters` values of the buffer, so over a buffer of ones each sum is
exactly `iters`; sizes outside the documented limits are refused."""
import numpy as np
import pytest

from paper_1901_06229_amd import dock

pytestmark = pytest.mark.gpu


def test_gather_probe_reads_every_lane_and_times_itself():
    import torch
    buf = torch.ones(1 << 16, device="cuda:0")
    out = torch.zeros(64 * 256, device="cuda:0")
    ms = dock.dock_probe_gather(buf, out, 16, 64, 128)
    assert ms > 0.0
    assert np.array_equal(out.cpu().numpy(), np.full(64 * 256, 128.0, np.float32))
    for log2, blocks, iters in ((5, 64, 128), (16, 0, 128), (16, 64, 12)):
        with pytest.raises(dock.DockError) as e:
            dock.dock_probe_gather(buf, out, log2, blocks, iters)
        assert e.value.code == dock.DOCK_E_LIMIT
    with pytest.raises(dock.DockError) as e:
        dock.dock_probe_gather(torch.ones(1 << 16), out, 16, 64, 128)
    assert e.value.code == dock.DOCK_E_INVAL


def test_valu_probe_counts_its_chains_and_refuses_bad_sizes():
    """FMA chains with a = b = 1 add exactly one per iteration: every sum is
    8 iters + 8 (tid & 7) + 28; the evaluation mix gives finite sums."""
    import torch
    out = torch.zeros(32 * 256, device="cuda:0")
    ms = dock.dock_probe_valu(out, 0, 32, 1000)
    assert ms > 0.0
    tid = np.arange(32 * 256)
    assert np.array_equal(out.cpu().numpy(), (8 * 1000 + 8 * (tid & 7) + 28).astype(np.float32))
    assert dock.dock_probe_valu(out, 1, 32, 100) > 0.0
    assert np.isfinite(out.cpu().numpy()).all()
    for kind, blocks, iters, code in ((2, 32, 10, dock.DOCK_E_INVAL), (0, 0, 10, dock.DOCK_E_LIMIT),
                                      (1, 32, 0, dock.DOCK_E_LIMIT)):
        with pytest.raises(dock.DockError) as e:
            dock.dock_probe_valu(out, kind, blocks, iters)
        assert e.value.code == code
