"""The measurement kernels: the latency probe changes no word of its buffer
(its compare-and-swaps expect and write 1, its stores write back the value
just read) and reports a positive time for every kind of access; the
random-read probe reads only inside its buffer (its sink is written, the
buffer is not)."""

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_latency_probe_leaves_buffer_unchanged():
    import torch
    from paper_1712_09624_amd import ckpp
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(3)
    host = rng.integers(0, 4, size=(1 << 20) // 8, dtype=np.int64)  # many words are 1
    buf = torch.from_numpy(host).to(dev)
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    for kind in ckpp.LATENCY_KINDS:
        say(f"latency probe kind={kind}")
        ckpp.probe_latency(buf, kind, 500, 11, out)
        torch.cuda.synchronize()
        assert int(out[0].item()) > 0
    assert np.array_equal(buf.cpu().numpy(), host), "the probe changed its buffer"
    with pytest.raises(ckpp.CkppError):
        ckpp.probe_latency(buf[:16], "load", 10, 1, out)  # 128 bytes: below 256


def test_random_read_probe_writes_only_its_sink():
    import torch
    from paper_1712_09624_amd import ckpp
    dev = torch.device("cuda", 0)
    host = np.arange((1 << 22) // 8, dtype=np.int64)
    buf = torch.from_numpy(host).to(dev)
    grid = 16
    sink = torch.zeros(grid * 256, dtype=torch.int64, device=dev)
    for coop in (False, True):
        for granule in (32, 64, 128):
            say(f"random-read probe granule={granule} coop={coop}")
            ckpp.probe_random_reads(buf, granule, 1 << 16, 4, 256, grid, 5, sink, coop)
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), host)
