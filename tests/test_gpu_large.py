"""The large single-stream workload (d = 1e6, ell = 100, 128-wide panels) at its full shapes.

The oracle costs a 1e6 x 100 Householder QR per product and two SVDs of 1e6-wide stacks, so it
is run once, on a prefix of the device-generated stream (one buffer folded by the query), with a
shortened iteration count q = 3 on both sides: every kernel runs at the workload's d and panel
width.
"""

import numpy as np
import pytest

from oracle import SFDOracle, evaluate

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(170)
def test_large_stream_prefix_matches_oracle(gpu_lib):
    import torch

    from workloads.device import stream_1e7_d1e6

    ptr, idx, val = stream_1e7_d1e6("cuda", n=3000)
    ptr_h, idx_h, val_h = ptr.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
    d, ell = 1_000_000, 100
    o = SFDOracle(d, ell, 0.25, 0, q=3, unit_roundoff=2.0 ** -24)
    o.append_csr(ptr_h, idx_h, val_h)
    sk = gpu_lib.Sketch(d, ell, 0.25, 0, q=3)
    sk.append_csr(ptr, idx, val)
    B = sk.sketch().cpu().numpy().astype(np.float64)
    Bo, live_o, _ = o.query()  # about a minute of FP64 work at d = 1e6: queried once
    assert sk.stats()["flushes"] == 0 and sk.last_live == live_o == ell - 1
    assert evaluate.gram_distance(B, Bo) <= 1e-4


def test_batch_streams_from_the_device_generator(gpu_lib):
    import torch

    from workloads.device import batch_streams_d2e4

    ptr, idx, val, starts = batch_streams_d2e4("cuda", streams=3, first=40)
    b = gpu_lib.Batch(3, 20_000, 32)
    b.append_csr(np.arange(3, dtype=np.int32), starts, ptr, idx, val)
    B = b.sketch()
    for s in range(3):
        one = gpu_lib.Sketch(20_000, 32, 0.25, 0, stream_id=s)
        lo, hi = int(starts[s]), int(starts[s + 1])
        one.append_csr(ptr[lo:hi + 1], idx, val)
        assert torch.equal(one.sketch(), B[s])
