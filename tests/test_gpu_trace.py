"""Kernel trace: the event pairs the library records around each streaming
dot-product kernel, one per traced launch in launch order, each no longer
than the whole call measured around it on the same stream."""
import numpy as np
import pytest
import torch

from tests.gpu_helpers import stored, to_dev

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")


def test_trace_records_each_streaming_kernel():
    F = fd.Field(65521, "zpz")
    n = 1 << 22
    x, y = to_dev(stored(65521, "zpz", n, 7, 0)), to_dev(stored(65521, "zpz", n, 7, 1))
    desc = fd.Field.make_desc([x[:1000], x[5:n], y[:300000]] * 300, [y[:1000], y[5:n], x[:300000]] * 300)
    out = torch.empty(900, dtype=torch.uint32, device="cuda")
    F.dot_many(desc, out=out)  # code objects, workspace
    F.dot(x, y)
    torch.cuda.synchronize()
    fd.trace_enable(True)
    calls = []
    for k in range(4):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        if k % 2:
            F.dot(x, y)
        else:
            F.dot_many(desc, out=out)
        e.record()
        calls.append((s, e))
    fd.trace_enable(False)
    F.dot(x, y)  # not recorded
    ms = fd.trace_read()
    torch.cuda.synchronize()
    assert len(ms) == 4
    for (s, e), t in zip(calls, ms):
        assert 0.0 < t <= s.elapsed_time(e) + 1e-3
    # a new record starts empty
    fd.trace_enable(True)
    fd.trace_enable(False)
    assert len(fd.trace_read()) == 0
