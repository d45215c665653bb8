"""Every compute call captured into a HIP graph and replayed several times,
with eager work (new inputs written by the generator) and synchronisations
between the replays.  Each replay must equal the oracle on the inputs of
that moment and the eager call on the same inputs, bit for bit.  The
library clears its workspace with a fill kernel, never a memset node."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import same, storage_range, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

TD = {"zpz": torch.uint32, "mont": torch.uint32, "fp64": torch.float64,
      "zech": torch.uint16, "centred": torch.int8}
REPLAYS = 4


def refill(tensors, p, rep, seed):
    m, lo = storage_range(p, rep)
    for j, t in enumerate(tensors):
        synth.fill_device(t, seed, j, m, lo)


def capture(fn):
    s = torch.cuda.Stream()
    fd.workspace_reserve(4096, stream=s)
    with torch.cuda.stream(s):
        fn()  # eager on the capture stream: sizes its workspace and scratch
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        out = fn()
    torch.cuda.synchronize()
    capture.stream = s
    return g, out


def replay_and_check(g, out, inputs, p, rep, eager_fn, oracle_fn):
    for r in range(REPLAYS):
        refill(inputs, p, rep, 700 + r)
        torch.cuda.synchronize()
        out.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        got = to_host(out).reshape(-1).copy()
        host = [to_host(t) for t in inputs]
        assert same(got, np.asarray(oracle_fn(*host)).reshape(-1)), (p, rep, r)
        assert same(got, to_host(eager_fn()).reshape(-1)), (p, rep, r)


@pytest.mark.parametrize("p,rep", [(32749, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                                   (32749, "zech"), (251, "centred"), (4294967291, "zpz")])
def test_graph_single_dot(p, rep):
    F = fd.Field(p, rep)
    n = 300_007
    x = torch.empty(n, dtype=TD[rep], device="cuda")
    y = torch.empty(n, dtype=TD[rep], device="cuda")
    refill([x, y], p, rep, 699)
    g, out = capture(lambda: F.dot(x, y))
    replay_and_check(g, out, [x, y], p, rep, lambda: F.dot(x, y),
                     lambda xh, yh: oracle.dot(p, rep, xh, yh))


@pytest.mark.parametrize("p,rep", [(65521, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                                   (32749, "zech")])
def test_graph_batched_dot(p, rep):
    F = fd.Field(p, rep)
    ns = [0, 1, 5000, 70_001, 3, 250_000, 64, 131_073]
    xs = [torch.empty(n, dtype=TD[rep], device="cuda") for n in ns]
    ys = [torch.empty(n, dtype=TD[rep], device="cuda") for n in ns]
    inputs = xs + ys
    refill(inputs, p, rep, 699)
    desc = fd.Field.make_desc(xs, ys)
    g, out = capture(lambda: F.dot_many(desc))

    def want(*host):
        k = len(ns)
        return oracle.dot_many(p, rep, list(host[:k]), list(host[k:]))
    replay_and_check(g, out, inputs, p, rep, lambda: F.dot_many(desc), want)


@pytest.mark.parametrize("p,rep", [(65521, "zpz"), (1048573, "fp64"), (251, "centred")])
def test_graph_gemv_and_gemm(p, rep):
    F = fd.Field(p, rep)
    M, N, K = 200, 136, 520
    A = torch.empty((M, K), dtype=TD[rep], device="cuda")
    B = torch.empty((K, N), dtype=TD[rep], device="cuda")
    v = torch.empty(K, dtype=TD[rep], device="cuda")
    refill([A, B, v], p, rep, 699)
    g, out = capture(lambda: F.gemm(A, B))
    replay_and_check(g, out, [A, B], p, rep, lambda: F.gemm(A, B),
                     lambda a, b: oracle.gemm(p, rep, a, b))
    g2, out2 = capture(lambda: F.gemv(A, v))
    replay_and_check(g2, out2, [A, v], p, rep, lambda: F.gemv(A, v),
                     lambda a, b: oracle.gemv(p, rep, a, b))


def test_graph_replays_are_independent_of_history():
    """Eager batched calls on the capture stream after the capture, large
    enough to regrow that stream's workspace, do not disturb the graph: the
    buffers it captured stay allocated and its replays stay exact."""
    F = fd.Field(65521, "zpz")
    x = torch.empty(1 << 20, dtype=torch.uint32, device="cuda")
    y = torch.empty(1 << 20, dtype=torch.uint32, device="cuda")
    refill([x, y], 65521, "zpz", 698)
    desc1 = fd.Field.make_desc([x], [y])
    g, out = capture(lambda: F.dot_many(desc1))
    s = capture.stream
    want = oracle.dot(65521, "zpz", to_host(x), to_host(y))
    for r in range(REPLAYS):
        count = 5000 + 3000 * r  # beyond the reserved 4096 instances: the workspace grows
        big = [torch.empty(1000 * (r + 1), dtype=torch.uint32, device="cuda") for _ in range(2)]
        refill(big, 65521, "zpz", 800 + r)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            res = F.dot_many(fd.Field.make_desc([big[0]] * count, [big[1]] * count))
        torch.cuda.synchronize()
        one = oracle.dot(65521, "zpz", to_host(big[0]), to_host(big[1]))
        assert (to_host(res) == one).all(), r
        out.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        assert same(to_host(out)[0], want), r


@pytest.mark.parametrize("p,rep", [(65521, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                                   (32749, "zech"), (251, "centred")])
def test_graph_elementwise(p, rep):
    """Every elementwise operation captured once and replayed on new inputs."""
    F = fd.Field(p, rep)
    n = 100_003
    x = torch.empty(n, dtype=TD[rep], device="cuda")
    y = torch.empty(n, dtype=TD[rep], device="cuda")
    refill([x, y], p, rep, 699)
    alpha = int(synth.uniform_int(5, 5, 1, *storage_range(p, rep))[0])
    for op in ("add", "sub", "neg", "mul", "div", "axpy"):
        kw = {"alpha": alpha} if op == "axpy" else {}
        yy = None if op == "neg" else y
        g, out = capture(lambda: F.elementwise(op, x, yy, **kw))

        def want(xh, yh, op=op, kw=kw):
            return oracle.elementwise(p, rep, op, xh, None if op == "neg" else yh, **kw)
        replay_and_check(g, out, [x, y], p, rep, lambda: F.elementwise(op, x, yy, **kw), want)


def test_graph_extension_field_dot():
    """Dot products over GF(2^16) captured once and replayed; their partials
    share the capture stream's workspace with the prime-field kernels, so a
    prime-field dot is replayed in the same graph after it."""
    E = fd.Field(2, "zech", degree=16)
    P = fd.Field(32749, "zpz")
    n = 300_007
    x = torch.empty(n, dtype=torch.uint16, device="cuda")
    y = torch.empty(n, dtype=torch.uint16, device="cuda")
    u = torch.empty(n, dtype=torch.uint32, device="cuda")
    v = torch.empty(n, dtype=torch.uint32, device="cuda")

    def both():  # both GF(2^16) schedules (value XOR, plus-one table), then GF(32749)
        return torch.cat([E.dot(x, y, algo="zech_exp").to(torch.int64),
                          E.dot(x, y, algo="zech_tplus1").to(torch.int64),
                          P.dot(u, v).to(torch.int64)])
    for r in range(REPLAYS):
        synth.fill_device(x, 710 + r, 0, 1 << 16, 0)
        synth.fill_device(y, 710 + r, 1, 1 << 16, 0)
        synth.fill_device(u, 710 + r, 2, 32749, 0)
        synth.fill_device(v, 710 + r, 3, 32749, 0)
        torch.cuda.synchronize()
        if r == 0:
            g, out = capture(both)
        out.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        got = to_host(out)
        want = oracle.ext_dot(2, 16, to_host(x), to_host(y))
        assert int(got[0]) == want and int(got[1]) == want, r
        assert int(got[2]) == int(oracle.dot(32749, "zpz", to_host(u), to_host(v))), r
