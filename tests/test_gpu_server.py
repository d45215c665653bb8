"""The request server on the GPU: a Poisson stream of dot, matrix-vector and
matrix products over the five primes of the served workload, in one mix.
Every result must be bit-identical to the same request computed alone (the
arithmetic is exact, so the tolerance is zero), and a sample is checked
against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import same, storage_range, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

# prime -> representation used for dot/gemv, and for gemm
PRIMES = {251: ("zpz", "centred"), 32749: ("zpz", "zpz"), 65521: ("zpz", "zpz"),
          67108859: ("fp64", "fp64"), 2147483647: ("mont", "mont")}
TD = {"zpz": torch.uint32, "mont": torch.uint32, "fp64": torch.float64, "centred": torch.int8}


def fill(t, p, rep, seed, stream):
    m, lo = storage_range(p, rep)
    synth.fill_device(t, seed, stream, m, lo)


def build_mix(n_req, seed):
    rng = np.random.default_rng(seed)
    fields, reqs, outs, meta = {}, [], [], []
    bufs = {}
    for p, (r1, r2) in PRIMES.items():
        for rep in {r1, r2}:
            fields[(p, rep)] = fd.Field(p, rep)
    for i in range(n_req):
        p = list(PRIMES)[rng.integers(len(PRIMES))]
        u = rng.random()
        if u < 0.6:
            op, n = "dot", int(10 ** rng.uniform(2, 5))
            rep = PRIMES[p][0]
            x = torch.empty(n, dtype=TD[rep], device="cuda"); fill(x, p, rep, 90 + i, 0)
            y = torch.empty(n, dtype=TD[rep], device="cuda"); fill(y, p, rep, 90 + i, 1)
            out = torch.empty(1, dtype=TD[rep], device="cuda")
            kw = dict(n=n)
        elif u < 0.9:
            op, m, n = "gemv", int(rng.integers(20, 400)), int(rng.integers(20, 400))
            rep = PRIMES[p][0]
            x = torch.empty((m, n), dtype=TD[rep], device="cuda"); fill(x, p, rep, 90 + i, 0)
            y = torch.empty(n, dtype=TD[rep], device="cuda"); fill(y, p, rep, 90 + i, 1)
            out = torch.empty(m, dtype=TD[rep], device="cuda")
            kw = dict(m=m, n=n)
        else:
            op, m, n, k = "gemm", *[int(v) for v in rng.integers(8, 160, 3)]
            rep = PRIMES[p][1]
            x = torch.empty((m, k), dtype=TD[rep], device="cuda"); fill(x, p, rep, 90 + i, 0)
            y = torch.empty((k, n), dtype=TD[rep], device="cuda"); fill(y, p, rep, 90 + i, 1)
            out = torch.empty((m, n), dtype=TD[rep], device="cuda")
            kw = dict(m=m, n=n, k=k)
        F = fields[(p, rep)]
        bufs[i] = (x, y)
        reqs.append(fd.make_request(op, F, x, y, out, **kw))
        outs.append(out)
        meta.append((op, p, rep, F, x, y))
    return fields, reqs, outs, meta, bufs


def alone(meta):
    res = []
    for op, p, rep, F, x, y in meta:
        if op == "dot":
            res.append(to_host(F.dot(x, y)))
        elif op == "gemv":
            res.append(to_host(F.gemv(x, y)))
        else:
            res.append(to_host(F.gemm(x, y)))
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("plain", [False, True])
def test_served_mix_equals_alone(plain):
    fields, reqs, outs, meta, bufs = build_mix(240, 11)
    want = alone(meta)
    for o in outs:
        o.zero_()
    torch.cuda.synchronize()
    srv = fd.Server(plain=plain, hbm_budget=1 << 30, max_inflight=64, streams=4)
    arrivals = np.cumsum(np.random.default_rng(12).exponential(2e-5, len(reqs)))
    tm = srv.replay(reqs, arrivals)
    assert (tm["status"] == 0).all()
    for i, (o, w) in enumerate(zip(outs, want)):
        assert same(to_host(o), w), (i, meta[i][:3])
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["peak_footprint"] <= 1 << 30
    if not plain:
        assert tm["batch_size"].max() > 1  # dots of one field were fused
    srv.close()
    # a sample against the oracle
    for i in range(0, len(reqs), 17):
        op, p, rep, F, x, y = meta[i]
        xh, yh = to_host(x), to_host(y)
        if op == "dot":
            ref = oracle.dot(p, rep, xh, yh)
        elif op == "gemv":
            ref = oracle.gemv(p, rep, xh, yh)
        else:
            ref = oracle.gemm(p, rep, xh, yh)
        assert same(np.asarray(want[i]).reshape(np.shape(ref)), ref), (i, op, p, rep)


def test_served_burst_and_back_pressure():
    """Everything arrives at once into a small queue: the load generator
    retries on back-pressure, all results still exact."""
    fields, reqs, outs, meta, bufs = build_mix(150, 13)
    want = alone(meta)
    srv = fd.Server(max_queue=16, max_inflight=8, hbm_budget=64 << 20)
    tm = srv.replay(reqs, np.zeros(len(reqs)))
    assert (tm["status"] == 0).all()
    for o, w in zip(outs, want):
        assert same(to_host(o), w)
    assert srv.stats()["peak_inflight"] <= 8
    srv.close()


def test_ready_event_orders_operands():
    """Operands written on another stream: each request names the event
    recorded after its operands, and its launch waits for it."""
    p, rep = 65521, "zpz"
    F = fd.Field(p, rep)
    side = torch.cuda.Stream()
    n = 1 << 20
    src = [torch.empty(n, dtype=torch.uint32, device="cuda") for _ in range(2)]
    fill(src[0], p, rep, 70, 0)
    fill(src[1], p, rep, 70, 1)
    torch.cuda.synchronize()
    x = torch.zeros(n, dtype=torch.uint32, device="cuda")
    y = torch.zeros(n, dtype=torch.uint32, device="cuda")
    out = torch.empty(1, dtype=torch.uint32, device="cuda")
    A = torch.zeros((512, 512), dtype=torch.uint32, device="cuda")
    v = torch.empty(512, dtype=torch.uint32, device="cuda")
    yv = torch.empty(512, dtype=torch.uint32, device="cuda")
    torch.cuda.synchronize()
    srv = fd.Server(streams=4)
    with torch.cuda.stream(side):
        for _ in range(20):  # keep the side stream busy for a while first
            x.copy_(src[1])
        x.copy_(src[0])
        y.copy_(src[1])
        A.copy_(src[0][:512 * 512].view(512, 512))
        v.copy_(src[1][:512])
        ev = torch.cuda.Event()
        ev.record(side)
    t1 = srv.submit(fd.make_request("dot", F, x, y, out, n=n, ready=ev))
    t2 = srv.submit(fd.make_request("gemv", F, A, v, yv, m=512, n=512, ready=ev))
    srv.drain(60000)
    assert srv.poll(t1)[1].status == 0 and srv.poll(t2)[1].status == 0
    srv.close()
    torch.cuda.synchronize()
    xh, yh = to_host(src[0]), to_host(src[1])
    assert same(to_host(out), oracle.dot(p, rep, xh, yh).reshape(1))
    assert same(to_host(yv), oracle.gemv(p, rep, xh[:512 * 512].reshape(512, 512), yh[:512]))
