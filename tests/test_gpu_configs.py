"""GPU parity at each benchmark workload's own size and launch configuration.

Every workload the benchmark times is compared here with the oracle, bit for
bit, on the very operands the kernels read (copied back from the device),
through the same calls and default tuning the benchmark uses:

* the single dot product over GF(32749), n = 10^6 (seed 1): the 64 distinct
  pairs the benchmark streams cold, eager and replayed from one HIP graph;
* the 4096-pair batch with lengths log-uniform in [10^3, 10^6] (seed 2) in
  its three batches (65521 delayed, 2^31-1 Montgomery, 4294967291 per term):
  every pair;
* 1024 pairs of length 4*10^6 (seed 3): residues in doubles modulo 2^26-5
  (a fold every two products) and discrete-log codes modulo 32749 in both
  accumulation schedules: every pair, checked in slices of the batch so that
  the host holds one slice at a time.

The results are exact, so the bar is equality of every result's bits (the
dot product is the building block of Sec. 1, each pair one result).
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import same, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")
bench = pytest.importorskip("bench")


def check_batch(b, step=64):
    """Every pair of a device-resident benchmark batch against the oracle,
    `step` pairs at a time (operands copied back per slice)."""
    got = to_host(b.out)
    for k0 in range(0, len(b.ns), step):
        k1 = min(k0 + step, len(b.ns))
        lo, hi = int(b.offs[k0]), int(b.offs[k1])
        X = to_host(b.X[lo:hi])
        Y = to_host(b.Y[lo:hi])
        xs = [X[int(b.offs[k]) - lo:int(b.offs[k]) - lo + int(b.ns[k])] for k in range(k0, k1)]
        ys = [Y[int(b.offs[k]) - lo:int(b.offs[k]) - lo + int(b.ns[k])] for k in range(k0, k1)]
        want = oracle.dot_many(b.p, b.rep, xs, ys)
        bad = np.nonzero(got[k0:k1] != want)[0]
        assert bad.size == 0, (b.p, b.rep, b.algo, [int(k0 + i) for i in bad[:8]])


def test_single_dot_1e6():
    """The single form at p = 32749, n = 10^6 on the benchmark's 64 buffer
    pairs (x = stream 2i, y = stream 2i+1 of seed 1), eager and as one
    replayed HIP graph of 64 calls."""
    import synth
    p, n, pairs = 32749, 1_000_000, 64
    F = fd.Field(p, "zpz")
    X = torch.empty((pairs, n), dtype=torch.uint32, device="cuda")
    Y = torch.empty((pairs, n), dtype=torch.uint32, device="cuda")
    for i in range(pairs):
        synth.fill_device(X[i], 1, 2 * i, p)
        synth.fill_device(Y[i], 1, 2 * i + 1, p)
    Xh, Yh = to_host(X), to_host(Y)
    want = oracle.dot_many(p, "zpz", list(Xh), list(Yh))
    # pair 0 is the workload itself: its operands are the generator's
    assert same(Xh[0], synth.uniform_int(1, 0, n, p).astype(np.uint32))
    assert same(Yh[0], synth.uniform_int(1, 1, n, p).astype(np.uint32))
    out = torch.empty(pairs, dtype=torch.uint32, device="cuda")
    for i in range(pairs):
        F.dot(X[i], Y[i], out=out[i:i + 1])
    assert same(to_host(out), want)

    def cold():
        for i in range(pairs):
            F.dot(X[i], Y[i], out=out[i:i + 1])

    s = torch.cuda.Stream()
    fd.workspace_reserve(4096, stream=s)
    with torch.cuda.stream(s):
        cold()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cold()
    for _ in range(3):
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same(to_host(out), want)


@pytest.mark.parametrize("which", range(3), ids=[lab for *_, lab in bench.BATCHES])
def test_batched_4096_pairs(which):
    """Every one of the 4096 pairs of a benchmark batch, after warm-up calls
    and timed-loop calls like the benchmark's."""
    p, rep, algo, _ = bench.BATCHES[which]
    ns = bench.lengths_config2()
    b = bench.Batch(fd, p, rep, algo, ns, torch.uint32)
    for _ in range(3):
        b.out.fill_(0)
        b.run()
    torch.cuda.synchronize()
    check_batch(b, step=512)


@pytest.mark.parametrize("p,rep,algo,dtype", [
    (67108859, "fp64", "delayed", torch.float64),
    (32749, "zech", "zech_exp", torch.uint16),
    (32749, "zech", "zech_tplus1", torch.uint16)], ids=["fp64", "zech_exp", "zech_tplus1"])
def test_batched_1024_pairs_of_4e6(p, rep, algo, dtype):
    """1024 pairs of 4*10^6 elements (65.5 GB of doubles, 16.4 GB of codes),
    every pair against the oracle."""
    ns = np.full(1024, 4_000_000, dtype=np.int64)
    b = bench.Batch(fd, p, rep, algo, ns, dtype, seed=3)
    b.out.fill_(0)
    b.run()
    b.run()
    torch.cuda.synchronize()
    try:
        check_batch(b, step=64)
    finally:
        del b
        torch.cuda.empty_cache()
