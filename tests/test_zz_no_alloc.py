"""fdot_modp_many_noalloc (the batched dot product on the library's fixed
scratch, no device allocation at the call) against fdot_modp_many_algo, the
entry point it mirrors, bit for bit: two calls in a row, the second on a
smaller batch, in every representation, through both batched launch forms
(plan inside the kernel for small batches, a separate plan launch for large
ones); and against the oracle on sampled pairs."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import NP_DTYPES as NP, TORCH_DTYPES, same, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

CASES = [(65521, "zpz", "delayed"), (4294967291, "zpz", "perterm"),
         (2147483647, "mont", "delayed"), (2147483647, "mont", "overflow"),
         (67108859, "fp64", "delayed"), (32749, "zech", "zech_exp"),
         (32749, "zech", "zech_tplus1"), (251, "centred", "delayed")]


def batch(p, rep, count, seed, max_n):
    """count pairs with lengths in [0, max_n) (some empty, some odd), each
    operand at its own offset of two pools so that pairs are misaligned."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(0, max_n, count)
    ns[::97] = 0
    offs = np.concatenate([[0], np.cumsum(ns + 3)])
    tot = int(offs[-1]) + 8
    X = stored(p, rep, tot, seed, 0)
    Y = stored(p, rep, tot, seed, 1)
    Xd, Yd = to_dev(X), to_dev(Y)
    xs = [Xd[int(offs[k]) + k % 3:int(offs[k]) + k % 3 + int(n)] for k, n in enumerate(ns)]
    ys = [Yd[int(offs[k]):int(offs[k]) + int(n)] for k, n in enumerate(ns)]
    host = [(X[int(offs[k]) + k % 3:int(offs[k]) + k % 3 + int(n)],
             Y[int(offs[k]):int(offs[k]) + int(n)]) for k, n in enumerate(ns)]
    return fd.Field.make_desc(xs, ys), host, (Xd, Yd)


@pytest.mark.parametrize("p,rep,algo", CASES, ids=lambda v: str(v))
def test_noalloc_matches_batched_entry_point(p, rep, algo):
    F = fd.Field(p, rep)
    for count, max_n, seed in ((1500, 6000, 1), (300, 3000, 2)):
        desc, host, keep = batch(p, rep, count, seed, max_n)
        # results start as garbage so that every written entry is checked
        got = torch.full((count,), 7, dtype=TORCH_DTYPES[rep], device="cuda")
        want = torch.full((count,), 5, dtype=TORCH_DTYPES[rep], device="cuda")
        F.dot_many_noalloc(desc, got, algo=algo)
        F.dot_many(desc, out=want, algo=algo)
        torch.cuda.synchronize()
        assert same(to_host(got), to_host(want)), (p, rep, algo, count)
        pick = list(range(0, count, max(1, count // 12))) + [count - 1]
        ref = oracle.dot_many(p, rep, [host[k][0] for k in pick], [host[k][1] for k in pick])
        assert same(to_host(got)[pick], ref), (p, rep, algo, count)


def test_noalloc_replayed_from_graph():
    """Captured into a HIP graph (the call allocates nothing), replayed with
    eager batched calls in between: every replay equals the eager result."""
    p, rep = 65521, "zpz"
    F = fd.Field(p, rep)
    desc, host, keep = batch(p, rep, 900, 3, 5000)
    want = F.dot_many(desc)
    s = torch.cuda.Stream()
    out = torch.zeros(900, dtype=TORCH_DTYPES[rep], device="cuda")
    with torch.cuda.stream(s):
        F.dot_many_noalloc(desc, out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        F.dot_many_noalloc(desc, out)
    other, _, keep2 = batch(p, rep, 200, 4, 3000)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert same(to_host(out), to_host(want))
        F.dot_many_noalloc(other, torch.empty(200, dtype=TORCH_DTYPES[rep], device="cuda"))
        torch.cuda.synchronize()


def test_noalloc_extension_field():
    F = fd.Field(2, "zech", degree=8)
    rng = np.random.default_rng(9)
    for count in (400, 50):
        xs = [torch.from_numpy(rng.integers(0, 256, int(n)).astype(np.uint16)).cuda()
              for n in rng.integers(0, 3000, count)]
        ys = [torch.from_numpy(rng.integers(0, 256, x.numel()).astype(np.uint16)).cuda()
              for x in xs]
        desc = fd.Field.make_desc(xs, ys)
        got = torch.empty(count, dtype=torch.uint16, device="cuda")
        F.dot_many_noalloc(desc, got)
        assert same(to_host(got), to_host(F.dot_many(desc)))


def test_noalloc_limits():
    F = fd.Field(65521, "zpz")
    out = torch.empty(1, dtype=torch.uint32, device="cuda")
    desc = torch.zeros((1, 3), dtype=torch.int64, device="cuda")
    L = fd.lib()
    import ctypes
    # more pairs than the fixed scratch holds: refused before any device work
    st = L.fdot_modp_many_noalloc(F.handle, 0, fd.NOALLOC_MAX_PAIRS + 1,
                                  ctypes.c_void_p(desc.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), None)
    assert st == -1
    assert L.fdot_modp_many_noalloc(F.handle, 0, 0, None, None, None) == 0
    # the largest batch it takes: every pair of length 1, x = y = p-1
    n = fd.NOALLOC_MAX_PAIRS
    v = torch.full((n,), 65520, dtype=torch.uint32, device="cuda")
    base = v.data_ptr()
    rows = torch.tensor([[base + 4 * k, base + 4 * k, 1] for k in range(0, n)],
                        dtype=torch.int64).cuda()
    got = torch.zeros(n, dtype=torch.uint32, device="cuda")
    F.dot_many_noalloc(rows, got)
    assert (got.cpu().numpy() == 1).all()  # (p-1)^2 = 1 mod p
