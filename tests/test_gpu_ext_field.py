"""GPU parity of extension fields GF(p^d) in discrete logarithms (Sec. 2.4.2)
against the oracle's polynomial arithmetic, bit for bit: the modulus, the
code <-> value maps, dot products of ragged and misaligned lengths (both
schedules in characteristic 2: plus-one table and value XOR), the
elementwise operations, the batched form, and the refusal of the forms that
are not built for extensions.  A prime-field dot product on the same stream
after an extension one checks that the shared workspace is left as the
prime-field kernels expect it."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import same, to_dev, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

EXT = [(2, 2), (2, 8), (2, 16), (3, 2), (3, 10), (5, 6), (7, 5), (251, 2)]
OPS = ("add", "sub", "neg", "mul", "div", "axpy", "axpyin")

_fields = {}


def field(p, d):
    if (p, d) not in _fields:
        _fields[(p, d)] = fd.Field(p, "zech", degree=d)
    return _fields[(p, d)]


def codes(q, n, seed, stream):
    return synth.uniform_int(seed, stream, n, q).astype(np.uint16)


@pytest.mark.parametrize("p,d", EXT, ids=lambda v: str(v))
def test_ext_constants_and_maps(p, d):
    F = field(p, d)
    q = p ** d
    assert F.info["degree"] == d and F.info["q"] == q and F.info["p"] == p
    assert F.info["modulus"] == oracle.ext_modulus(p, d)
    values = np.arange(q, dtype=np.uint32)
    enc = to_host(F.encode(to_dev(values)))
    assert same(enc, oracle.ext_encode(p, d, values))
    dec = to_host(F.decode(to_dev(enc)))
    assert same(dec, values)


def schedules(p):
    """Dot-product schedules over GF(p^d): the plus-one table always, the
    value XOR in characteristic 2."""
    return ("auto", "zech_tplus1", "zech_exp") if p == 2 else ("auto", "zech_tplus1")


@pytest.mark.parametrize("p,d", EXT, ids=lambda v: str(v))
def test_ext_dot_matches_oracle(p, d):
    F = field(p, d)
    q = p ** d
    for algo in schedules(p):
        for n in (0, 1, 7, 8, 9, 1000, 100003):
            x = codes(q, n, 60 + n % 5, 0)
            y = codes(q, n, 60 + n % 5, 1)
            if n >= 8:
                x[:3] = [0, q - 1, 5 % (q - 1) + 1]   # zero, one, and a product with zero
                y[:3] = [q - 1, q - 1, 0]
            got = to_host(F.dot(to_dev(x), to_dev(y), algo=algo))[0]
            assert int(got) == oracle.ext_dot(p, d, x, y), (p, d, n, algo)
        # misaligned operands (element path)
        n = 50001
        x = codes(q, n + 1, 61, 0)
        y = codes(q, n + 1, 61, 1)
        xd, yd = to_dev(x), to_dev(y)
        got = to_host(F.dot(xd[1:], yd[1:], algo=algo))[0]
        assert int(got) == oracle.ext_dot(p, d, x[1:], y[1:]), (p, d, algo)
    if p != 2:
        with pytest.raises(fd.FdotError):
            F.dot(to_dev(codes(q, 16, 61, 0)), to_dev(codes(q, 16, 61, 1)), algo="zech_exp")


def test_ext_char2_value_schedule_cancels_pairs():
    """In characteristic 2 every element is its own negative: a vector
    dotted with itself twice over (x || x) . (y || y) sums each product twice
    and must give zero, through both schedules."""
    F = field(2, 16)
    x = codes(1 << 16, 40000, 67, 0)
    y = codes(1 << 16, 40000, 67, 1)
    xx, yy = to_dev(np.concatenate([x, x])), to_dev(np.concatenate([y, y]))
    for algo in ("zech_exp", "zech_tplus1"):
        assert int(to_host(F.dot(xx, yy, algo=algo))[0]) == 0, algo


def test_ext_dot_large_and_workspace_left_clean():
    p, d = 2, 16
    F = field(p, d)
    n = (1 << 22) + 5
    x = codes(p ** d, n, 62, 0)
    y = codes(p ** d, n, 62, 1)
    got = to_host(F.dot(to_dev(x), to_dev(y)))[0]
    assert int(got) == oracle.ext_dot(p, d, x, y)
    # a prime-field dot on the same stream, whose combination words share the
    # workspace the extension dot used for its partials
    G = fd.Field(32749, "zpz")
    u = synth.uniform_int(63, 0, 300001, 32749).astype(np.uint32)
    v = synth.uniform_int(63, 1, 300001, 32749).astype(np.uint32)
    for _ in range(3):
        assert same(to_host(G.dot(to_dev(u), to_dev(v))), [oracle.dot(32749, "zpz", u, v)])
        F.dot(to_dev(x[:1000]), to_dev(y[:1000]))


@pytest.mark.parametrize("p,d", EXT, ids=lambda v: str(v))
def test_ext_elementwise_matches_oracle(p, d):
    F = field(p, d)
    q = p ** d
    n = 10007
    x, y, r = (codes(q, n, 64, k) for k in range(3))
    x[:4] = [0, q - 1, 1, 0]
    y[:4] = [0, 0, q - 1, 1]                 # zero divisors among them
    alpha = int(codes(q, 1, 64, 3)[0])
    for op in OPS:
        ins_y = y if op in ("add", "sub", "mul", "div", "axpy") else None
        out = to_dev(r) if op == "axpyin" else None
        got = F.elementwise(op, to_dev(x), to_dev(ins_y) if ins_y is not None else None,
                            alpha=alpha if op in ("axpy", "axpyin") else None, out=out)
        want = oracle.ext_elementwise(p, d, op, x, ins_y, alpha if op in ("axpy", "axpyin") else None,
                                      r if op == "axpyin" else None)
        assert same(to_host(got), want), (p, d, op)


@pytest.mark.parametrize("p,d", [(2, 16), (3, 2), (251, 2)])
def test_ext_batched_dot_matches_oracle(p, d):
    """The batched form over an extension field: uneven lengths (empty,
    single, ragged, long), misaligned pairs, each result against the oracle."""
    F = field(p, d)
    q = p ** d
    count = 200 if q <= 4096 else 30  # the oracle rebuilds its tables per pair
    ns = [int(v) for v in synth.log_uniform_lengths(65, 0, count, 0.0, 4.5)]
    ns[:4] = [0, 1, 9, 300001 if p == 2 else 20001]
    xs, ys, hx, hy = [], [], [], []
    for k, n in enumerate(ns):
        off = k % 3  # some pairs start off the 16-byte grid
        a = codes(q, n + off, 66, 2 * k)
        b = codes(q, n + off, 66, 2 * k + 1)
        xs.append(to_dev(a)[off:])
        ys.append(to_dev(b)[off:])
        hx.append(a[off:])
        hy.append(b[off:])
    want = [oracle.ext_dot(p, d, hx[k], hy[k]) for k in range(len(ns))]
    for algo in schedules(p):
        got = to_host(F.dot_many(fd.Field.make_desc(xs, ys), algo=algo))
        for k in range(len(ns)):
            assert int(got[k]) == want[k], (p, d, k, ns[k], algo)


@pytest.mark.parametrize("p,d", [(2, 2), (3, 2), (2, 8), (7, 5)], ids=str)
def test_ext_one_code_step_small_fields(p, d):
    """The one-code plus-one step (eight table reads of a vector grouped; the
    form every field above 32768 elements takes) forced on small fields
    (tune key zech.packed = 0), where running sums, products and sums of the
    form 1 + g^k = 0 are frequent: single and batched dot products against
    the oracle."""
    q = p ** d
    fd.tune_set("zech.packed", 0)
    try:
        F = fd.Field(p, "zech", degree=d)
        for n in (8, 9, 1000, 100003):
            x = codes(q, n, 68 + n % 7, 0)
            y = codes(q, n, 68 + n % 7, 1)
            x[::5] = 0                      # zero products
            got = to_host(F.dot(to_dev(x), to_dev(y), algo="zech_tplus1"))[0]
            assert int(got) == oracle.ext_dot(p, d, x, y), (p, d, n)
        ns = [0, 1, 9, 4096, 20001]
        hx = [codes(q, n, 69, 2 * k) for k, n in enumerate(ns)]
        hy = [codes(q, n, 69, 2 * k + 1) for k, n in enumerate(ns)]
        got = to_host(F.dot_many(fd.Field.make_desc([to_dev(v) for v in hx],
                                                    [to_dev(v) for v in hy]), algo="zech_tplus1"))
        for k in range(len(ns)):
            assert int(got[k]) == oracle.ext_dot(p, d, hx[k], hy[k]), (p, d, k)
    finally:
        fd.tune_set("zech.packed", None)


def test_ext_unsupported_forms():
    F = field(3, 2)
    x = torch.zeros(16, dtype=torch.uint16, device="cuda")
    with pytest.raises(fd.FdotError):
        F.dot_many(fd.Field.make_desc([x], [x]), algo="zech_exp")
    with pytest.raises(fd.FdotError):
        F.gemm(x.reshape(4, 4), x.reshape(4, 4))
    with pytest.raises(fd.FdotError):
        F.gemv(x.reshape(4, 4), x[:4])
    with pytest.raises(fd.FdotError):
        fd.Field(2, "zech", degree=17)         # q > 65536
    with pytest.raises(fd.FdotError):
        fd.Field(4, "zech", degree=2)          # p not prime


@pytest.mark.parametrize("p,d", [(2, 2), (2, 8), (3, 2), (3, 5)], ids=str)
def test_ext_sums_exhaustive(p, d):
    """Sums, differences and AXPY over small extension fields (two codes per
    packed step, -1 = 1 in characteristic 2): every pair of codes."""
    F = field(p, d)
    q = p ** d
    c = np.arange(q, dtype=np.uint16)
    x, y = np.repeat(c, q), np.tile(c, q)
    r = codes(q, x.size, 65, 0)
    for op in ("add", "sub", "axpy", "axpyin"):
        for alpha in ((None,) if op in ("add", "sub") else (0, 1, q - 1, (q - 1) // 2 or 1)):
            ins_y = y if op != "axpyin" else None
            out = to_dev(r) if op == "axpyin" else None
            got = F.elementwise(op, to_dev(x), to_dev(ins_y) if ins_y is not None else None,
                                alpha=alpha, out=out)
            want = oracle.ext_elementwise(p, d, op, x, ins_y, alpha, r if op == "axpyin" else None)
            assert same(to_host(got), want), (p, d, op, alpha)
