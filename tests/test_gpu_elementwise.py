"""GPU parity of the elementwise field operations (fdot_elementwise) against
the oracle, bit for bit: the seven operations of Sec. 2 in every
representation, lengths that leave ragged tails of the 16-byte vector path,
misaligned operands (element-wise path), in-place results, zero divisors and
the edge elements 0, 1 and p-1."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import ELEM_BYTES, TORCH_DTYPES, same, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

OPS = ("add", "sub", "neg", "mul", "div", "axpy", "axpyin")
FIELDS = [(32749, "zpz"), (65521, "zpz"), (2147483647, "zpz"), (4294967291, "zpz"), (2, "zpz"),
          (2147483647, "mont"), (65521, "mont"), (2654435761, "mont"),
          (67108859, "fp64"), (1048573, "fp64"), (2, "fp64"),
          (32749, "zech"), (65521, "zech"), (3, "zech"),
          (251, "centred"), (3, "centred")]

_fields = {}


def field(p, rep):
    if (p, rep) not in _fields:
        _fields[(p, rep)] = fd.Field(p, rep)
    return _fields[(p, rep)]


def inputs(p, rep, n, seed):
    x = stored(p, rep, n, seed, 0)
    y = stored(p, rep, n, seed, 1)
    r = stored(p, rep, n, seed, 2)
    edge = oracle.encode(p, rep, [0, 1 % p, p - 1, 0, 1 % p, p - 1])
    k = min(n, 6)
    x[:k] = edge[:k]
    y[:k] = edge[::-1][:k]       # zero divisors among them
    alpha = stored(p, rep, 1, seed, 3)[0]
    return x, y, r, alpha


def run(F, op, x, y, r, alpha, offset=0):
    """op on device copies; offset > 0 shifts every operand by that many
    elements inside a larger buffer (misaligned for the vector path)."""
    def dev(a):
        buf = torch.zeros(a.size + offset, dtype=F.dtype, device="cuda")
        buf[offset:] = to_dev(a)
        return buf[offset:]
    xd, yd, rd = dev(x), dev(y), dev(r)
    out = rd if op == "axpyin" else None
    got = F.elementwise(op, xd, yd if op in ("add", "sub", "mul", "div", "axpy") else None,
                        alpha=alpha if op in ("axpy", "axpyin") else None, out=out)
    return to_host(got)


def want(p, rep, op, x, y, r, alpha):
    return oracle.elementwise(p, rep, op, x, y if op in ("add", "sub", "mul", "div", "axpy") else None,
                              alpha if op in ("axpy", "axpyin") else None,
                              r if op == "axpyin" else None)


@pytest.mark.parametrize("p,rep", FIELDS, ids=lambda v: str(v))
def test_elementwise_matches_oracle(p, rep):
    F = field(p, rep)
    for n in (0, 1, 5, 15, 17, 4099, 100003):
        x, y, r, alpha = inputs(p, rep, n, 80 + n % 7)
        for op in OPS:
            got = run(F, op, x, y, r, alpha)
            assert same(got, want(p, rep, op, x, y, r, alpha)), (p, rep, op, n)


@pytest.mark.parametrize("p,rep", [(65521, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                                   (32749, "zech"), (251, "centred")])
def test_elementwise_misaligned_and_in_place(p, rep):
    F = field(p, rep)
    n = 10007
    x, y, r, alpha = inputs(p, rep, n, 90)
    for op in OPS:
        got = run(F, op, x, y, r, alpha, offset=1)
        assert same(got, want(p, rep, op, x, y, r, alpha)), (p, rep, op)
    # r = x in place, and r = y
    xd, yd = to_dev(x), to_dev(y)
    F.elementwise("mul", xd, yd, out=xd)
    assert same(to_host(xd), oracle.elementwise(p, rep, "mul", x, y))
    xd = to_dev(x)
    F.elementwise("sub", xd, yd, out=yd)
    assert same(to_host(yd), oracle.elementwise(p, rep, "sub", x, y))


@pytest.mark.parametrize("p,rep", [(32749, "zpz"), (67108859, "fp64"), (32749, "zech")])
def test_elementwise_large(p, rep):
    """A length of 2^24 + 3 (many grid strides, ragged tail)."""
    F = field(p, rep)
    n = (1 << 24) + 3
    x, y, r, alpha = inputs(p, rep, n, 91)
    for op in ("add", "mul", "axpy"):
        got = run(F, op, x, y, r, alpha)
        assert same(got, want(p, rep, op, x, y, r, alpha)), (p, rep, op)


def test_elementwise_argument_errors():
    F = field(65521, "zpz")
    x = torch.zeros(8, dtype=torch.uint32, device="cuda")
    with pytest.raises(ValueError):
        F.elementwise("axpy", x, x)            # no alpha
    with pytest.raises(ValueError):
        F.elementwise("axpyin", x, alpha=1)    # no out
    with pytest.raises(TypeError):
        F.elementwise("add", x, torch.zeros(8, dtype=torch.float64, device="cuda"))
    import ctypes
    L = fd.lib()
    assert L.fdot_elementwise(F.handle, 9, 8, None, ctypes.c_void_p(x.data_ptr()),
                              ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                              None) == -1      # unknown operation
    assert L.fdot_elementwise(F.handle, 0, 8, None, ctypes.c_void_p(x.data_ptr()), None,
                              ctypes.c_void_p(x.data_ptr()), None) == -1  # add without y
    assert ELEM_BYTES["zpz"] == 4 and TORCH_DTYPES["zpz"] == torch.uint32


@pytest.mark.parametrize("p,rep", [(32749, "zpz"), (4294967291, "zpz"), (2654435761, "mont"),
                                   (67108859, "fp64"), (251, "centred"), (3, "centred"),
                                   (2, "zpz")])
def test_division_shares_one_inversion_per_vector(p, rep):
    """The vector path inverts all the divisors of a lane's 16 bytes at once:
    zero divisors at every position of a vector, vectors of zeros only,
    vectors of ones, the largest residues, and a ragged tail."""
    F = field(p, rep)
    n = 4096 + 7
    x = stored(p, rep, n, 95, 0)
    y = stored(p, rep, n, 95, 1)
    canon = oracle.decode(p, rep, y).astype(np.int64)
    per = 16 // ELEM_BYTES[rep]
    for k in range(per):                        # one zero at lane position k
        canon[per * (2 + k) + k] = 0
    canon[per * 40: per * 42] = 0               # whole vectors of zeros
    canon[per * 50: per * 52] = 1 % p           # and of ones
    canon[per * 60: per * 62] = p - 1
    y = oracle.encode(p, rep, canon)
    got = run(F, "div", x, y, x, None)
    assert same(got, want(p, rep, "div", x, y, x, None)), (p, rep)


@pytest.mark.parametrize("p", [251, 241, 3, 5, 127])
def test_centred_products_exhaustive(p):
    """Centred residues (Sec. 3.2.2): every product and every AXPY a x + y
    (with the extreme multipliers +-h) over all pairs (x, y) of residues,
    against the oracle: the signed remainder over its whole domain."""
    F = field(p, "centred")
    h = (p - 1) // 2
    vals = np.arange(-h, h + 1, dtype=np.int8)
    x = np.repeat(vals, vals.size)
    y = np.tile(vals, vals.size)
    for op, alpha in (("mul", None), ("axpy", np.int8(h)), ("axpy", np.int8(-h))):
        got = run(F, op, x, y, y, alpha)
        assert same(got, want(p, "centred", op, x, y, y, alpha)), (p, op, alpha)


@pytest.mark.parametrize("p", [251, 241, 3, 5, 127])
def test_centred_division_exhaustive(p):
    """Centred division reads the inverse of each divisor from a table built
    at field creation: every quotient x / y over all pairs of residues (zero
    divisors give zero), on the vector path and the misaligned one."""
    F = field(p, "centred")
    h = (p - 1) // 2
    vals = np.arange(-h, h + 1, dtype=np.int8)
    x = np.repeat(vals, vals.size)
    y = np.tile(vals, vals.size)
    for offset in (0, 3):
        got = run(F, "div", x, y, x, None, offset=offset)
        assert same(got, want(p, "centred", "div", x, y, x, None)), (p, offset)


@pytest.mark.parametrize("rep", ["zpz", "mont", "fp64"])
def test_powered_division_exhaustive(rep):
    """The Fermat inverse b^(p-2) by sliding windows: every quotient x / y over
    all pairs of residues for small primes whose exponents p - 2 take every
    window shape (1, 11, 101, 1001, 1011, 1111, ... up to 255), on the vector
    path (one exponentiation per lane's batch of divisors) and the
    misaligned one (one exponentiation per element)."""
    for p in (3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 61, 67, 127, 131, 251, 257):
        F = field(p, rep)
        vals = oracle.encode(p, rep, np.arange(p, dtype=np.int64))
        x = np.repeat(vals, p)
        y = np.tile(vals, p)
        for offset in (0, 3):
            got = run(F, "div", x, y, x, None, offset=offset)
            assert same(got, want(p, rep, "div", x, y, x, None)), (p, rep, offset)


@pytest.mark.parametrize("packed", [1, 0])
@pytest.mark.parametrize("p", [3, 5, 7, 11, 257, 4099])
def test_zech_sums_exhaustive(p, packed):
    """Discrete-log sums, differences and AXPY over fields of at most 32768
    elements, on the packed step (two codes per instruction) and on the
    one-code step every larger field uses (tune key zech.packed = 0): every
    pair of codes (0 = the zero element, q - 1 = the unit), sampled pairs for
    q = 4099, with the multipliers 0, 1, -1 and a generic one, aligned and
    misaligned."""
    fd.tune_set("zech.packed", packed)
    try:
        _zech_sums(p)
    finally:
        fd.tune_set("zech.packed", None)


def _zech_sums(p):
    F = field(p, "zech")
    if p <= 257:
        c = np.arange(p, dtype=np.uint16)
        x, y = np.repeat(c, p), np.tile(c, p)
    else:
        x, y = stored(p, "zech", 300007, 96, 0), stored(p, "zech", 300007, 96, 1)
        x[:p], y[:p] = np.arange(p, dtype=np.uint16), np.arange(p, dtype=np.uint16)[::-1]
    r = y.copy()
    half = (p - 1) // 2
    alphas = sorted({0, p - 1, half if half else p - 1, min(p - 1, 2)})
    for offset in (0, 1):
        for op in ("add", "sub"):
            got = run(F, op, x, y, r, None, offset=offset)
            assert same(got, want(p, "zech", op, x, y, r, None)), (p, op, offset)
        for a in alphas:
            alpha = np.uint16(a)
            for op in ("axpy", "axpyin"):
                got = run(F, op, x, y, r, alpha, offset=offset)
                assert same(got, want(p, "zech", op, x, y, r, alpha)), (p, op, a, offset)


@pytest.mark.parametrize("p,rep", [(32749, "zpz"), (4294967291, "zpz"), (2147483647, "mont"),
                                   (67108859, "fp64"), (2, "fp64")], ids=str)
@pytest.mark.parametrize("elems", [8, 16, 32])
def test_division_batched_inversion(p, rep, elems):
    """The aligned division kernel inverts the divisors of 8, 16 or 32 elements
    per lane (whole vectors a workgroup's width apart) with one
    exponentiation: about one divisor in ten zero, lengths that leave a
    partial last workgroup, partial vectors and a ragged tail, in place."""
    F = field(p, rep)
    rng = np.random.default_rng(97)
    fd.tune_set("ew.div_elems", elems)
    try:
        for n in (1, 7, 4096 * 3 + 11, (1 << 20) + 5):
            x = stored(p, rep, n, 98, 0)
            canon = oracle.decode(p, rep, stored(p, rep, n, 98, 1)).astype(np.int64)
            canon[rng.random(n) < 0.1] = 0
            y = oracle.encode(p, rep, canon)
            expect = want(p, rep, "div", x, y, x, None)
            assert same(run(F, "div", x, y, x, None), expect), (p, rep, n)
            xd, yd = to_dev(x), to_dev(y)
            F.elementwise("div", xd, yd, out=xd)
            assert same(to_host(xd), expect), (p, rep, n, "in place")
    finally:
        fd.tune_set("ew.div_elems", None)
