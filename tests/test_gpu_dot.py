"""GPU parity of the dot-product path against the oracle, bit for bit.

Sizes span several chunks and ragged tails; every representation and every
accumulation schedule; edge cases: empty, one element, misaligned and
aliased operands, the maximal-product pattern that fills each block to its
bound, and batches mixing empty, tiny and multi-chunk instances.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import (ELEM_BYTES, NP_DTYPES as NP, TORCH_DTYPES, same, storage_range,
                               stored, to_dev, to_host)

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

P_LAMBDA100 = 429496709   # lambda_u64 = 100: folds inside a chunk
P_FP_LAMBDA3 = 54794149   # lambda_f64 = 3
P_FP_MAX = 94906249       # largest prime with lambda_f64 >= 1

CASES = (
    [(p, "zpz", a) for p in (251, 32749, 65521, P_LAMBDA100, 2147483647, 4294967291)
     for a in ("auto", "delayed", "perterm", "overflow", "hybrid")]
    + [(p, "mont", a) for p in (3, 32749, 65521, 2147483647, 2654435761, 4294967291)
       for a in ("auto", "delayed", "perterm", "overflow", "hybrid")]
    + [(p, "fp64", a) for p in (251, 1048573, 67108859, P_FP_LAMBDA3, P_FP_MAX)
       for a in ("auto", "delayed", "perterm")]
    + [(p, "zech", a) for p in (3, 251, 32749, 65521) for a in ("auto", "zech_exp", "zech_tplus1")]
    + [(p, "centred", a) for p in (3, 251) for a in ("auto", "delayed")]
)


def default_chunk(rep):
    return 65536 // ELEM_BYTES[rep]


def lengths(rep):
    C = default_chunk(rep)
    return [0, 1, 3, 63, 64, 65, 1000, C - 1, C, C + 1, 3 * C + 17]


_fields = {}


def field(p, rep):
    if (p, rep) not in _fields:
        _fields[(p, rep)] = fd.Field(p, rep)
    return _fields[(p, rep)]


@pytest.mark.parametrize("p,rep,algo", CASES, ids=lambda v: str(v))
def test_dot_matches_oracle(p, rep, algo):
    F = field(p, rep)
    for k, n in enumerate(lengths(rep)):
        for pattern in ("random", "maxprod"):
            x = stored(p, rep, n, 100 + k, 0, pattern)
            y = stored(p, rep, n, 100 + k, 1, pattern)
            want = oracle.dot(p, rep, x, y)
            got = to_host(F.dot(to_dev(x), to_dev(y), algo=algo))[0]
            assert same(got, want), (p, rep, algo, n, pattern, got, want)
    # the same pairs as one batch (long chunks: exercises the in-chunk folds)
    for pattern in ("random", "maxprod"):
        xs = [stored(p, rep, n, 100 + k, 0, pattern) for k, n in enumerate(lengths(rep))]
        ys = [stored(p, rep, n, 100 + k, 1, pattern) for k, n in enumerate(lengths(rep))]
        xd, yd = [to_dev(v) for v in xs], [to_dev(v) for v in ys]
        got = to_host(F.dot_many(fd.Field.make_desc(xd, yd), algo=algo))
        assert same(got, oracle.dot_many(p, rep, xs, ys)), (p, rep, algo, pattern)


@pytest.mark.parametrize("range_bytes", [None, 4096])
@pytest.mark.parametrize("p,rep,algo", [c for c in CASES if c[1] != "zech"],
                         ids=lambda v: str(v))
def test_batched_separate_plan(p, rep, algo, range_bytes):
    """The batched form with its plan built by a separate launch, the path
    of every batch above the in-kernel plan limit (tables: always), for
    every policy and schedule: ragged and empty pairs, misaligned views, the
    maximal-product pattern; with the default ranges and with ranges of 4 KiB
    per operand, so that pairs are cut across many ranges."""
    F = field(p, rep)
    keys = {f"many.fused.{rep}": 0, f"many.range.{rep}": range_bytes}
    for k, v in keys.items():
        fd.tune_set(k, v)
    try:
        C = default_chunk(rep)
        ns = [0, 1, 3, 63, 64, 65, 1000, C - 1, C, C + 1, 0, 3 * C + 17, 5, 2 * C + 3, 777]
        for pattern in ("random", "maxprod"):
            xs = [stored(p, rep, n, 150 + k, 0, pattern) for k, n in enumerate(ns)]
            ys = [stored(p, rep, n, 150 + k, 1, pattern) for k, n in enumerate(ns)]
            xd, yd = [to_dev(v) for v in xs], [to_dev(v) for v in ys]
            big = to_dev(stored(p, rep, 9000, 151, 0, pattern))
            xd.append(big[1:4001]); yd.append(big[3:4003])
            xs.append(to_host(big[1:4001])); ys.append(to_host(big[3:4003]))
            desc = fd.Field.make_desc(xd, yd)
            for _ in range(2):
                got = to_host(F.dot_many(desc, algo=algo))
                assert same(got, oracle.dot_many(p, rep, xs, ys)), (p, rep, algo, pattern)
    finally:
        for k in keys:
            fd.tune_set(k, None)


@pytest.mark.parametrize("p,rep", [(32749, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                                   (32749, "zech"), (251, "centred"), (4294967291, "zpz")])
def test_misaligned_and_aliased(p, rep):
    F = field(p, rep)
    n = 3 * default_chunk(rep) + 5
    xb = to_dev(stored(p, rep, n + 8, 7, 0))
    yb = to_dev(stored(p, rep, n + 8, 7, 1))
    xh, yh = to_host(xb), to_host(yb)
    for ox, oy in [(1, 1), (1, 2), (3, 0), (0, 5)]:
        got = to_host(F.dot(xb[ox:ox + n], yb[oy:oy + n]))[0]
        want = oracle.dot(p, rep, xh[ox:ox + n], yh[oy:oy + n])
        assert same(got, want), (ox, oy)
    got = to_host(F.dot(xb[:n], xb[:n]))[0]
    assert same(got, oracle.dot(p, rep, xh[:n], xh[:n]))


@pytest.mark.parametrize("p,rep,algo", [(65521, "zpz", "auto"), (2147483647, "mont", "delayed"),
                                        (4294967291, "zpz", "perterm"),
                                        (4294967291, "zpz", "overflow"),
                                        (2897, "zpz", "hybrid"), (2147483647, "mont", "hybrid"),
                                        (67108859, "fp64", "auto"), (32749, "zech", "zech_exp"),
                                        (32749, "zech", "zech_tplus1"), (251, "centred", "auto")])
def test_batched_matches_oracle_and_single(p, rep, algo):
    F = field(p, rep)
    C = default_chunk(rep)
    ns = [0, 1, 5, 64, 1000, C - 3, C, C + 1, 2 * C + 7, 0, 17, 5 * C + 3, 333, 12345]
    xs = [to_dev(stored(p, rep, n, 31, 2 * k)) for k, n in enumerate(ns)]
    ys = [to_dev(stored(p, rep, n, 31, 2 * k + 1)) for k, n in enumerate(ns)]
    # misaligned views in the middle of the batch
    big = to_dev(stored(p, rep, 9000, 32, 0))
    xs.append(big[1:4001]); ys.append(big[3:4003])
    xs.append(big[2:8002]); ys.append(big[2:8002])
    desc = fd.Field.make_desc(xs, ys)
    got = to_host(F.dot_many(desc, algo=algo))
    want = oracle.dot_many(p, rep, [to_host(x) for x in xs], [to_host(y) for y in ys])
    assert same(got, want)
    single = np.array([to_host(F.dot(x, y, algo=algo))[0] for x, y in zip(xs, ys)])
    assert same(got, single)
    again = to_host(F.dot_many(desc, algo=algo))
    assert same(got, again)


@pytest.mark.parametrize("fused", [None, 0, 7680])
@pytest.mark.parametrize("slices,groups,range_bytes",
                         [(1, None, None), (4, None, None), (2, 7, 64), (4, 3, None),
                          (1, 1, 256), (8, 5000, 1 << 20), (1, 65536, 4096), (4, None, 64),
                          (8, 2, 1 << 30)])
def test_batched_range_shapes(slices, groups, range_bytes, fused):
    """The batched form with few groups (each streams pieces of many pairs)
    and many (each pair split over many ranges), one to eight wavefronts per
    range, and ranges from 64 bytes to the whole batch; with the plan built
    by a separate launch and inside the kernel."""
    p, rep = 65521, "zpz"
    F = field(p, rep)
    keys = {"many.slices.zpz": slices, "many.groups.zpz": groups, "many.range.zpz": range_bytes,
            "many.fused.zpz": fused}
    for k, v in keys.items():
        fd.tune_set(k, v)
    try:
        ns = [int(v) for v in synth.log_uniform_lengths(9, 0, 300, 0.0, 5.0)]
        ns[7] = 0
        ns[100] = 1_000_003
        xs = [to_dev(stored(p, rep, n, 33, 2 * k)) for k, n in enumerate(ns)]
        ys = [to_dev(stored(p, rep, n, 33, 2 * k + 1)) for k, n in enumerate(ns)]
        want = oracle.dot_many(p, rep, [to_host(x) for x in xs], [to_host(y) for y in ys])
        for _ in range(2):
            got = to_host(F.dot_many(fd.Field.make_desc(xs, ys)))
            assert same(got, want)
        # a batch of one pair and a batch smaller than the number of ranges
        got = to_host(F.dot_many(fd.Field.make_desc(xs[100:101], ys[100:101])))
        assert same(got, want[100:101])
        got = to_host(F.dot_many(fd.Field.make_desc(xs[:5], ys[:5])))
        assert same(got, want[:5])
    finally:
        for k in keys:
            fd.tune_set(k, None)


def test_centred_fold_path():
    """A piece long enough that a lane's int32 accumulator must be flushed
    to 64 bits several times, in the single and the batched form."""
    p, rep = 251, "centred"
    F = field(p, rep)
    fd.tune_set("chunk.centred", 1 << 24)
    fd.tune_set("min_chunk.centred", 1 << 24)
    fd.tune_set("many.slices.centred", 1)
    fd.tune_set("many.groups.centred", 1)
    fd.tune_set("many.range.centred", 1 << 30)
    try:
        n = (1 << 24) + 77
        for pattern in ("random", "maxprod"):
            x, y = stored(p, rep, n, 35, 0, pattern), stored(p, rep, n, 35, 1, pattern)
            want = oracle.dot(p, rep, x, y)
            xd, yd = to_dev(x), to_dev(y)
            assert same(to_host(F.dot(xd, yd))[0], want)
            got = to_host(F.dot_many(fd.Field.make_desc([xd, xd[:1000]], [yd, yd[:1000]])))
            assert same(got[0], want)
            assert same(got[1], oracle.dot(p, rep, x[:1000], y[:1000]))
    finally:
        for k in ("chunk.centred", "min_chunk.centred", "many.slices.centred",
                  "many.groups.centred", "many.range.centred"):
            fd.tune_set(k, None)


@pytest.mark.parametrize("p,rep", [(32749, "zpz"), (2147483647, "mont"), (4294967291, "mont"),
                                   (67108859, "fp64"), (32749, "zech"), (65521, "zech"),
                                   (251, "centred")])
def test_encode_decode(p, rep):
    F = field(p, rep)
    n = 100003
    canon = synth.uniform_int(41, 0, n, p).astype(np.uint32)
    canon[:4] = [0, 1, p - 1, min(2, p - 1)]
    enc = F.encode(to_dev(canon))
    assert enc.dtype == TORCH_DTYPES[rep]
    assert same(to_host(enc), oracle.encode(p, rep, canon.astype(np.uint64)))
    dec = F.decode(enc)
    assert same(to_host(dec), canon)


@pytest.mark.parametrize("rep,primes", [("zpz", [32749, 65521, 4294967291, 2]),
                                        ("mont", [2147483647, 65521, 32749]),
                                        ("fp64", [67108859, 1048573])])
def test_batched_over_several_fields(rep, primes):
    """fdot_modp_many_mixed: one batch whose pairs name different primes of
    one representation (uneven lengths, empty pairs), each result bit-exact
    against the oracle over its own field; a pair naming no field keeps the
    value already in its result slot."""
    fields = [fd.Field(p, rep) for p in primes]
    ns = [int(v) for v in synth.log_uniform_lengths(21, 0, 300, 0.0, 5.0)]
    ns[:3] = [0, 1, 64]
    which = synth.uniform_int(21, 1, len(ns), len(primes))
    xs, ys, hx, hy = [], [], [], []
    for k, (n, w) in enumerate(zip(ns, which)):
        p = primes[int(w)]
        m, lo = storage_range(p, rep)
        a = synth.uniform_int(22, 2 * k, int(n), m, lo).astype(NP[rep])
        b = synth.uniform_int(22, 2 * k + 1, int(n), m, lo).astype(NP[rep])
        hx.append(a)
        hy.append(b)
        xs.append(to_dev(a))
        ys.append(to_dev(b))
    field_index = [int(w) for w in which]
    field_index[5] = len(primes)  # names no field
    desc = fd.make_mixed_desc(xs, ys, field_index)
    out = torch.full((len(ns),), 7, dtype=fields[0].dtype, device="cuda")
    got = to_host(fd.dot_many_mixed(fields, desc, out=out))
    for k in range(len(ns)):
        if k == 5:
            assert got[k] == 7
            continue
        p = primes[field_index[k]]
        assert same(got[k], oracle.dot(p, rep, hx[k], hy[k])), (k, p)
    with pytest.raises(fd.FdotError):
        fd.dot_many_mixed([fd.Field(32749, "zpz"), fd.Field(32749, "mont")], desc)


@pytest.mark.parametrize("spread", [1, 2, 7, 32, 64])
def test_single_form_spread_combination(spread):
    """Single form with its units spread over first-level combination words:
    unit counts below, at and above the word count, a ragged last round of
    words, the largest residues (p = 4294967291, maximal products), and three
    calls in a row on each size (every word must be back at zero)."""
    p, rep = 4294967291, "zpz"
    F = field(p, rep)
    keys = ("chunk.zpz", "min_chunk.zpz", "spread.zpz")
    old = {k: fd.tune_get(k) for k in keys}
    try:
        fd.tune_set("chunk.zpz", 64)
        fd.tune_set("min_chunk.zpz", 64)
        fd.tune_set("spread.zpz", spread)
        for k, n in enumerate((1, 64, 65, 64 * 7 + 3, 64 * 64, 64 * 65 + 1, 100003)):
            for pattern in ("random", "maxprod"):
                x = stored(p, rep, n, 140 + k, 0, pattern)
                y = stored(p, rep, n, 140 + k, 1, pattern)
                want = oracle.dot(p, rep, x, y)
                xd, yd = to_dev(x), to_dev(y)
                for _ in range(3):
                    got = to_host(F.dot(xd, yd))[0]
                    assert same(got, want), (spread, n, pattern)
    finally:
        for k, v in old.items():
            fd.tune_set(k, v)


@pytest.mark.parametrize("p", [3, 5, 251, 32749, 65521])
def test_one_code_plus_one_step(p):
    """The plus-one schedule with one code per lane (the form every q above
    32768 takes, and small q with tune key zech.packed = 0): single and
    batched dot products, random and maximal codes, lengths with ragged
    tails; and the matrix-vector product of a field created for the plus-one
    schedule, which stages the same table."""
    fd.tune_set("zech.packed", 0)
    try:
        F = fd.Field(p, "zech", algo="zech_tplus1")
        for k, n in enumerate((1, 7, 4099, 3 * 16384 + 17, 300007)):
            for pattern in ("random", "maxprod"):
                x = stored(p, "zech", n, 120 + k, 0, pattern)
                y = stored(p, "zech", n, 120 + k, 1, pattern)
                got = to_host(F.dot(to_dev(x), to_dev(y)))[0]
                assert same(got, oracle.dot(p, "zech", x, y)), (p, n, pattern)
        xs = [stored(p, "zech", n, 130 + n, 0) for n in (0, 1, 63, 1000, 70001)]
        ys = [stored(p, "zech", n, 130 + n, 1) for n in (0, 1, 63, 1000, 70001)]
        xd, yd = [to_dev(v) for v in xs], [to_dev(v) for v in ys]
        got = to_host(F.dot_many(fd.Field.make_desc(xd, yd)))
        assert same(got, oracle.dot_many(p, "zech", xs, ys)), p
        A = stored(p, "zech", 37 * 1003, 131, 0).reshape(37, 1003)
        v = stored(p, "zech", 1003, 131, 1)
        assert same(to_host(F.gemv(to_dev(A), to_dev(v))), oracle.gemv(p, "zech", A, v)), p
    finally:
        fd.tune_set("zech.packed", None)


@pytest.mark.parametrize("p,rep", [(65521, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                                   (32749, "zech"), (65521, "zech"), (251, "centred")], ids=str)
@pytest.mark.parametrize("fused", [None, 0])
def test_make_desc_keeps_operands(p, rep, fused):
    """A descriptor built from temporary tensors keeps them alive: the batch
    (with empty pairs among short ones, planned inside the batched kernel or
    by a separate launch) still reads its operands after other allocations
    that could have reused their memory."""
    if fused is not None:
        fd.tune_set(f"many.fused.{rep}", fused)
    try:
        _keeps_operands(p, rep)
    finally:
        if fused is not None:
            fd.tune_set(f"many.fused.{rep}", None)


def _keeps_operands(p, rep):
    F = field(p, rep)
    lens = (3, 0, 1, 0, 0, 5, 64, 65)
    xs = [stored(p, rep, n, 150 + k, 0) for k, n in enumerate(lens)]
    ys = [stored(p, rep, n, 150 + k, 1) for k, n in enumerate(lens)]
    desc = fd.Field.make_desc([to_dev(v) for v in xs], [to_dev(v) for v in ys])
    filler = [torch.full((n + 1,), 7, dtype=torch.uint8, device="cuda") for n in lens]
    got = to_host(F.dot_many(desc))
    assert same(got, oracle.dot_many(p, rep, xs, ys))
    del filler
