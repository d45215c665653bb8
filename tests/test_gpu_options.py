"""Field creation options on the GPU.

validate: inputs outside their representation's canonical range (Sec. 2.1:
a residue is an integer in [0, p); a double must be integral in [0, p); a
discrete-log code below q; a centred residue within (p-1)/2) are reported as
FDOT_E_NONCANON by every compute form before anything is computed, canonical
inputs give the oracle's result; fdot_validate counts them.  algo: the
schedule used for "auto".  block: a delay block shorter than lambda still
gives the exact result (it only folds more often)."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import TORCH_DTYPES, same, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

NONCANON = -9
REPS = [(65521, "zpz"), (2147483647, "mont"), (67108859, "fp64"), (32749, "zech"),
        (251, "centred")]


def bad_values(p, rep):
    """Stored values just outside each representation's canonical range."""
    if rep in ("zpz", "mont"):
        return [p, 0xFFFFFFFF]
    if rep == "fp64":
        return [float(p), 0.5, -1.0, float("nan"), float("inf")]
    if rep == "zech":
        return [p, 65535]
    return [(p - 1) // 2 + 1, -((p - 1) // 2) - 1]


def with_bad(a, v, pos):
    b = a.copy()
    b[pos] = v
    return b


@pytest.mark.parametrize("p,rep", REPS, ids=str)
def test_validate_every_form(p, rep):
    F = fd.Field(p, rep, validate=True)
    n = 5000
    x, y = stored(p, rep, n, 31, 0), stored(p, rep, n, 31, 1)
    got = to_host(F.dot(to_dev(x), to_dev(y)))
    assert same(got, np.asarray(oracle.dot(p, rep, x, y)).reshape(1))
    for v in bad_values(p, rep):
        for pos in (0, n - 1):
            with pytest.raises(fd.FdotError) as e:
                F.dot(to_dev(with_bad(x, v, pos)), to_dev(y))
            assert e.value.status == NONCANON
    # batched: a bad element in the last pair only
    xs = [to_dev(x[:100]), to_dev(x[:n]), to_dev(with_bad(x[:7], bad_values(p, rep)[0], 6))]
    ys = [to_dev(y[:100]), to_dev(y[:n]), to_dev(y[:7])]
    with pytest.raises(fd.FdotError) as e:
        F.dot_many(fd.Field.make_desc(xs, ys))
    assert e.value.status == NONCANON
    good = F.dot_many(fd.Field.make_desc(xs[:2], ys[:2]))
    assert same(to_host(good), oracle.dot_many(p, rep, [x[:100], x], [y[:100], y]))
    # the allocation-free batched form checks as well
    out = torch.empty(3, dtype=TORCH_DTYPES[rep], device="cuda")
    with pytest.raises(fd.FdotError) as e:
        F.dot_many_noalloc(fd.Field.make_desc(xs, ys), out)
    assert e.value.status == NONCANON
    # matrix-vector product: a bad entry of A
    A = stored(p, rep, 64 * 80, 32, 0).reshape(64, 80)
    xv = stored(p, rep, 80, 32, 1)
    assert same(to_host(F.gemv(to_dev(A), to_dev(xv))), oracle.gemv(p, rep, A, xv))
    Ab = A.copy()
    Ab[63, 79] = bad_values(p, rep)[0]
    with pytest.raises(fd.FdotError) as e:
        F.gemv(to_dev(Ab), to_dev(xv))
    assert e.value.status == NONCANON
    # matrix product: a bad entry of B
    B = stored(p, rep, 80 * 48, 33, 0).reshape(80, 48)
    Bb = B.copy()
    Bb[40, 0] = bad_values(p, rep)[-1]
    with pytest.raises(fd.FdotError) as e:
        F.gemm(to_dev(A), to_dev(Bb))
    assert e.value.status == NONCANON
    # elementwise: a bad y, and a bad scalar
    with pytest.raises(fd.FdotError) as e:
        F.elementwise("add", to_dev(x), to_dev(with_bad(y, bad_values(p, rep)[0], 17)))
    assert e.value.status == NONCANON
    with pytest.raises(fd.FdotError) as e:
        F.elementwise("axpy", to_dev(x), to_dev(y), alpha=bad_values(p, rep)[0])
    assert e.value.status == NONCANON
    r = F.elementwise("add", to_dev(x), to_dev(y))
    assert same(to_host(r), oracle.elementwise(p, rep, "add", x, y))


@pytest.mark.parametrize("p,rep", REPS, ids=str)
def test_validate_counts(p, rep):
    F = fd.Field(p, rep)
    n = 100003
    x = stored(p, rep, n, 34, 0)
    rng = np.random.default_rng(35)
    pos = np.unique(rng.integers(0, n, 777))
    bads = bad_values(p, rep)
    for i, k in enumerate(pos):
        x[k] = bads[i % len(bads)]
    cnt = F.validate(to_dev(x))
    assert int(cnt.item()) == len(pos)
    cnt = F.validate(to_dev(stored(p, rep, n, 36, 0)), cnt)  # adds nothing
    assert int(cnt.item()) == len(pos)


@pytest.mark.parametrize("p,rep,algo", [(65521, "zpz", "overflow"), (65521, "zpz", "perterm"),
                                        (2147483647, "mont", "hybrid"),
                                        (32749, "zech", "zech_tplus1"),
                                        (67108859, "fp64", "perterm")], ids=str)
def test_algo_option_sets_auto(p, rep, algo):
    F = fd.Field(p, rep, algo=algo)
    G = fd.Field(p, rep)
    n = 3 * 16384 + 17
    x, y = stored(p, rep, n, 37, 0), stored(p, rep, n, 37, 1)
    a = to_host(F.dot(to_dev(x), to_dev(y)))
    b = to_host(G.dot(to_dev(x), to_dev(y), algo=algo))
    assert same(a, b)
    assert same(a, np.asarray(oracle.dot(p, rep, x, y)).reshape(1))


@pytest.mark.parametrize("p,rep,block", [(65521, "zpz", 2), (65521, "zpz", 9), (32749, "zpz", 1),
                                         (2147483647, "mont", 2), (67108859, "fp64", 1),
                                         (1048573, "fp64", 3), (32749, "zech", 4),
                                         (251, "centred", 16), (251, "centred", 100)], ids=str)
def test_block_option_exact(p, rep, block):
    F = fd.Field(p, rep, block=block)
    for n, pattern in ((1, "random"), (1000, "maxprod"), (3 * 16384 + 17, "random"),
                       (3 * 16384 + 17, "maxprod")):
        x, y = stored(p, rep, n, 38, 0, pattern), stored(p, rep, n, 38, 1, pattern)
        want = np.asarray(oracle.dot(p, rep, x, y)).reshape(1)
        assert same(to_host(F.dot(to_dev(x), to_dev(y))), want), (n, pattern)
        xs, ys = [to_dev(x), to_dev(x[: n // 2])], [to_dev(y), to_dev(y[: n // 2])]
        many = to_host(F.dot_many(fd.Field.make_desc(xs, ys)))
        assert same(many, oracle.dot_many(p, rep, [x, x[: n // 2]], [y, y[: n // 2]]))
    m = 37
    A = stored(p, rep, m * 1000, 39, 0, "maxprod").reshape(m, 1000)
    v = stored(p, rep, 1000, 39, 1, "maxprod")
    assert same(to_host(F.gemv(to_dev(A), to_dev(v))), oracle.gemv(p, rep, A, v))
