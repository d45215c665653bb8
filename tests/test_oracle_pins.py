"""Pins of the oracle against things other than itself (no GPU needed).

Each test checks the oracle against a value the paper prints, a closed form, an
algebraic invariant, or a brute-force evaluation written independently in
Python's unbounded integers, so that a dropped term, a wrong sign or index, a
swapped operand or a wrong representation map fails at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import bounds
from tests.conftest import GOLDEN

B = 1 << 32
CONFIG_PRIMES = [251, 32749, 65521, 1048573, 67108859, 2147483647, 4294967291]


# ----------------------------------------------------------- python brute force
def _order(g, p):
    k, v = 1, g % p
    while v != 1:
        v = v * g % p
        k += 1
    return k


def _smallest_generator(p):
    for g in range(2, p):
        if _order(g, p) == p - 1:
            return g
    raise AssertionError


def py_decode(p, rep, v, g=None):
    v = int(v)
    if rep == "zpz":
        return v
    if rep == "mont":
        return v * pow(B, -1, p) % p
    if rep == "fp64":
        return int(v)
    if rep == "zech":
        return 0 if v == 0 else pow(g, v, p)
    if rep == "centred":
        return v % p
    raise AssertionError(rep)


def py_encode(p, rep, r, g=None):
    if rep == "zpz":
        return r
    if rep == "mont":
        return (r * B) % p
    if rep == "fp64":
        return float(r)
    if rep == "zech":
        if r == 0:
            return 0
        for i in range(1, p):
            if pow(g, i, p) == r:
                return i
        raise AssertionError
    if rep == "centred":
        return r - p if r > (p - 1) // 2 else r
    raise AssertionError(rep)


def py_dot(p, rep, x, y, g=None):
    s = sum(py_decode(p, rep, a, g) * py_decode(p, rep, b, g) for a, b in zip(x, y))
    return py_encode(p, rep, s % p, g)


def stored_range(p, rep):
    """All stored values that are canonical in rep."""
    if rep in ("zpz", "mont", "fp64"):
        return list(range(p))
    if rep == "zech":
        return list(range(p))  # indices 0..q-1
    if rep == "centred":
        h = (p - 1) // 2
        return list(range(-h, h + 1))
    raise AssertionError


def random_stored(p, rep, n, seed, stream):
    if rep == "centred":
        h = (p - 1) // 2
        return synth.uniform_int(seed, stream, n, 2 * h + 1, lo=-h)
    return synth.uniform_int(seed, stream, n, p)


def reps_for(p):
    out = ["zpz"]
    if p % 2:
        out.append("mont")
    if p < (1 << 26) + (1 << 25):
        out.append("fp64")
    if 2 < p <= 65521:
        out.append("zech")
    if 2 < p < 256:
        out.append("centred")
    return out


# ------------------------------------------------------------------- paper pins
def test_paper_printed_bounds():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        gold = json.load(f)
    assert bounds.axpy_max_prime(32, True) == gold["axpy_signed_max_prime"]["m32"]
    assert bounds.axpy_max_prime(64, True) == gold["axpy_signed_max_prime"]["m64"]
    assert bounds.axpy_max_prime(32, False) == gold["axpy_unsigned_max_prime"]["m32"]
    assert bounds.axpy_max_prime(64, False) == gold["axpy_unsigned_max_prime"]["m64"]
    assert bounds.montgomery_axpy_max_prime(16) == gold["montgomery_axpy_max_prime"]["b16"]
    assert bounds.montgomery_axpy_max_prime(32) == gold["montgomery_axpy_max_prime"]["b32"]
    assert bounds.zech_max_prime(32) == gold["zech_index_max_prime_32bit"]["value"]
    t = gold["zech_table_bytes_2pow26"]
    assert t["entries"] * t["bytes_per_entry"] == t["megabytes"] << 20
    e = gold["eq1_no_reduction_length"]
    lam = bounds.eq1_lambda(e["p"], e["m"])
    assert abs(lam - e["approx"]) / e["approx"] < 0.005
    assert lam == 11524604743
    # The carried residue of the blocked loop does not change this lambda.
    assert bounds.carried_lambda_int(e["p"], e["m"]) == lam
    h = gold["hybrid_threshold_n512"]
    p_ok = bounds.hybrid_max_prime(h["n"], h["m"])
    # The printed threshold 2897 is the first prime that fails the bound.
    assert h["n"] * h["printed"] * (h["printed"] - 1) >= (1 << h["m"])
    assert p_ok < h["printed"] and all(not bounds.is_prime(q) for q in range(p_ok + 1, h["printed"]))
    z = gold["zech_subtraction_correction_q101"]
    assert bounds.zech_subtraction_correction_fraction(z["q"]) == z["fraction"]
    m = gold["zech_mean_ops"]
    assert sum(m["adds"]) == m["adds_total"] and sum(m["tests"]) == m["tests_total"]


def test_bound_sanity_against_definition():
    for p in CONFIG_PRIMES:
        lam = bounds.carried_lambda_int(p, 64)
        assert (p - 1) + lam * (p - 1) ** 2 <= (1 << 64) - 1
        assert (p - 1) + (lam + 1) * (p - 1) ** 2 > (1 << 64) - 1
        if p < (1 << 27):
            lf = bounds.carried_lambda_fp64(p)
            assert (p - 1) + lf * (p - 1) ** 2 <= 1 << 53 < (p - 1) + (lf + 1) * (p - 1) ** 2
    assert bounds.carried_lambda_fp64(67108859) == 2
    assert bounds.carried_lambda_fp64(1048573) == 8192
    assert bounds.centred_lambda(251, 32) == 137438
    assert bounds.montgomery_redc_terms(2147483647) == 2


# ------------------------------------------------------------ number theory
def test_primality_and_inverse():
    small = [n for n in range(2, 2000) if all(n % d for d in range(2, int(n ** 0.5) + 1))]
    assert [n for n in range(2000) if oracle.is_prime(n)] == small
    for p in CONFIG_PRIMES:
        assert oracle.is_prime(p)
        assert not oracle.is_prime(p + 2) or bounds.is_prime(p + 2)
        a = 123456789 % p or 1
        assert a * oracle.inv_mod(a, p) % p == 1


def test_primitive_roots_have_full_order():
    for p in [3, 5, 7, 11, 101, 251, 32749, 65521]:
        g = oracle.primitive_root(p)
        assert g == _smallest_generator(p)
        assert _order(g, p) == p - 1
    assert oracle.primitive_root(32749) == 2
    assert oracle.primitive_root(65521) == 17


# ---------------------------------------------------------- brute force pins
@pytest.mark.parametrize("p", [3, 5, 7])
def test_exhaustive_tiny_fields(p):
    """Every pair of vectors of length <= 3 over GF(p), every representation."""
    for rep in reps_for(p):
        g = _smallest_generator(p) if rep == "zech" else None
        vals = stored_range(p, rep)
        for n in range(0, 4):
            vecs = list(itertools.product(vals, repeat=n))
            xs, ys, want = [], [], []
            for x in vecs:
                for y in vecs:
                    xs.append(np.array(x))
                    ys.append(np.array(y))
                    want.append(py_dot(p, rep, x, y, g))
            got = oracle.dot_many(p, rep, xs, ys)
            assert [float(v) if rep == "fp64" else int(v) for v in got] == want, (p, rep, n)


@pytest.mark.parametrize("p", CONFIG_PRIMES)
def test_random_against_bigint(p):
    for rep in reps_for(p):
        g = oracle.primitive_root(p) if rep == "zech" else None
        for k, n in enumerate([1, 2, 3, 17, 1000, 10007]):
            x = random_stored(p, rep, n, 11, 2 * k)
            y = random_stored(p, rep, n, 11, 2 * k + 1)
            if rep == "zech" and n > 1000:
                continue  # python discrete log search is slow
            want = py_dot(p, rep, x, y, g)
            got = oracle.dot(p, rep, x, y)
            assert (float(got) if rep == "fp64" else int(got)) == want, (p, rep, n)


# ---------------------------------------------------------------- closed forms
def _lengths_around_lambda(p):
    lam = bounds.carried_lambda_int(p, 64)
    out = {1, 2, 3, 63, 64, 65, 1000}
    for L in (lam, bounds.carried_lambda_fp64(p) if p < (1 << 27) else 0):
        for n in (L - 1, L, L + 1, 2 * L + 1):
            if 0 < n <= 300000:
                out.add(n)
    return sorted(out)


@pytest.mark.parametrize("p", CONFIG_PRIMES)
def test_closed_forms(p):
    for rep in reps_for(p):
        if rep == "zech" and p > 70000:
            continue
        for n in _lengths_around_lambda(p):
            i = np.arange(n, dtype=np.uint64)
            # every product is (p-1)^2 = 1 mod p: the tightest block for Eq. 1
            full = oracle.encode(p, rep, np.full(n, p - 1, dtype=np.uint64))
            assert int(oracle.decode(p, rep, [oracle.dot(p, rep, full, full)])[0]) == n % p
            # sum of i, and sum of i^2 (i mod p is congruent to i)
            xi = oracle.encode(p, rep, i % p)
            one = oracle.encode(p, rep, np.ones(n, dtype=np.uint64))
            s1 = oracle.decode(p, rep, [oracle.dot(p, rep, xi, one)])[0]
            s2 = oracle.decode(p, rep, [oracle.dot(p, rep, xi, xi)])[0]
            assert int(s1) == (n * (n - 1) // 2) % p
            assert int(s2) == ((n - 1) * n * (2 * n - 1) // 6) % p


# ----------------------------------------------------------- representations
def test_montgomery_maps():
    for p in [3, 40499, 65521]:
        x = np.arange(p, dtype=np.uint64)
        enc = oracle.encode(p, "mont", x)
        assert [int(v) for v in enc] == [(int(v) << 32) % p for v in x]
        assert np.array_equal(oracle.decode(p, "mont", enc), x)
    p = 2147483647
    # 2^31 = 1 mod p, so B = 2^32 = 2 and B^-1 = 2^30 (worked by hand)
    assert int(oracle.encode(p, "mont", [1])[0]) == 2
    assert int(oracle.decode(p, "mont", [1])[0]) == 1 << 30
    x = synth.uniform_int(5, 0, 5000, p).astype(np.uint64)
    assert np.array_equal(oracle.decode(p, "mont", oracle.encode(p, "mont", x)), x)
    # dot in Montgomery form = (sum X_i Y_i) * B^-1 mod p
    X = synth.uniform_int(5, 1, 3000, p)
    Y = synth.uniform_int(5, 2, 3000, p)
    closed = sum(int(a) * int(b) for a, b in zip(X, Y)) * (1 << 30) % p
    assert int(oracle.dot(p, "mont", X, Y)) == closed


@pytest.mark.parametrize("p", [3, 7, 101, 251, 32749])
def test_zech_maps(p):
    g = oracle.primitive_root(p)
    vals = np.arange(p, dtype=np.uint64)
    idx = oracle.encode(p, "zech", vals)
    assert int(idx[0]) == 0 and int(idx[1]) == p - 1 and int(idx[g]) == 1
    assert sorted(int(v) for v in idx) == list(range(p))  # a bijection
    assert np.array_equal(oracle.decode(p, "zech", idx), vals)
    # decode(i) = g^i by an independent power
    for i in [1, 2, (p - 1) // 2, p - 2, p - 1]:
        assert int(oracle.decode(p, "zech", [i])[0]) == pow(g, i, p)


def test_cross_representation_agreement():
    for p in [251, 32749, 65521, 1048573, 67108859, 2147483647, 4294967291]:
        n = 4099
        xc = synth.uniform_int(7, 0, n, p).astype(np.uint64)
        yc = synth.uniform_int(7, 1, n, p).astype(np.uint64)
        want = int(sum(int(a) * int(b) for a, b in zip(xc, yc)) % p)
        for rep in reps_for(p):
            r = oracle.dot(p, rep, oracle.encode(p, rep, xc), oracle.encode(p, rep, yc))
            assert int(oracle.decode(p, rep, [r])[0]) == want, (p, rep)


# --------------------------------------------------------------------- algebra
@pytest.mark.parametrize("p", [251, 65521, 2147483647])
def test_algebraic_invariants(p):
    for rep in reps_for(p):
        n = 777
        x = random_stored(p, rep, n, 9, 0)
        y = random_stored(p, rep, n, 9, 1)
        z = random_stored(p, rep, n, 9, 2)
        zero = oracle.encode(p, rep, np.zeros(n, dtype=np.uint64))
        dec = lambda v: int(oracle.decode(p, rep, [v])[0])  # noqa: E731
        assert dec(oracle.dot(p, rep, x, zero)) == 0
        assert oracle.dot(p, rep, x, y) == oracle.dot(p, rep, y, x)
        for i in [0, 5, n - 1]:
            e = zero.copy()
            e[i] = oracle.encode(p, rep, [1])[0]
            assert oracle.dot(p, rep, x, e) == x[i]
        # bilinearity: dot(a x + b y, z) = a dot(x,z) + b dot(y,z)
        a, b = 3 % p, (p - 2)
        xc, yc = oracle.decode(p, rep, x), oracle.decode(p, rep, y)
        comb = oracle.encode(p, rep, (xc * a + yc * b) % p if p < (1 << 31) else
                             np.array([(int(u) * a + int(v) * b) % p for u, v in zip(xc, yc)], dtype=np.uint64))
        lhs = dec(oracle.dot(p, rep, comb, z))
        rhs = (a * dec(oracle.dot(p, rep, x, z)) + b * dec(oracle.dot(p, rep, y, z))) % p
        assert lhs == rhs
        # concatenation: dot(x||x', y||y') = dot(x,y) + dot(x',y')
        whole = dec(oracle.dot(p, rep, np.concatenate([x, z]), np.concatenate([y, x])))
        assert whole == (dec(oracle.dot(p, rep, x, y)) + dec(oracle.dot(p, rep, z, x))) % p


def test_noncanonical_inputs_are_rejected():
    with pytest.raises(ValueError):
        oracle.dot(65521, "zpz", [65521], [1])
    with pytest.raises(ValueError):
        oracle.dot(67108859, "fp64", [0.5], [1.0])
    with pytest.raises(ValueError):
        oracle.dot(251, "centred", [126], [1])
    with pytest.raises(ValueError):
        oracle.dot(32749, "zech", [32749], [1])


# ------------------------------------------------------------- matrix forms
def _bigint_matmul(p, A, Bm):
    A = [[int(v) for v in row] for row in A]
    Bm = [[int(v) for v in row] for row in Bm]
    K, N = len(Bm), len(Bm[0])
    return [[sum(r[k] * Bm[k][j] for k in range(K)) % p for j in range(N)] for r in A]


@pytest.mark.parametrize("p,rep", [(251, "centred"), (1048573, "fp64"), (65521, "zpz"),
                                   (2147483647, "mont"), (32749, "zech")])
def test_gemm_special_cases(p, rep):
    M, N, K = 7, 5, 9
    A = random_stored(p, rep, M * K, 4, 0).reshape(M, K)
    Bm = random_stored(p, rep, K * N, 4, 1).reshape(K, N)
    C = oracle.gemm(p, rep, A, Bm)
    Ac, Bc, Cc = (oracle.decode(p, rep, v.ravel()).reshape(v.shape) for v in (A, Bm, C))
    assert (Cc == np.array(_bigint_matmul(p, Ac, Bc), dtype=np.uint64)).all()
    # identity
    I = oracle.encode(p, rep, np.eye(K, dtype=np.uint64).ravel()).reshape(K, K)
    assert np.array_equal(oracle.gemm(p, rep, A, I), A)
    # K = 1: outer product
    col, row = A[:, :1], Bm[:1, :]
    outer = oracle.gemm(p, rep, col, row)
    oc = (oracle.decode(p, rep, col.ravel())[:, None].astype(object) *
          oracle.decode(p, rep, row.ravel())[None, :].astype(object)) % p
    assert (oracle.decode(p, rep, outer.ravel()).reshape(M, N) == oc.astype(np.uint64)).all()
    # N = 1 equals gemv, 1x1xK equals dot, entries equal the full product
    assert np.array_equal(oracle.gemm(p, rep, A, Bm[:, :1]).ravel(), oracle.gemv(p, rep, A, Bm[:, 0]))
    assert oracle.gemm(p, rep, A[:1], Bm[:, 1:2])[0, 0] == oracle.dot(p, rep, A[0], Bm[:, 1])
    rows, cols = np.array([0, 3, 6, 6]), np.array([0, 4, 2, 4])
    assert np.array_equal(oracle.gemm_entries(p, rep, A, Bm, rows, cols), C[rows, cols])
    # Freivalds with random r: A (B r) = C r mod p
    for t in range(4):
        r = synth.uniform_int(40, t, N, p).astype(object)
        Br = (Bc.astype(object) @ r) % p
        assert np.array_equal((Ac.astype(object) @ Br) % p, (Cc.astype(object) @ r) % p)


# ------------------------------------------------ elementwise operations (Sec. 2)
EW_BINARY = ("add", "sub", "mul", "div")


def _py_ew(p, op, a, u, v, r_old):
    """The seven operations on residues, in Python integers; the inverse from
    Python's own modular exponent -1 (division by zero gives zero)."""
    if op == "add":
        return (u + v) % p
    if op == "sub":
        return (u - v) % p
    if op == "neg":
        return (-u) % p
    if op == "mul":
        return u * v % p
    if op == "div":
        return 0 if v == 0 else u * pow(v, -1, p) % p
    if op == "axpy":
        return (a * u + v) % p
    if op == "axpyin":
        return (a * u + r_old) % p
    raise AssertionError(op)


class _Codec:
    """Python encode/decode with a log table (Zech at large p)."""

    def __init__(self, p, rep):
        self.p, self.rep = p, rep
        self.g = oracle.primitive_root(p) if rep == "zech" else None
        if rep == "zech":
            self.log = {}
            v = 1
            for i in range(1, p):
                v = v * self.g % p
                self.log[v] = i

    def dec(self, v):
        return py_decode(self.p, self.rep, v, self.g)

    def enc(self, r):
        if self.rep == "zech":
            return 0 if r == 0 else self.log[r]
        return py_encode(self.p, self.rep, r, self.g)


def _check_ew(p, rep, op, x, y, alpha, r_old):
    c = _Codec(p, rep)
    got = oracle.elementwise(p, rep, op, x, y if op not in ("neg", "axpyin") else None,
                             alpha if op in ("axpy", "axpyin") else None,
                             r_old if op == "axpyin" else None)
    a = c.dec(alpha) if alpha is not None else 0
    for i in range(len(x)):
        want = c.enc(_py_ew(p, op, a, c.dec(x[i]), c.dec(y[i]), c.dec(r_old[i])))
        g = float(got[i]) if rep == "fp64" else int(got[i])
        assert g == want, (p, rep, op, i, x[i], y[i], alpha)


@pytest.mark.parametrize("p", [3, 5, 7, 11])
def test_elementwise_exhaustive_tiny_fields(p):
    """Every operation on every pair of stored values (and every a for the
    AXPY forms) of every representation of GF(p)."""
    for rep in reps_for(p):
        vals = stored_range(p, rep)
        pairs = list(itertools.product(vals, repeat=2))
        x = np.array([u for u, _ in pairs])
        y = np.array([v for _, v in pairs])
        for op in EW_BINARY + ("neg",):
            _check_ew(p, rep, op, x, y, None, y)
        for a in vals:
            _check_ew(p, rep, "axpy", x, y, a, y)
            _check_ew(p, rep, "axpyin", x, y, a, y)


@pytest.mark.parametrize("p", CONFIG_PRIMES)
def test_elementwise_random_against_bigint(p):
    for rep in reps_for(p):
        n = 3000
        x = random_stored(p, rep, n, 12, 0)
        y = random_stored(p, rep, n, 12, 1)
        r = random_stored(p, rep, n, 12, 2)
        alpha = random_stored(p, rep, 1, 12, 3)[0]
        for op in EW_BINARY + ("neg", "axpy", "axpyin"):
            _check_ew(p, rep, op, x, y, alpha, r)


def test_elementwise_invariants():
    """x - x = 0, x + (-x) = 0, (x y) / y = x for y != 0, x (1 / x) = 1,
    axpy with a = 1 is addition and with a = 0 returns y, and every
    representation gives the same residues for the same field elements."""
    p = 32749
    x = synth.uniform_int(13, 0, 5000, p)
    y = synth.uniform_int(13, 1, 5000, p)
    y[:10] = 0
    ew = oracle.elementwise
    assert (ew(p, "zpz", "sub", x, x) == 0).all()
    assert (ew(p, "zpz", "add", x, ew(p, "zpz", "neg", x)) == 0).all()
    q = ew(p, "zpz", "div", ew(p, "zpz", "mul", x, y), y)
    assert (q[y != 0] == x[y != 0]).all() and (q[y == 0] == 0).all()
    ones = np.ones(5000, dtype=np.uint64)
    nz = x != 0
    assert (ew(p, "zpz", "mul", x, ew(p, "zpz", "div", ones, x))[nz] == 1).all()
    assert (ew(p, "zpz", "axpy", x, y, alpha=1) == ew(p, "zpz", "add", x, y)).all()
    assert (ew(p, "zpz", "axpy", x, y, alpha=0) == y).all()
    for op in ("add", "sub", "neg", "mul", "div", "axpy", "axpyin"):
        res = set()
        for rep in ("zpz", "mont", "fp64", "zech"):
            xs, ys = oracle.encode(p, rep, x), oracle.encode(p, rep, y)
            a = oracle.encode(p, rep, [12345])[0]
            out = ew(p, rep, op, xs, ys if op not in ("neg", "axpyin") else None,
                     a if op in ("axpy", "axpyin") else None, ys if op == "axpyin" else None)
            res.add(tuple(oracle.decode(p, rep, out).tolist()))
        assert len(res) == 1, op


# ------------------------------------------------ extension fields (Sec. 2.4.2)
def test_ext_moduli_match_published_primitive_polynomials():
    """The smallest primitive polynomials over GF(2) of degrees 2..8 and 16,
    as tabulated in the coding literature (x^2+x+1, x^3+x+1, x^4+x+1,
    x^5+x^2+1, x^6+x+1, x^7+x+1, x^8+x^4+x^3+x^2+1, x^16+x^5+x^3+x^2+1), and
    x^2+x+2 for GF(9) and GF(25)."""
    want = {(2, 2): 0x7, (2, 3): 0xB, (2, 4): 0x13, (2, 5): 0x25, (2, 6): 0x43, (2, 7): 0x83,
            (2, 8): 0x11D, (2, 16): 0x1002D, (3, 2): 9 + 3 + 2, (5, 2): 25 + 5 + 2}
    for (p, d), f in want.items():
        assert oracle.ext_modulus(p, d) == f, (p, d)


def test_ext_gf4_multiplication_table():
    """GF(4) = GF(2)[X]/(X^2+X+1), values 0, 1, X = 2, X+1 = 3: the
    multiplication table every textbook prints."""
    table = {(2, 2): 3, (2, 3): 1, (3, 3): 2, (3, 2): 1}
    vals = [0, 1, 2, 3]
    for a in vals:
        for b in vals:
            ca, cb = oracle.ext_encode(2, 2, [a, b])
            got = oracle.ext_decode(2, 2, oracle.ext_elementwise(2, 2, "mul", [ca], [cb]))[0]
            want = 0 if 0 in (a, b) else (b if a == 1 else a if b == 1 else table[(a, b)])
            assert got == want, (a, b)
            # addition in characteristic 2 is XOR of the coefficient bits
            s = oracle.ext_decode(2, 2, oracle.ext_elementwise(2, 2, "add", [ca], [cb]))[0]
            assert s == a ^ b


@pytest.mark.parametrize("p,d", [(2, 3), (3, 2), (3, 3), (5, 2), (2, 5), (7, 2)])
def test_ext_field_axioms(p, d):
    """Over every element of small extension fields: codes round-trip, the
    code q-1 is 1 and code 1 is X; every nonzero element times its inverse
    is 1; a(b + c) = ab + ac and (a + b)^p = a^p + b^p (Frobenius) on all
    triples / pairs; x - x = 0 and x + (-x) = 0."""
    q = p ** d
    codes = np.arange(q, dtype=np.uint16)
    vals = oracle.ext_decode(p, d, codes)
    assert sorted(vals.tolist()) == list(range(q))
    assert (oracle.ext_encode(p, d, vals) == codes).all()
    assert vals[q - 1] == 1 and vals[1] == p
    ew = lambda op, x, y=None: oracle.ext_elementwise(p, d, op, x, y)
    one = np.full(q - 1, q - 1, dtype=np.uint16)
    nz = codes[1:]
    assert (ew("mul", nz, ew("div", one, nz)) == q - 1).all()
    assert (ew("sub", codes, codes) == 0).all()
    assert (ew("add", codes, ew("neg", codes)) == 0).all()
    A, B, C = np.meshgrid(codes, codes, codes, indexing="ij") if q <= 27 else \
        (synth.uniform_int(14, k, 4000, q).astype(np.uint16) for k in range(3))
    A, B, C = (np.ascontiguousarray(t.reshape(-1).astype(np.uint16)) for t in (A, B, C))
    assert (ew("mul", A, ew("add", B, C)) == ew("add", ew("mul", A, B), ew("mul", A, C))).all()

    def pw(x, e):
        r = np.full(x.size, q - 1, dtype=np.uint16)
        for _ in range(e):
            r = ew("mul", r, x)
        return r
    assert (pw(ew("add", A, B), p) == ew("add", pw(A, p), pw(B, p))).all()


def test_ext_dot_against_elementwise_and_bruteforce():
    """The dot product equals the sum of elementwise products, and over GF(4)
    it matches a Python sum of the multiplication table, for every pair of
    vectors of length 2."""
    p, d = 3, 4
    q = p ** d
    x = synth.uniform_int(15, 0, 777, q).astype(np.uint16)
    y = synth.uniform_int(15, 1, 777, q).astype(np.uint16)
    prods = oracle.ext_elementwise(p, d, "mul", x, y)
    acc = np.zeros(1, dtype=np.uint16)
    for c in prods:
        acc = oracle.ext_elementwise(p, d, "add", acc, [c])
    assert oracle.ext_dot(p, d, x, y) == acc[0]
    assert oracle.ext_dot(p, d, [], []) == 0
    mul4 = {(2, 2): 3, (2, 3): 1, (3, 3): 2, (3, 2): 1}

    def m(a, b):
        return 0 if 0 in (a, b) else (b if a == 1 else a if b == 1 else mul4[(a, b)])
    for x0, x1, y0, y1 in itertools.product(range(4), repeat=4):
        want = m(x0, y0) ^ m(x1, y1)
        cx = oracle.ext_encode(2, 2, [x0, x1])
        cy = oracle.ext_encode(2, 2, [y0, y1])
        assert oracle.ext_decode(2, 2, [oracle.ext_dot(2, 2, cx, cy)])[0] == want


def test_ext_noncanonical_codes_are_rejected():
    """Codes of GF(q) are 0 .. q-1 (Sec. 2.4): every extension-field entry
    point refuses a code >= q in any operand it reads, and the scalar of
    AXPY/AXPYIN too; a code it does not read is not checked."""
    p, d = 3, 2  # q = 9
    good = np.array([0, 1, 8, 4], dtype=np.uint16)
    bad = np.array([0, 9, 1, 2], dtype=np.uint16)
    with pytest.raises(ValueError):
        oracle.ext_dot(p, d, bad, good)
    with pytest.raises(ValueError):
        oracle.ext_decode(p, d, bad)
    for op in ("add", "sub", "mul", "div", "axpy"):
        with pytest.raises(ValueError):
            oracle.ext_elementwise(p, d, op, good, bad, alpha=1)
        with pytest.raises(ValueError):
            oracle.ext_elementwise(p, d, op, bad, good, alpha=1)
    with pytest.raises(ValueError):
        oracle.ext_elementwise(p, d, "neg", bad)
    with pytest.raises(ValueError):
        oracle.ext_elementwise(p, d, "axpy", good, good, alpha=9)
    with pytest.raises(ValueError):
        oracle.ext_elementwise(p, d, "axpyin", good, alpha=1, r=bad)
    with pytest.raises(ValueError):
        oracle.ext_elementwise(p, d, "axpyin", good, alpha=200, r=good)
    # neg reads no y: a y outside the field is not an operand
    assert oracle.ext_elementwise(p, d, "neg", good, bad).shape == good.shape
