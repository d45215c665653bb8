"""Host logic of the product library (no GPU): field validation, block
lengths, the fold primitives and the Zech tables, each checked against the
oracle's plain definitions, the paper's printed constants or Python's own
integer arithmetic."""
import json
import os
import random

import numpy as np
import pytest

import oracle
from oracle import bounds
from tests.conftest import GOLDEN

fd = pytest.importorskip("paper_cs_0404008_amd")

CONFIG_PRIMES = [251, 32749, 65521, 1048573, 67108859, 2147483647, 4294967291]


def test_printed_prime_bounds():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        g = json.load(f)
    assert fd.max_prime("axpy_signed", 32) == g["axpy_signed_max_prime"]["m32"]
    assert fd.max_prime("axpy_signed", 64) == g["axpy_signed_max_prime"]["m64"]
    assert fd.max_prime("axpy_unsigned", 32) == g["axpy_unsigned_max_prime"]["m32"]
    assert fd.max_prime("axpy_unsigned", 64) == g["axpy_unsigned_max_prime"]["m64"]
    assert fd.max_prime("montgomery", 16) == g["montgomery_axpy_max_prime"]["b16"]
    assert fd.max_prime("montgomery", 32) == g["montgomery_axpy_max_prime"]["b32"]
    assert fd.max_prime("zech_index", 32) == g["zech_index_max_prime_32bit"]["value"]
    e = g["eq1_no_reduction_length"]
    assert fd.lambda_for(e["p"], "u64") == bounds.carried_lambda_int(e["p"], e["m"])


@pytest.mark.parametrize("p", CONFIG_PRIMES + [3, 5, 40009, 94906249])
def test_lambdas_match_oracle_definitions(p):
    assert fd.lambda_for(p, "u64") == bounds.carried_lambda_int(p, 64)
    assert fd.lambda_for(p, "u32") == max(0, bounds.carried_lambda_int(p, 32))
    assert fd.lambda_for(p, "f64") == max(0, bounds.carried_lambda_fp64(p))
    assert fd.lambda_for(p, "i32_centred") == bounds.centred_lambda(p, 32)
    assert fd.lambda_for(p, "mont_redc") == bounds.montgomery_redc_terms(p)
    assert fd.lambda_for(p, "u64_hybrid") == bounds.hybrid_lambda(p, 64)


def test_field_validation():
    assert fd.field_params_status(32749, "zpz") == 0
    assert fd.field_params_status(32751, "zpz") == -2           # 32751 = 3 * 10917
    assert fd.field_params_status(1, "zpz") == -2
    assert fd.field_params_status(4294967311, "zpz") == -3      # a prime above 2^32
    assert fd.field_params_status(2, "mont") == -3              # gcd(p, 2^32) != 1
    assert fd.field_params_status(94906249, "fp64") == 0 or fd.lambda_for(94906249, "f64") == 0
    big = 2147483647
    assert fd.field_params_status(big, "fp64") == -3            # (p-1)^2 > 2^53
    assert fd.field_params_status(65521, "zech") == 0
    assert fd.field_params_status(65537, "zech") == -3          # codes above 16 bits
    assert fd.field_params_status(251, "centred") == 0
    assert fd.field_params_status(257, "centred") == -3
    for p in [2, 3, 5, 7, 11, 13, 65521, 2147483647, 4294967291, 3037000493 % (1 << 32)]:
        assert (fd.field_params_status(p, "zpz") == 0) == oracle.is_prime(p) or p >= 1 << 32


@pytest.mark.parametrize("p", CONFIG_PRIMES + [2, 3, 65537, 40009])
def test_field_constants(p):
    info = fd.field_params(p, "zpz")
    assert info["corr"] == (1 << 64) % p
    assert info["b_mod_p"] == ((1 << 32) % p if p % 2 else 0)
    if p % 2:
        assert (info["n_im"] * p) % (1 << 32) == (1 << 32) - 1       # n_im = -p^-1 mod B
        assert info["binv_mod_p"] * (1 << 32) % p == 1 % p
    assert info["inv_p"] == 1.0 / p
    d = p << info["norm_shift"]
    assert (1 << 31) <= d < (1 << 32)
    assert info["recip"] == ((1 << 64) - 1) // d - (1 << 32)


@pytest.mark.parametrize("p", CONFIG_PRIMES + [2, 3, 5, 40009, 94906249, 2654435761])
def test_fold_primitives(p):
    rnd = random.Random(p)
    cases = [0, 1, p - 1, p, p + 1, (1 << 64) - 1, 1 << 63, p * (p - 1), (p - 1) ** 2 + p - 1,
             (1 << 32) - 1, 1 << 32]
    cases += [rnd.getrandbits(64) for _ in range(3000)]
    cases += [rnd.randrange(p * (1 << 32)) for _ in range(1000)]
    for T in cases:
        T &= (1 << 64) - 1
        assert fd.host_fold(p, "zpz", "remainder", T) == T % p
    if p % 2:
        binv = pow(1 << 32, -1, p)
        for T in [0, 1, p * (1 << 32) - 1] + [rnd.randrange(p * (1 << 32)) for _ in range(3000)]:
            assert fd.host_fold(p, "zpz", "redc", T) == T * binv % p
        with pytest.raises(fd.FdotError):
            fd.host_fold(p, "zpz", "redc", p * (1 << 32))
    if fd.lambda_for(p, "f64") >= 1:
        for T in [0, 1, p - 1, p, 1 << 53, (1 << 53) - 1] + \
                 [rnd.randrange((1 << 53) + 1) for _ in range(3000)]:
            assert fd.host_fold(p, "zpz", "fp64", T) == T % p


@pytest.mark.parametrize("p", [3, 5, 7, 101, 251, 32749, 65521])
def test_zech_tables_match_definitions(p):
    val, idx, plus1 = fd.zech_tables(p)
    g = oracle.primitive_root(p)
    assert fd.field_params(p, "zech")["g"] == g
    # value table: the oracle's decoding; index table: the oracle's encoding
    codes = np.arange(p, dtype=np.uint16)
    assert np.array_equal(val.astype(np.uint64), oracle.decode(p, "zech", codes))
    assert np.array_equal(idx, oracle.encode(p, "zech", np.arange(p, dtype=np.uint64)))
    # plus-one table: g^plus1[k] = 1 + g^k (code 0 when 1 + g^k = 0)
    pv = [int(v) for v in val]
    for k in range(1, p):
        s = (pow(g, k, p) + 1) % p
        h = int(plus1[k])
        assert (h == 0 and s == 0) or (h != 0 and pow(g, h, p) == s)
    assert int(plus1[(p - 1) // 2]) == 0          # g^((q-1)/2) = -1
    assert int(plus1[0]) == p - 1 and pv[p - 1] == 1


def test_status_strings():
    for code in range(-8, 1):
        assert fd.status_string(code)
    assert fd.status_string(-2) == "modulus is not prime"


def test_tune_table_roundtrip():
    assert fd.tune_get("no.such.key") is None
    fd.tune_set("test.key", 1234)
    assert fd.tune_get("test.key") == 1234


def _balanced_digits(c, ndig):
    """Balanced base-256 digits in [-128, 127], lowest first, and what is
    left after ndig of them (zero when ndig digits represent c)."""
    out = []
    for _ in range(ndig):
        t = c & 255
        if t >= 128:
            t -= 256
        out.append(t)
        c = (c - t) // 256
    return out, c


@pytest.mark.parametrize("ndig", [1, 2, 3, 4])
def test_balanced_digit_ranges(ndig):
    """The digit-product matrix path writes a centred residue |c| <= h with
    ndig balanced base-256 digits when h <= 127 (256^ndig - 1) / 255 (127,
    32639, 8355711, 2139062143): every such c is represented exactly, the
    next value up is not, and the digit range keeps each product within
    2^14 so that 131071 of them fit in int32."""
    top = 127 * (256 ** ndig - 1) // 255
    assert top == [127, 32639, 8355711, 2139062143][ndig - 1]
    rng = random.Random(ndig)
    for c in [0, 1, -1, top, -top, -top - 1] + [rng.randint(-top, top) for _ in range(2000)]:
        d, rest = _balanced_digits(c, ndig)
        assert rest == 0 and all(-128 <= x <= 127 for x in d)
        assert sum(x * 256 ** i for i, x in enumerate(d)) == c
    assert _balanced_digits(top + 1, ndig)[1] != 0
    assert 131071 * 128 * 128 <= 2 ** 31 - 1
    # the primes of the workloads and the digits they take
    for p, want in [(251, 1), (32749, 2), (65521, 3), (1048573, 3), (67108859, 4),
                    (2147483647, 4), (4278124237, 4)]:
        h = (p - 1) // 2
        assert min(k for k in (1, 2, 3, 4) if h <= 127 * (256 ** k - 1) // 255) == want


def test_choose_rep_model_and_tuned_override():
    """Representation choice: the fewest bytes per element among the
    representations that admit p, unless the tuning table holds a measured
    choice for p's bit length (and n's decade) that admits p."""
    want = {3: "centred", 251: "centred", 257: "zech", 32749: "zech", 65521: "zech",
            65537: "zpz", 67108859: "zpz", 2147483647: "zpz", 4294967291: "zpz"}
    for p, rep in want.items():
        assert fd.choose_rep(p) == rep, p
        assert fd.field_params_status(p, rep) == 0
    with pytest.raises(fd.FdotError):
        fd.choose_rep(65535)                     # not prime
    with pytest.raises(fd.FdotError):
        fd.choose_rep(2 ** 61 - 1)               # no representation admits it
    try:
        fd.tune_set("auto.rep.b8", fd.REPS["fp64"])
        fd.tune_set("auto.rep.b8.n6", fd.REPS["mont"])
        fd.tune_set("auto.rep.b17", fd.REPS["centred"])  # does not admit 65537
        assert fd.choose_rep(251) == "fp64"
        assert fd.choose_rep(251, 10 ** 6) == "mont"
        assert fd.choose_rep(251, 9 * 10 ** 6) == "mont"
        assert fd.choose_rep(251, 10 ** 7) == "fp64"
        assert fd.choose_rep(65537) == "zpz"
    finally:
        for k in ("auto.rep.b8", "auto.rep.b8.n6", "auto.rep.b17"):
            fd.tune_set(k, None)
    assert fd.choose_rep(251) == "centred"


def test_table_bytes_per_representation():
    """Device bytes of a field's tables: discrete logs hold the value, index
    and plus-one tables (2 bytes per code each, Sec. 2.4) and, for q <= 32768,
    the packed step's plus-one table (padded to 16 bytes); centred residues
    hold 256 inverses; the other representations none."""
    assert fd.field_params(65521, "zech")["table_bytes"] == 3 * 2 * 65521
    assert fd.field_params(32749, "zech")["table_bytes"] == 3 * 2 * 32749 + 2 * 32752
    assert fd.field_params(3, "zech")["table_bytes"] == 3 * 2 * 3 + 16
    assert fd.field_params(251, "centred")["table_bytes"] == 256
    for p, rep in ((65521, "zpz"), (2147483647, "mont"), (67108859, "fp64")):
        assert fd.field_params(p, rep)["table_bytes"] == 0
