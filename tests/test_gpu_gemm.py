"""GPU parity of the matrix forms (fgemv_modp, fgemm_modp) against the oracle.

Covers every kernel path: FP64 matrix cores with residues as stored and
centred, classical and Montgomery residues converted on load, int8 matrix
cores on centred residues, and the exact vector-ALU kernel; ragged shapes,
K beyond the fold bound (so the in-loop folds run), unaligned leading
dimensions, and the full 8192 x 8192 x 4096 products on sampled entries.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import same, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")

FIELDS = [
    (1048573, "fp64"),       # FP64 MFMA, residues as stored
    (67108859, "fp64"),      # FP64 MFMA, centred, fold every 8 products
    (65521, "zpz"),          # FP64 MFMA from uint32 residues
    (32749, "mont"),         # FP64 MFMA on Montgomery residues, one REDC at the end
    (251, "centred"),        # int8 MFMA
    (2147483647, "zpz"),     # int8 MFMA on four balanced base-256 digits
    (4278124237, "zpz"),     # largest prime the digit split covers
    (4294967291, "mont"),    # vector-ALU kernel
    (32749, "zech"),         # vector-ALU kernel
]
SHAPES = [(1, 1, 1), (7, 5, 9), (130, 129, 33), (257, 300, 100), (128, 128, 64), (64, 48, 1000),
          (3, 200, 17)]

_fields = {}


def field(p, rep):
    if (p, rep) not in _fields:
        _fields[(p, rep)] = fd.Field(p, rep)
    return _fields[(p, rep)]


def mat(p, rep, rows, cols, seed, stream, pattern="random"):
    return stored(p, rep, rows * cols, seed, stream, pattern).reshape(rows, cols)


@pytest.mark.parametrize("p,rep", FIELDS, ids=lambda v: str(v))
def test_gemm_matches_oracle(p, rep):
    F = field(p, rep)
    for t, (M, N, K) in enumerate(SHAPES):
        for pattern in ("random", "maxprod"):
            A = mat(p, rep, M, K, 50 + t, 0, pattern)
            B = mat(p, rep, K, N, 50 + t, 1, pattern)
            got = to_host(F.gemm(to_dev(A), to_dev(B)))
            assert same(got, oracle.gemm(p, rep, A, B)), (p, rep, M, N, K, pattern)


@pytest.mark.parametrize("p,rep,K", [(1048573, "fp64", 3 * 8192 + 5), (67108859, "fp64", 301),
                                     (65521, "zpz", 5000), (251, "centred", (1 << 18) + 3)])
def test_gemm_folds_beyond_lambda(p, rep, K):
    F = field(p, rep)
    M, N = 40, 36
    for pattern in ("random", "maxprod"):
        A = mat(p, rep, M, K, 60, 0, pattern)
        B = mat(p, rep, K, N, 60, 1, pattern)
        got = to_host(F.gemm(to_dev(A), to_dev(B)))
        assert same(got, oracle.gemm(p, rep, A, B)), (p, rep, K, pattern)


@pytest.mark.parametrize("p,rep", [(251, "centred"), (1048573, "fp64"), (2147483647, "zpz")])
def test_gemm_strided_operands(p, rep):
    """Leading dimensions larger than the row length, not multiples of 16."""
    F = field(p, rep)
    M, N, K = 70, 45, 83
    Aw = to_dev(mat(p, rep, M, K + 3, 61, 0))
    Bw = to_dev(mat(p, rep, K, N + 5, 61, 1))
    A, B = Aw[:, 1:K + 1], Bw[:, 2:N + 2]
    C = torch.zeros((M, N + 7), dtype=F.dtype, device="cuda")
    F.gemm(A, B, out=C[:, :N])
    want = oracle.gemm(p, rep, to_host(A).copy(), to_host(B).copy())
    assert same(to_host(C[:, :N]).copy(), want)
    assert not to_host(C[:, N:]).any()  # nothing written past the output view


@pytest.mark.parametrize("p,rep", FIELDS, ids=lambda v: str(v))
def test_gemv_matches_oracle(p, rep):
    F = field(p, rep)
    for t, (m, n) in enumerate([(1, 1), (5, 3), (33, 1000), (257, 2049), (1000, 4099)]):
        for pattern in ("random", "maxprod"):
            A = mat(p, rep, m, n, 70 + t, 0, pattern)
            x = stored(p, rep, n, 70 + t, 1, pattern)
            got = to_host(F.gemv(to_dev(A), to_dev(x)))
            assert same(got, oracle.gemv(p, rep, A, x)), (p, rep, m, n, pattern)


GEMV_BALANCED = [(65521, "zpz"), (4294967291, "zpz"), (2147483647, "mont"), (67108859, "fp64"),
                 (32749, "zech"), (251, "centred")]


@pytest.mark.parametrize("p,rep", GEMV_BALANCED, ids=lambda v: str(v))
def test_gemv_row_blocks_match_oracle(p, rep):
    """Rows go four to a wavefront, grouped by their 16-byte phase: rows that
    are a whole number of 16-byte units and in phase with x (x read
    directly), rows out of phase with x (one shifted copy of x), and
    contiguous rows of ragged length whose phases cycle (a copy of x per
    phase class); row counts that are not a multiple of four or of the
    cycle, maximal products; the one-wavefront-per-row kernel on the same
    operands."""
    F = field(p, rep)
    eb = {"zpz": 4, "mont": 4, "fp64": 8, "zech": 2, "centred": 1}[rep]
    w16 = 16 // eb                    # elements per 16 bytes
    cases = [  # m, n, lda, offset of A's first row, offset of x
        (4201, 4099, (4099 + w16 - 1) // w16 * w16 + w16, 0, 0),
        (2103, 8193, (8194 + w16 - 1) // w16 * w16 + w16, 1, 1),
        (9, 300, (301 + w16 - 1) // w16 * w16, 1, 1),
        (64, 1000, 1000 + w16, 0, 1),
        (1003, 4099, 4099, 0, 0),
        (777, 2051, 2051, 0, 1),
        (5, 257, 257, 1, 0),
    ]
    for t, (m, n, lda, oa, ox) in enumerate(cases):
        pattern = "maxprod" if t % 2 == 0 else "random"
        flat = stored(p, rep, m * lda + oa, 75 + t, 0, pattern)
        xw = stored(p, rep, n + ox, 75 + t, 1, pattern)
        A = np.lib.stride_tricks.as_strided(flat[oa:], shape=(m, n),
                                            strides=(lda * flat.itemsize, flat.itemsize))
        want = oracle.gemv(p, rep, np.ascontiguousarray(A), xw[ox:])
        Ad = torch.as_strided(to_dev(flat)[oa:], (m, n), (lda, 1))
        xd = to_dev(xw)[ox:]
        for rows in (4, 1):
            fd.tune_set("gemv.rows", rows)
            try:
                for _ in range(2):
                    got = to_host(F.gemv(Ad, xd))
                    assert same(got, want), (p, rep, m, n, lda, oa, ox, rows)
            finally:
                fd.tune_set("gemv.rows", None)


def test_gemm_special_cases():
    p, rep = 1048573, "fp64"
    F = field(p, rep)
    A = mat(p, rep, 50, 40, 80, 0)
    eye = np.eye(40, dtype=np.float64)
    assert same(to_host(F.gemm(to_dev(A), to_dev(eye))), A)
    # K = 0: C is the zero matrix
    Z = to_host(F.gemm(torch.empty((5, 0), dtype=torch.float64, device="cuda"),
                       torch.empty((0, 6), dtype=torch.float64, device="cuda")))
    assert not Z.any()


def _matvec_mod(X, v, p):
    """X v mod p, exact in int64 for |X| < 2^27 and K <= 8192: v is split
    into 13-bit halves so that no partial sum passes 2^53."""
    lo = (X @ (v & 8191)) % p
    hi = (X @ (v >> 13)) % p
    return (lo + hi * 8192) % p


@pytest.mark.parametrize("p,rep,dtype,path", [(251, "centred", torch.int8, "int8"),
                                              (1048573, "fp64", torch.float64, "fp64"),
                                              (1048573, "fp64", torch.float64, "digits"),
                                              (67108859, "fp64", torch.float64, "digits")])
def test_gemm_full_size_sampled(p, rep, dtype, path):
    """The 8192 x 8192 times 8192 x 4096 product, checked on 4096 entries
    and by Freivalds' test, on the FP64 matrix cores and on the int8 digit
    products (the default at this size for both primes)."""
    fd.tune_set("gemm.split.disable", 1 if path == "fp64" else None)
    try:
        _full_size_case(p, rep, dtype)
    finally:
        fd.tune_set("gemm.split.disable", None)


def _full_size_case(p, rep, dtype):
    M, K, N = 8192, 8192, 4096
    F = field(p, rep)
    m, lo = (p, 0) if rep != "centred" else (p, -((p - 1) // 2))
    A = torch.empty((M, K), dtype=dtype, device="cuda")
    B = torch.empty((K, N), dtype=dtype, device="cuda")
    synth.fill_device(A, 4, 0, m, lo)
    synth.fill_device(B, 4, 1, m, lo)
    C = to_host(F.gemm(A, B))
    del A, B
    torch.cuda.empty_cache()
    Ah = synth.uniform_int(4, 0, M * K, m, lo).reshape(M, K)
    Bh = synth.uniform_int(4, 1, K * N, m, lo).reshape(K, N)
    Ah = Ah.astype(np.int8 if rep == "centred" else np.float64)
    Bh = Bh.astype(np.int8 if rep == "centred" else np.float64)
    rows = synth.uniform_int(4, 2, 4096, M)
    cols = synth.uniform_int(4, 3, 4096, N)
    rows[:4] = [0, 0, M - 1, M - 1]
    cols[:4] = [0, N - 1, 0, N - 1]
    want = oracle.gemm_entries(p, rep, Ah, Bh, rows, cols)
    assert same(C[rows, cols], want)
    # Freivalds: A (B r) = C r mod p for random r; a wrong C passes one trial
    # with probability at most 1/p.
    Ai, Bi, Ci = (v.astype(np.int64) for v in (Ah, Bh, C))
    for t in range(8):
        r = synth.uniform_int(4, 10 + t, N, p).astype(np.int64)
        lhs = _matvec_mod(Ai, _matvec_mod(Bi, r, p), p)
        rhs = _matvec_mod(Ci, r, p)
        assert np.array_equal(lhs, rhs), t


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_gemm_int8_tile_variants(shape):
    """Every int8 matrix-core tiling (register-staged, double-buffered and
    direct-to-LDS), on ragged M and N and a K that some of them take in one
    fold block, against the oracle."""
    p, rep = 251, "centred"
    F = field(p, rep)
    fd.tune_set("gemm.i8.tile", shape)
    try:
        for (M, N, K) in [(1100, 1030, 1024), (1024, 1280, 2048 + 64), (1100, 1030, 1000),
                          (300, 257, 1001)]:
            A = mat(p, rep, M, K, 70, 0, "random")
            B = mat(p, rep, K, N, 70, 1, "random")
            got = to_host(F.gemm(to_dev(A), to_dev(B)))
            rows = synth.uniform_int(71, 0, 512, M)
            cols = synth.uniform_int(71, 1, 512, N)
            rows[:2] = [0, M - 1]
            cols[:2] = [0, N - 1]
            want = oracle.gemm_entries(p, rep, A, B, rows, cols)
            assert same(got[rows, cols], want), (shape, M, N, K)
    finally:
        fd.tune_set("gemm.i8.tile", None)


@pytest.mark.parametrize("shape", [1, 2])
def test_gemm_int8_double_buffered_ktile64(shape):
    """The register-staged int8 tilings with K-tiles of 64, where two LDS
    buffers fit (the next K-tile written halfway through the current one's
    products): ragged shapes, K not a multiple of the tile, and K beyond one
    fold block with maximal products, against the oracle."""
    p, rep = 251, "centred"
    F = field(p, rep)
    fd.tune_set("gemm.i8.tile", shape)
    fd.tune_set("gemm.i8.ktile", 64)
    try:
        for (M, N, K) in [(1100, 1030, 1024), (300, 257, 1001), (64, 64, 64), (70, 33, 65)]:
            A = mat(p, rep, M, K, 72, 0, "random")
            B = mat(p, rep, K, N, 72, 1, "random")
            got = to_host(F.gemm(to_dev(A), to_dev(B)))
            rows = synth.uniform_int(73, 0, 512, M)
            cols = synth.uniform_int(73, 1, 512, N)
            rows[:2] = [0, M - 1]
            cols[:2] = [0, N - 1]
            assert same(got[rows, cols], oracle.gemm_entries(p, rep, A, B, rows, cols)), (shape, M, N, K)
        M, N, K = 40, 36, (1 << 18) + 3
        for pattern in ("random", "maxprod"):
            A = mat(p, rep, M, K, 74, 0, pattern)
            B = mat(p, rep, K, N, 74, 1, pattern)
            got = to_host(F.gemm(to_dev(A), to_dev(B)))
            assert same(got, oracle.gemm(p, rep, A, B)), (shape, K, pattern)
    finally:
        fd.tune_set("gemm.i8.tile", None)
        fd.tune_set("gemm.i8.ktile", None)


@pytest.mark.parametrize("pad", [1, 0])
def test_gemm_int8_zero_padded_operands(pad):
    """K not a multiple of 64 and A rows at an odd stride (a column slice of a
    wider matrix): the direct-to-LDS kernel on zero-padded copies (pad=1,
    default) and the register-staged fallback (pad=0), both against the
    oracle, maximal products included."""
    p, rep = 251, "centred"
    F = field(p, rep)
    fd.tune_set("gemm.i8.pad", pad)
    try:
        for pattern in ("random", "maxprod"):
            M, N, K = 1037, 1100, 2517
            W = mat(p, rep, M, K + 3, 75, 0, pattern)
            B = mat(p, rep, K, N, 75, 1, pattern)
            Wd = to_dev(W)
            got = to_host(F.gemm(Wd[:, 1:K + 1], to_dev(B)))
            A = W[:, 1:K + 1]
            rows = synth.uniform_int(76, 0, 400, M)
            cols = synth.uniform_int(76, 1, 400, N)
            rows[:2] = [0, M - 1]
            cols[:2] = [0, N - 1]
            want = oracle.gemm_entries(p, rep, np.ascontiguousarray(A), B, rows, cols)
            assert same(got[rows, cols], want), (pad, pattern)
    finally:
        fd.tune_set("gemm.i8.pad", None)


@pytest.mark.parametrize("p,rep", [(1048573, "fp64"), (67108859, "fp64"), (65521, "zpz"),
                                   (32749, "mont")])
def test_gemm_fp64_unpadded_element_loads(p, rep):
    """Odd K and N through the FP64 matrix-core kernel's element loads (the
    zero-padded copies switched off), against the oracle."""
    F = field(p, rep)
    fd.tune_set("gemm.f64.pad", 0)
    try:
        for (M, N, K) in [(7, 5, 9), (130, 129, 33), (257, 301, 1001)]:
            A = mat(p, rep, M, K, 77, 0, "random")
            B = mat(p, rep, K, N, 77, 1, "random")
            got = to_host(F.gemm(to_dev(A), to_dev(B)))
            assert same(got, oracle.gemm(p, rep, A, B)), (p, rep, M, N, K)
    finally:
        fd.tune_set("gemm.f64.pad", None)


@pytest.mark.parametrize("waves", [4, 8, 16])
def test_gemm_fp64_wave_layouts(waves):
    """The FP64 matrix-core kernel with 4, 8 and 16 wavefronts per workgroup,
    plain and centred residues, ragged shapes, against the oracle."""
    fd.tune_set("gemm.f64.waves", waves)
    try:
        for p, K in [(1048573, 300), (67108859, 130), (1048573, 3 * 8192 + 6)]:
            F = field(p, "fp64")
            M, N = 150, 142
            A = mat(p, "fp64", M, K, 72, 0, "random")
            B = mat(p, "fp64", K, N, 72, 1, "random")
            got = to_host(F.gemm(to_dev(A), to_dev(B)))
            assert same(got, oracle.gemm(p, "fp64", A, B)), (waves, p, K)
    finally:
        fd.tune_set("gemm.f64.waves", None)


@pytest.mark.parametrize("p,rep", [(2147483647, "zpz"), (2147483647, "mont"), (4278124237, "zpz"),
                                   (2654435761, "mont"), (67108859, "fp64"), (67108859, "zpz"),
                                   (67108859, "mont"), (1048573, "fp64"), (65521, "zpz"),
                                   (32749, "mont"), (32749, "zpz"), (251, "zpz"), (251, "fp64"),
                                   (32749, "zech"), (65521, "zech"), (3, "zech")])
@pytest.mark.parametrize("M,N,K,tiles", [(300, 260, 700, "auto"), (1030, 1100, 1000, "auto"),
                                         (1030, 1100, 1000, "large"), (40, 36, 131008, "auto")])
def test_gemm_digit_split(p, rep, M, N, K, tiles):
    """Primes on the int8 matrix cores through D^2 digit products, D = 4, 3,
    2 and 1 balanced base-256 digits by the size of p, discrete-log codes
    included (the size thresholds are lowered so that every shape here takes
    them): ragged shapes, K not a
    multiple of 64, the largest K without folds, the large-tile kernel and
    the small one; sampled entries against the oracle, maximal products
    included."""
    F = field(p, rep)
    fd.tune_set("gemm.split.min_work", 1)
    fd.tune_set("gemm.split.zech_min_work", 1)
    fd.tune_set("gemm.split.small", 0 if tiles == "large" else None)
    try:
        _digit_split_case(F, p, rep, M, N, K)
    finally:
        fd.tune_set("gemm.split.min_work", None)
        fd.tune_set("gemm.split.zech_min_work", None)
        fd.tune_set("gemm.split.small", None)


def _digit_split_case(F, p, rep, M, N, K):
    for pattern in ("random", "maxprod"):
        A = mat(p, rep, M, K, 73, 0, pattern)
        B = mat(p, rep, K, N, 73, 1, pattern)
        got = to_host(F.gemm(to_dev(A), to_dev(B)))
        rows = synth.uniform_int(74, 0, 160, M)
        cols = synth.uniform_int(74, 1, 160, N)
        rows[:2] = [0, M - 1]
        cols[:2] = [0, N - 1]
        want = oracle.gemm_entries(p, rep, A, B, rows, cols)
        assert same(got[rows, cols], want), (p, rep, M, N, K, pattern)
