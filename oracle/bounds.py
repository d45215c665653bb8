"""The paper's overflow bounds, written as plain integer definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function states
the inequality the paper gives and solves it in Python's unbounded integers
(a quotient, or a bisection for the threshold followed by a downward walk to a
prime), so each can be checked by eye against the text.

* Sec. 2.1  AXPY a*x + y with a, x, y in [0, p-1] must not overflow an m-bit
            machine integer: p(p-1) <= 2^(m-1) - 1 when signed,
            p(p-1) <= 2^m - 1 when unsigned.
* Sec. 2.2  Montgomery AXPY: (p-1)^2 + p(B-1) < B^2.
* Sec. 2.4  Zech index arithmetic: indices lie in [0, q-1] and the sum of two
            of them must fit a signed m-bit integer: 2(q-1) <= 2^(m-1) - 1.
* Sec. 3.1  Eq. 1: lambda (p-1)^2 < 2^m.  Because the blocked loop of Sec. 3.2
            carries the residue of the previous block, the bound actually used
            by a schedule is (p-1) + lambda (p-1)^2 <= 2^m - 1 for integers and
            <= 2^53 for doubles (every integer up to 2^53 is exact).
* Sec. 3.2.2 centred: lambda ((p-1)/2)^2 < 2^(m-1).
* Sec. 3.4  Eq. 2 (hybrid block-overflow): lambda p (p-1) < 2^m.
"""
from __future__ import annotations


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    d = 3
    while d * d <= n:
        if n % d == 0:
            return False
        d += 2
    return True


def largest_prime_satisfying(pred, start: int) -> int:
    """Largest prime p <= start with pred(p); pred must be monotone (true for
    every integer up to some threshold, false above it).  The threshold is
    found by bisection, then primes are tried downwards from it."""
    lo, hi = 1, start
    if not pred(lo):
        raise ValueError("no integer satisfies the predicate")
    while lo < hi:  # invariant: pred(lo) holds
        mid = (lo + hi + 1) // 2
        if pred(mid):
            lo = mid
        else:
            hi = mid - 1
    p = lo
    while p >= 2:
        if is_prime(p):
            return p
        p -= 1
    raise ValueError("no prime satisfies the predicate")


def _isqrt(n: int) -> int:
    x = int(n ** 0.5)
    while x * x > n:
        x -= 1
    while (x + 1) * (x + 1) <= n:
        x += 1
    return x


def axpy_max_prime(m: int, signed: bool) -> int:
    """Sec. 2.1: largest prime whose AXPY p(p-1) fits an m-bit word."""
    limit = (1 << (m - 1)) - 1 if signed else (1 << m) - 1
    return largest_prime_satisfying(lambda p: p * (p - 1) <= limit, _isqrt(limit) + 2)


def montgomery_axpy_max_prime(b_bits: int) -> int:
    """Sec. 2.2: largest prime with (p-1)^2 + p(B-1) < B^2."""
    B = 1 << b_bits
    return largest_prime_satisfying(lambda p: (p - 1) ** 2 + p * (B - 1) < B * B, B)


def zech_max_prime(m: int) -> int:
    """Sec. 2.4: largest prime whose index sums 2(q-1) stay in a signed m-bit
    word."""
    limit = (1 << (m - 1)) - 1
    return largest_prime_satisfying(lambda p: 2 * (p - 1) <= limit, (1 << (m - 2)) + 1)


def eq1_lambda(p: int, m: int) -> int:
    """Eq. 1 read literally: largest lambda with lambda (p-1)^2 < 2^m."""
    return ((1 << m) - 1) // ((p - 1) ** 2)


def carried_lambda_int(p: int, m: int) -> int:
    """Largest lambda with (p-1) + lambda (p-1)^2 <= 2^m - 1 (unsigned m-bit)."""
    return ((1 << m) - 1 - (p - 1)) // ((p - 1) ** 2)


def carried_lambda_fp64(p: int) -> int:
    """Largest lambda with (p-1) + lambda (p-1)^2 <= 2^53 (double mantissa)."""
    return ((1 << 53) - (p - 1)) // ((p - 1) ** 2)


def centred_lambda(p: int, m: int) -> int:
    """Sec. 3.2.2: largest lambda with lambda ((p-1)/2)^2 < 2^(m-1)."""
    h = (p - 1) // 2
    return ((1 << (m - 1)) - 1) // (h * h)


def hybrid_lambda(p: int, m: int) -> int:
    """Eq. 2 (strict reading): largest lambda with lambda p (p-1) < 2^m."""
    return ((1 << m) - 1) // (p * (p - 1))


def hybrid_max_prime(n: int, m: int) -> int:
    """Sec. 3.4: largest prime with n p (p-1) < 2^m (one division for size n)."""
    return largest_prime_satisfying(lambda p: n * p * (p - 1) < (1 << m),
                                    _isqrt((1 << m) // n) + 2)


def montgomery_redc_terms(p: int, b_bits: int = 32) -> int:
    """Products X*Y (X, Y in [0,p)) that can be summed before a Montgomery
    reduction, whose input must stay below p*B (Sec. 2.2)."""
    return (p * (1 << b_bits) - 1) // ((p - 1) ** 2)


def zech_subtraction_correction_fraction(q: int) -> float:
    """Sec. 2.4: share of pairs (i, j), 1 <= i, j <= q-1, for which the index
    k = j - i + (q-1)/2 leaves [0, q-1) and needs one correction by q-1."""
    qb = q - 1
    half = qb // 2
    bad = 0
    for i in range(1, q):
        for j in range(1, q):
            k = j - i + half
            if k < 0 or k >= qb:
                bad += 1
    return bad / float(qb * qb)
