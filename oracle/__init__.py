"""Python face of the reference oracle (oracle.c) plus the paper's bounds.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the GPU path.  See oracle.c for what is computed and why it is the plain
definition of the result.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import bounds  # noqa: F401  (re-exported)

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c (the sanitizer run's)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

REPS = {"zpz": 0, "mont": 1, "fp64": 2, "zech": 3, "centred": 4}
DTYPES = {"zpz": np.uint32, "mont": np.uint32, "fp64": np.float64,
          "zech": np.uint16, "centred": np.int8}
MONT_B = 1 << 32

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with the host C compiler."""
    if os.environ.get("ORACLE_LIB"):
        return LIB_PATH  # built elsewhere
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC",
                               "-shared", SRC_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        u64, sz, vp, i32 = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int
        L.orc_is_prime.argtypes = [u64]
        L.orc_inv_mod.argtypes = [u64, u64]
        L.orc_inv_mod.restype = u64
        L.orc_primitive_root.argtypes = [u64]
        L.orc_primitive_root.restype = u64
        L.orc_encode_array.argtypes = [u64, i32, vp, vp, sz]
        L.orc_decode_array.argtypes = [u64, i32, vp, vp, sz]
        L.orc_dot.argtypes = [u64, i32, vp, vp, sz, vp]
        L.orc_dot_many.argtypes = [u64, i32, sz, vp, vp, vp, vp]
        L.orc_gemm.argtypes = [u64, i32, sz, sz, sz, vp, sz, vp, sz, vp, sz]
        L.orc_gemm_entries.argtypes = [u64, i32, sz, vp, sz, vp, sz, sz, vp, vp, vp]
        L.orc_gemv.argtypes = [u64, i32, sz, sz, vp, sz, vp, vp]
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_elementwise.argtypes = [u64, i32, i32, sz, vp, vp, vp, vp]
        L.orc_ext_modulus.argtypes = [u64, i32, vp]
        L.orc_ext_encode.argtypes = [u64, i32, vp, vp, sz]
        L.orc_ext_decode.argtypes = [u64, i32, vp, vp, sz]
        L.orc_ext_dot.argtypes = [u64, i32, vp, vp, sz, vp]
        L.orc_ext_elementwise.argtypes = [u64, i32, i32, sz, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _arr(a, rep):
    return np.ascontiguousarray(np.asarray(a), dtype=DTYPES[rep])


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def set_threads(n: int) -> None:
    """Threads of the batched oracle entry points (n <= 0: one per processor);
    only the time changes, never a result."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def is_prime(p: int) -> bool:
    return bool(lib().orc_is_prime(p))


def inv_mod(a: int, p: int) -> int:
    return int(lib().orc_inv_mod(a, p))


def primitive_root(p: int) -> int:
    return int(lib().orc_primitive_root(p))


def encode(p: int, rep: str, canon) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(canon, dtype=np.uint64))
    out = np.empty(c.shape, dtype=DTYPES[rep])
    _check(lib().orc_encode_array(p, REPS[rep], _ptr(c), _ptr(out), c.size), "encode")
    return out


def decode(p: int, rep: str, v) -> np.ndarray:
    a = _arr(v, rep)
    out = np.empty(a.shape, dtype=np.uint64)
    _check(lib().orc_decode_array(p, REPS[rep], _ptr(a), _ptr(out), a.size), "decode")
    return out


def dot(p: int, rep: str, x, y):
    """Exact dot product in representation rep; returns a numpy scalar."""
    xa, ya = _arr(x, rep), _arr(y, rep)
    if xa.size != ya.size:
        raise ValueError("length mismatch")
    out = np.zeros(1, dtype=DTYPES[rep])
    _check(lib().orc_dot(p, REPS[rep], _ptr(xa), _ptr(ya), xa.size, _ptr(out)), "dot")
    return out[0]


def dot_many(p: int, rep: str, xs, ys) -> np.ndarray:
    """Independent dot products of the pairs (xs[k], ys[k])."""
    xs = [_arr(a, rep) for a in xs]
    ys = [_arr(a, rep) for a in ys]
    count = len(xs)
    xp = (ctypes.c_void_p * max(count, 1))(*[_ptr(a) for a in xs])
    yp = (ctypes.c_void_p * max(count, 1))(*[_ptr(a) for a in ys])
    ns = np.array([a.size for a in xs], dtype=np.uint64)
    for a, b in zip(xs, ys):
        if a.size != b.size:
            raise ValueError("length mismatch")
    out = np.zeros(count, dtype=DTYPES[rep])
    _check(lib().orc_dot_many(p, REPS[rep], count, ctypes.addressof(xp),
                              ctypes.addressof(yp), _ptr(ns), _ptr(out)), "dot_many")
    return out


def gemm(p: int, rep: str, A, B) -> np.ndarray:
    A, B = _arr(A, rep), _arr(B, rep)
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimension mismatch")
    C = np.zeros((M, N), dtype=DTYPES[rep])
    _check(lib().orc_gemm(p, REPS[rep], M, N, K, _ptr(A), K, _ptr(B), N, _ptr(C), N), "gemm")
    return C


def gemm_entries(p: int, rep: str, A, B, rows, cols) -> np.ndarray:
    A, B = _arr(A, rep), _arr(B, rep)
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimension mismatch")
    r = np.ascontiguousarray(rows, dtype=np.uint64)
    c = np.ascontiguousarray(cols, dtype=np.uint64)
    if r.size and (r.max() >= M or c.max() >= N):
        raise ValueError("entry out of range")
    out = np.zeros(r.size, dtype=DTYPES[rep])
    _check(lib().orc_gemm_entries(p, REPS[rep], K, _ptr(A), K, _ptr(B), N, r.size,
                                  _ptr(r), _ptr(c), _ptr(out)), "gemm_entries")
    return out


def gemv(p: int, rep: str, A, x) -> np.ndarray:
    A, x = _arr(A, rep), _arr(x, rep)
    m, n = A.shape
    if x.size != n:
        raise ValueError("length mismatch")
    y = np.zeros(m, dtype=DTYPES[rep])
    _check(lib().orc_gemv(p, REPS[rep], m, n, _ptr(A), n, _ptr(x), _ptr(y)), "gemv")
    return y


EW_OPS = {"add": 0, "sub": 1, "neg": 2, "mul": 3, "div": 4, "axpy": 5, "axpyin": 6}


def elementwise(p: int, rep: str, op: str, x, y=None, alpha=None, r=None) -> np.ndarray:
    """The elementwise operation op (Sec. 2) on stored values of rep:
    add/sub/mul/div (x, y), neg (x), axpy (alpha * x + y), axpyin
    (alpha * x + r); returns a new array."""
    xa = _arr(x, rep)
    ya = _arr(y, rep) if y is not None else np.zeros_like(xa)
    out = _arr(r, rep).copy() if r is not None else np.zeros_like(xa)
    al = _arr([alpha if alpha is not None else 0], rep)
    if ya.size != xa.size or out.size != xa.size:
        raise ValueError("length mismatch")
    _check(lib().orc_elementwise(p, REPS[rep], EW_OPS[op], xa.size, _ptr(al), _ptr(xa),
                                 _ptr(ya), _ptr(out)), "elementwise")
    return out


# ------------------------------------------------- extension fields GF(p^d)
def ext_modulus(p: int, d: int) -> int:
    """The modulus polynomial f of GF(p^d) as the integer f(p)."""
    out = np.zeros(1, dtype=np.uint64)
    _check(lib().orc_ext_modulus(p, d, _ptr(out)), "ext_modulus")
    return int(out[0])


def ext_encode(p: int, d: int, values) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(values, dtype=np.uint32))
    out = np.empty(v.shape, dtype=np.uint16)
    _check(lib().orc_ext_encode(p, d, _ptr(v), _ptr(out), v.size), "ext_encode")
    return out


def ext_decode(p: int, d: int, codes) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(codes, dtype=np.uint16))
    out = np.empty(c.shape, dtype=np.uint32)
    _check(lib().orc_ext_decode(p, d, _ptr(c), _ptr(out), c.size), "ext_decode")
    return out


def ext_dot(p: int, d: int, x, y) -> int:
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint16))
    ya = np.ascontiguousarray(np.asarray(y, dtype=np.uint16))
    if xa.size != ya.size:
        raise ValueError("length mismatch")
    out = np.zeros(1, dtype=np.uint16)
    _check(lib().orc_ext_dot(p, d, _ptr(xa), _ptr(ya), xa.size, _ptr(out)), "ext_dot")
    return int(out[0])


def ext_elementwise(p: int, d: int, op: str, x, y=None, alpha=None, r=None) -> np.ndarray:
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint16))
    ya = np.ascontiguousarray(np.asarray(y if y is not None else np.zeros_like(xa), dtype=np.uint16))
    out = np.ascontiguousarray(np.asarray(r, dtype=np.uint16)).copy() if r is not None else np.zeros_like(xa)
    al = np.array([alpha if alpha is not None else 0], dtype=np.uint16)
    _check(lib().orc_ext_elementwise(p, d, EW_OPS[op], xa.size, _ptr(al), _ptr(xa), _ptr(ya),
                                     _ptr(out)), "ext_elementwise")
    return out
