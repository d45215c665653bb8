"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds the input generator only: no field arithmetic, no reduction,
nothing of the dot-product method.  Both sides of every parity test draw their
inputs from here (the host side below, or the device twin in ``synth.hip`` that
produces the same bits on the GPU for inputs too large to ship over PCIe).

Generator (published definitions, restated):

* SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom
  number generators", OOPSLA 2014): the state advances by the golden gamma
  0x9E3779B97F4A7C15 and each output is ``mix64(state)`` with the
  finaliser (z ^ z>>30)*0xBF58476D1CE4E5B9, (z ^ z>>27)*0x94D049BB133111EB,
  z ^ z>>31.  Used here in counter form: output i of a stream is
  ``mix64(key + (i+1)*gamma)``.
* key(seed, stream) = mix64(mix64(seed + gamma) + stream*gamma).
* Range reduction to [0, m) for m <= 2**32 is Lemire's multiply-shift
  (D. Lemire, "Fast random integer generation in an interval", TOMACS 2019)
  applied to the high 32 bits: ((z >> 32) * m) >> 32.  The small bias is
  irrelevant for synthetic inputs.
* A uniform double in [0, 1) is (z >> 11) * 2**-53.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1

__all__ = [
    "mix64_int", "key", "raw_u64", "uniform_int", "uniform_float",
    "log_uniform_lengths",
]


def mix64_int(z: int) -> int:
    """Scalar SplitMix64 finaliser on a Python int (mod 2**64)."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def key(seed: int, stream: int) -> int:
    """Per-(seed, stream) starting state."""
    g = int(GAMMA)
    return mix64_int((mix64_int((seed + g) & _MASK) + stream * g) & _MASK)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def raw_u64(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+n-1 of stream (seed, stream) as uint64."""
    k = np.uint64(key(seed, stream))
    i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(k + i * GAMMA)


def uniform_int(seed: int, stream: int, n: int, m: int, lo: int = 0,
                offset: int = 0) -> np.ndarray:
    """n integers uniform in [lo, lo+m), m <= 2**32, returned as int64."""
    if not (1 <= m <= (1 << 32)):
        raise ValueError("range size must be in [1, 2**32]")
    z = raw_u64(seed, stream, n, offset)
    with np.errstate(over="ignore"):
        u = ((z >> np.uint64(32)) * np.uint64(m)) >> np.uint64(32)
    return u.astype(np.int64) + lo


def uniform_float(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """n doubles uniform in [0, 1)."""
    z = raw_u64(seed, stream, n, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def log_uniform_lengths(seed: int, stream: int, count: int, lo_exp: float,
                        hi_exp: float) -> np.ndarray:
    """count lengths floor(10**(lo_exp + (hi_exp-lo_exp)*u)), u uniform."""
    u = uniform_float(seed, stream, count)
    n = np.floor(10.0 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
    return np.maximum(n, 1)


# ------------------------------------------------------------- device twin
_DTYPE_CODES = {"uint32": 0, "uint16": 1, "float64": 2, "int8": 3, "int64": 4}
_dev_lib = None


def _device_lib():
    global _dev_lib
    if _dev_lib is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it first")
        L = ctypes.CDLL(path)
        L.synth_fill.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p]
        L.synth_fill.restype = ctypes.c_int
        _dev_lib = L
    return _dev_lib


def fill_device(t, seed: int, stream: int, m: int, lo: int = 0, offset: int = 0,
                hip_stream=None) -> None:
    """Write uniform_int(seed, stream, t.numel(), m, lo, offset) into the
    contiguous CUDA tensor t (uint32, uint16, float64, int8 or int64) on the
    GPU: the same values the host generator produces."""
    import ctypes
    import torch
    if not t.is_cuda or not t.is_contiguous():
        raise TypeError("t must be a contiguous CUDA tensor")
    name = str(t.dtype).replace("torch.", "")
    if name not in _DTYPE_CODES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    s = hip_stream if hip_stream is not None else torch.cuda.current_stream().cuda_stream
    rc = _device_lib().synth_fill(seed, stream, offset, t.numel(), m, lo, _DTYPE_CODES[name],
                                  ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(s))
    if rc != 0:
        raise RuntimeError(f"synth_fill failed ({rc})")
