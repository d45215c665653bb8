"""Exact dot products and matrix products over GF(p) on MI355X (gfx950).

A thin binding over the C ABI of libfdot.so (include/fdot.h): it passes device
pointers of torch tensors and the current HIP stream, nothing else.  Every
step of the computation runs in the library's HIP kernels; there is no host
fallback, and importing this package fails loudly when the library is
missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDOT_LIB names another build of the same library (the host-instrumented
# copy the sanitizer run uses)
LIB_PATH = os.environ.get("FDOT_LIB") or os.path.join(_HERE, "libfdot.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python paper_cs_0404008_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

REPS = {"zpz": 0, "mont": 1, "fp64": 2, "zech": 3, "centred": 4}
ALGOS = {"auto": 0, "delayed": 1, "perterm": 2, "overflow": 3, "zech_tplus1": 4, "zech_exp": 5,
         "hybrid": 6}
ACCS = {"u64": 0, "u32": 1, "f64": 2, "i32_centred": 3, "f64_centred": 4, "mont_redc": 5,
        "u64_hybrid": 6}
BOUNDS = {"axpy_signed": 0, "axpy_unsigned": 1, "montgomery": 2, "zech_index": 3}
FOLDS = {"remainder": 0, "redc": 1, "fp64": 2}
NOALLOC_MAX_PAIRS = 65536  # FDOT_NOALLOC_MAX_PAIRS
EW_OPS = {"add": 0, "sub": 1, "neg": 2, "mul": 3, "div": 4, "axpy": 5, "axpyin": 6}
NP_DTYPES = {"zpz": "uint32", "mont": "uint32", "fp64": "float64", "zech": "uint16",
             "centred": "int8"}
TORCH_DTYPES = {"zpz": torch.uint32, "mont": torch.uint32, "fp64": torch.float64,
                "zech": torch.uint16, "centred": torch.int8}


class FieldInfo(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint64), ("rep", ctypes.c_int32), ("elem_bytes", ctypes.c_uint32),
                ("lambda_u64", ctypes.c_uint64), ("lambda_f64", ctypes.c_uint64),
                ("lambda_i32c", ctypes.c_uint64), ("lambda_redc", ctypes.c_uint64),
                ("corr", ctypes.c_uint64), ("norm_shift", ctypes.c_uint32),
                ("recip", ctypes.c_uint32), ("n_im", ctypes.c_uint32), ("b_mod_p", ctypes.c_uint32),
                ("binv_mod_p", ctypes.c_uint32), ("b2_mod_p", ctypes.c_uint32),
                ("g", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("inv_p", ctypes.c_double),
                ("table_bytes", ctypes.c_uint64), ("degree", ctypes.c_uint32),
                ("reserved2", ctypes.c_uint32), ("q", ctypes.c_uint64), ("modulus", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_
                if name not in ("reserved", "reserved2")}


_u64, _sz, _vp, _i32, _i64 = (ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int,
                             ctypes.c_int64)


def _sig(name, args, res=ctypes.c_int):
    fn = getattr(_lib, name)
    fn.argtypes = args
    fn.restype = res
    return fn


_sig("fdot_status_string", [_i32], ctypes.c_char_p)
_sig("fdot_version", [])
_sig("fdot_field_params", [_u64, _i32, ctypes.POINTER(FieldInfo)])
_sig("fdot_lambda", [_u64, _i32, ctypes.POINTER(_u64)])
_sig("fdot_max_prime", [_i32, ctypes.c_uint32, ctypes.POINTER(_u64)])
_sig("fdot_choose_rep", [_u64, _u64, ctypes.POINTER(_i32)])
_sig("fdot_host_fold", [ctypes.POINTER(FieldInfo), _i32, _u64, ctypes.POINTER(_u64)])
_sig("fdot_zech_tables", [_u64, _vp, _vp, _vp])
class Options(ctypes.Structure):
    _fields_ = [("validate", ctypes.c_uint32), ("algo", ctypes.c_int32), ("block", ctypes.c_uint64),
                ("reserved", ctypes.c_uint64 * 2)]


_sig("fdot_field_create", [_u64, _i32, ctypes.POINTER(Options), ctypes.POINTER(_vp)])
_sig("fdot_validate", [_vp, _vp, _sz, _vp, _vp])
_sig("fdot_field_create_ext", [_u64, ctypes.c_uint32, ctypes.POINTER(_vp)])
_sig("fdot_field_create_host", [_u64, _i32, ctypes.POINTER(_vp)])
_sig("fdot_field_destroy", [_vp])
_sig("fdot_field_info", [_vp, ctypes.POINTER(FieldInfo)])
_sig("fdot_encode", [_vp, _vp, _vp, _sz, _vp])
_sig("fdot_decode", [_vp, _vp, _vp, _sz, _vp])
_sig("fdot_modp", [_vp, _vp, _vp, _sz, _vp, _vp])
_sig("fdot_modp_algo", [_vp, _i32, _vp, _vp, _sz, _vp, _vp])
_sig("fdot_elementwise", [_vp, _i32, _sz, _vp, _vp, _vp, _vp, _vp])
_sig("fdot_modp_many_mixed", [_sz, _vp, _vp, _sz, _vp, _vp])
_sig("fdot_modp_many", [_vp, _sz, _vp, _vp, _vp])
_sig("fdot_modp_many_algo", [_vp, _i32, _sz, _vp, _vp, _vp])
_sig("fdot_modp_many_noalloc", [_vp, _i32, _sz, _vp, _vp, _vp])
_sig("fgemv_modp", [_vp, _sz, _sz, _vp, _sz, _vp, _vp, _vp])
_sig("fgemm_modp", [_vp, _sz, _sz, _sz, _vp, _sz, _vp, _sz, _vp, _sz, _vp])
_sig("fdot_workspace_reserve", [_vp, _sz])
_sig("fdot_trace_enable", [_i32])
_sig("fdot_trace_read", [_vp, _sz, ctypes.POINTER(_sz)])
_sig("fdot_tune_set", [ctypes.c_char_p, _i64])
_sig("fdot_tune_get", [ctypes.c_char_p, ctypes.POINTER(_i64)])
_sig("fdot_calib_read", [_vp, _sz, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp])
_sig("fdot_calib_mfma", [_i32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                         _vp, ctypes.POINTER(_u64), _vp])


class FdotError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_lib.fdot_status_string(status).decode()} ({status})")


def _check(status: int, what: str) -> None:
    if status != 0:
        raise FdotError(status, what)


def lib():
    return _lib


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ host only
def status_string(status: int) -> str:
    return _lib.fdot_status_string(status).decode()


def field_params(p: int, rep: str) -> dict:
    info = FieldInfo()
    _check(_lib.fdot_field_params(p, REPS[rep], ctypes.byref(info)), "fdot_field_params")
    return info.as_dict()


def field_params_status(p: int, rep: str) -> int:
    info = FieldInfo()
    return _lib.fdot_field_params(p, REPS[rep], ctypes.byref(info))


def lambda_for(p: int, acc: str) -> int:
    out = _u64()
    _check(_lib.fdot_lambda(p, ACCS[acc], ctypes.byref(out)), "fdot_lambda")
    return out.value


def max_prime(kind: str, bits: int) -> int:
    out = _u64()
    _check(_lib.fdot_max_prime(BOUNDS[kind], bits, ctypes.byref(out)), "fdot_max_prime")
    return out.value


def make_mixed_desc(xs, ys, field_index, device=None) -> torch.Tensor:
    """Device descriptor array {x, y, n, field} (fdot_mixed_desc_t) for a
    batch over several fields."""
    rows = []
    for x, y, k in zip(xs, ys, field_index):
        if x.numel() != y.numel():
            raise ValueError("length mismatch")
        rows.append([x.data_ptr(), y.data_ptr(), x.numel(), int(k)])
    dev = device or (xs[0].device if len(xs) else "cuda")
    return torch.tensor(rows, dtype=torch.int64).reshape(-1, 4).to(dev)


def dot_many_mixed(fields, desc: torch.Tensor, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """fdot_modp_many_mixed: results[k] over fields[desc[k].field] (all of one
    representation)."""
    if desc.dtype != torch.int64 or desc.dim() != 2 or desc.shape[1] != 4 or not desc.is_cuda:
        raise TypeError("desc must be a CUDA int64 tensor of shape [count, 4]")
    count = desc.shape[0]
    if out is None:
        out = torch.empty(count, dtype=fields[0].dtype, device=desc.device)
    handles = (_vp * max(len(fields), 1))(*[f.handle.value for f in fields])
    _check(_lib.fdot_modp_many_mixed(count, _ptr(desc), handles, len(fields), _ptr(out),
                                     _stream(stream)), "fdot_modp_many_mixed")
    return out


def choose_rep(p: int, n: int = 0) -> str:
    """The representation for dot products of length about n over GF(p) on
    this device (fdot_choose_rep): a measured choice from the tuning table,
    else the admissible one with the fewest bytes per element."""
    out = ctypes.c_int32()
    _check(_lib.fdot_choose_rep(p, n, ctypes.byref(out)), "fdot_choose_rep")
    return {v: k for k, v in REPS.items()}[out.value]


def host_fold(p: int, rep: str, kind: str, T: int) -> int:
    info = FieldInfo()
    _check(_lib.fdot_field_params(p, REPS[rep], ctypes.byref(info)), "fdot_field_params")
    out = _u64()
    _check(_lib.fdot_host_fold(ctypes.byref(info), FOLDS[kind], T, ctypes.byref(out)),
           "fdot_host_fold")
    return out.value


def zech_tables(p: int):
    import numpy as np
    val = np.zeros(p, dtype=np.uint16)
    idx = np.zeros(p, dtype=np.uint16)
    plus1 = np.zeros(p, dtype=np.uint16)
    _check(_lib.fdot_zech_tables(p, val.ctypes.data, idx.ctypes.data, plus1.ctypes.data),
           "fdot_zech_tables")
    return val, idx, plus1


def tune_set(key: str, value) -> None:
    """Set a tuned launch parameter; value None removes the key."""
    v = -(1 << 63) if value is None else int(value)
    _check(_lib.fdot_tune_set(key.encode(), v), "fdot_tune_set")


def tune_get(key: str):
    out = _i64()
    st = _lib.fdot_tune_get(key.encode(), ctypes.byref(out))
    return None if st != 0 else out.value


def trace_enable(on: bool = True) -> None:
    """Start (on) or stop recording the device time of every streaming
    dot-product kernel (fdot_trace_enable)."""
    _check(_lib.fdot_trace_enable(1 if on else 0), "fdot_trace_enable")


def trace_read():
    """Device milliseconds of each traced kernel since trace_enable(True), in
    launch order (waits for them)."""
    import numpy as np
    n = _sz()
    _check(_lib.fdot_trace_read(None, 0, ctypes.byref(n)), "fdot_trace_read")
    out = np.zeros(max(n.value, 1), dtype=np.float64)
    _check(_lib.fdot_trace_read(out.ctypes.data, n.value, ctypes.byref(n)), "fdot_trace_read")
    return out[:n.value]


def workspace_reserve(count: int, stream=None) -> None:
    _check(_lib.fdot_workspace_reserve(_stream(stream), count), "fdot_workspace_reserve")


def calib_read(x: torch.Tensor, out: torch.Tensor, blocks: int = 0, unroll: int = 8,
               stream=None) -> None:
    """Measured-peak read kernel: out[0] (int64 device tensor) = sum of the
    32-bit words of x mod 2^64, x read once."""
    if x.numel() * x.element_size() % 16:
        raise FdotError(2, "calib_read: size not a multiple of 16 bytes")
    _check(_lib.fdot_calib_read(_ptr(x), x.numel() * x.element_size() // 4, blocks, unroll,
                                _ptr(out), _stream(stream)), "fdot_calib_read")


def calib_mfma(kind: str, iters: int, a, b, out: torch.Tensor, blocks: int = 0,
               stream=None) -> int:
    """Matrix-core issue loop (kind "i8", "f64", or "i8_random" with a = seed);
    out: two-element device tensor (int32 or float64).  Returns the
    operations it executes."""
    ops = _u64()
    _check(_lib.fdot_calib_mfma({"i8": 0, "f64": 1, "i8_random": 2}[kind], blocks, iters, float(a), float(b),
                                _ptr(out), ctypes.byref(ops), _stream(stream)),
           "fdot_calib_mfma")
    return ops.value


# ---------------------------------------------------------------------- field
class Field:
    """GF(p) in one representation, or GF(p^degree) in discrete logarithms
    (rep "zech", degree >= 2); the handle owns the device tables."""

    def __init__(self, p: int, rep: str = "zpz", host_only: bool = False, degree: int = 1,
                 validate: bool = False, algo: str = "auto", block: int = 0):
        """validate / algo / block: the creation options of fdot_field_create
        (check inputs before every compute call, the schedule used for
        "auto", the delay block of the delayed schedules; 0 = lambda)."""
        self.p = int(p)
        self.rep = rep
        h = _vp()
        opts = None
        if validate or algo != "auto" or block:
            if degree > 1 or host_only:
                raise ValueError("options apply to device prime fields")
            opts = ctypes.byref(Options(1 if validate else 0, ALGOS[algo], int(block)))
        if degree > 1:
            if rep != "zech" or host_only:
                raise ValueError("extension fields are held in discrete logarithms on the device")
            _check(_lib.fdot_field_create_ext(self.p, degree, ctypes.byref(h)),
                   "fdot_field_create_ext")
        elif host_only:  # constants only, no GPU (compute calls are refused)
            _check(_lib.fdot_field_create_host(self.p, REPS[rep], ctypes.byref(h)),
                   "fdot_field_create_host")
        else:
            _check(_lib.fdot_field_create(self.p, REPS[rep], opts, ctypes.byref(h)),
                   "fdot_field_create")
        self._h = h
        info = FieldInfo()
        _check(_lib.fdot_field_info(h, ctypes.byref(info)), "fdot_field_info")
        self.info = info.as_dict()
        self.dtype = TORCH_DTYPES[rep]

    def __del__(self, _destroy=_lib.fdot_field_destroy):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def _need(self, t: torch.Tensor, name: str):
        if t.dtype != self.dtype or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor of dtype {self.dtype}")

    def validate(self, x: torch.Tensor, count: torch.Tensor | None = None, stream=None):
        """fdot_validate: add the number of non-canonical stored values of x to
        count (a one-element int64 device tensor, created zeroed if None)."""
        self._need(x, "x")
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        if count is None:
            count = torch.zeros(1, dtype=torch.int64, device=x.device)
        _check(_lib.fdot_validate(self._h, _ptr(x), x.numel(), _ptr(count), _stream(stream)),
               "fdot_validate")
        return count

    def encode(self, canon: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        if canon.dtype != torch.uint32 or not canon.is_cuda or not canon.is_contiguous():
            raise TypeError("canon must be a contiguous CUDA uint32 tensor")
        if out is None:
            out = torch.empty(canon.shape, dtype=self.dtype, device=canon.device)
        _check(_lib.fdot_encode(self._h, _ptr(canon), _ptr(out), canon.numel(), _stream(stream)),
               "fdot_encode")
        return out

    def decode(self, rep: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        self._need(rep, "rep")
        if out is None:
            out = torch.empty(rep.shape, dtype=torch.uint32, device=rep.device)
        _check(_lib.fdot_decode(self._h, _ptr(rep), _ptr(out), rep.numel(), _stream(stream)),
               "fdot_decode")
        return out

    def elementwise(self, op: str, x: torch.Tensor, y: torch.Tensor | None = None,
                    alpha=None, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """fdot_elementwise: op in EW_OPS; y for add/sub/mul/div/axpy, alpha (a
        stored value of this representation) for axpy/axpyin; axpyin updates
        out in place (out is required)."""
        import numpy as np
        code = EW_OPS[op]
        self._need(x, "x")
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        if op in ("add", "sub", "mul", "div", "axpy"):
            self._need(y, "y")
            if y.numel() != x.numel() or not y.is_contiguous():
                raise ValueError("y must be contiguous and as long as x")
        if op == "axpyin" and out is None:
            raise ValueError("axpyin updates out in place")
        if out is None:
            out = torch.empty_like(x)
        self._need(out, "out")
        if out.numel() != x.numel() or not out.is_contiguous():
            raise ValueError("out must be contiguous and as long as x")
        a = None
        if op in ("axpy", "axpyin"):
            if alpha is None:
                raise ValueError(f"{op} needs alpha")
            a = np.array([alpha], dtype=NP_DTYPES[self.rep])
        _check(_lib.fdot_elementwise(self._h, code, x.numel(), a.ctypes.data if a is not None else None,
                                     _ptr(x), _ptr(y) if y is not None else None, _ptr(out),
                                     _stream(stream)), "fdot_elementwise")
        return out

    def dot(self, x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None,
            algo: str = "auto", stream=None) -> torch.Tensor:
        self._need(x, "x")
        self._need(y, "y")
        if x.numel() != y.numel() or not x.is_contiguous() or not y.is_contiguous():
            raise ValueError("x and y must be contiguous and of equal length")
        if out is None:
            out = torch.empty(1, dtype=self.dtype, device=x.device)
        _check(_lib.fdot_modp_algo(self._h, ALGOS[algo], _ptr(x), _ptr(y), x.numel(), _ptr(out),
                                   _stream(stream)), "fdot_modp")
        return out

    @staticmethod
    def make_desc(xs, ys, device=None) -> torch.Tensor:
        """Device descriptor array {x, y, n} for a batch of tensor pairs.  The
        returned tensor keeps references to the operand tensors, so that their
        memory outlives the descriptors that point into it."""
        rows = []
        xs, ys = list(xs), list(ys)
        for x, y in zip(xs, ys):
            if x.numel() != y.numel():
                raise ValueError("length mismatch")
            rows.append([x.data_ptr(), y.data_ptr(), x.numel()])
        dev = device or (xs[0].device if len(xs) else "cuda")
        desc = torch.tensor(rows, dtype=torch.int64).reshape(-1, 3).to(dev)
        desc._fdot_operands = (xs, ys)
        return desc

    def dot_many(self, desc: torch.Tensor, out: torch.Tensor | None = None, algo: str = "auto",
                 stream=None) -> torch.Tensor:
        if desc.dtype != torch.int64 or desc.dim() != 2 or desc.shape[1] != 3 or not desc.is_cuda:
            raise TypeError("desc must be a CUDA int64 tensor of shape [count, 3]")
        count = desc.shape[0]
        if out is None:
            out = torch.empty(count, dtype=self.dtype, device=desc.device)
        _check(_lib.fdot_modp_many_algo(self._h, ALGOS[algo], count, _ptr(desc), _ptr(out),
                                        _stream(stream)), "fdot_modp_many")
        return out

    def dot_many_noalloc(self, desc: torch.Tensor, out: torch.Tensor, algo: str = "auto",
                         stream=None) -> torch.Tensor:
        """fdot_modp_many_noalloc: dot_many with the library's fixed scratch
        (no device allocation at the call; at most NOALLOC_MAX_PAIRS pairs)."""
        if desc.dtype != torch.int64 or desc.dim() != 2 or desc.shape[1] != 3 or not desc.is_cuda:
            raise TypeError("desc must be a CUDA int64 tensor of shape [count, 3]")
        self._need(out, "out")
        if out.numel() < desc.shape[0]:
            raise ValueError("out is shorter than the batch")
        _check(_lib.fdot_modp_many_noalloc(self._h, ALGOS[algo], desc.shape[0], _ptr(desc),
                                           _ptr(out), _stream(stream)), "fdot_modp_many_noalloc")
        return out

    def gemv(self, A: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
        self._need(A, "A")
        self._need(x, "x")
        m, n = A.shape
        if A.stride(1) != 1 or x.numel() != n or not x.is_contiguous():
            raise ValueError("A must be row-major and x of length A.shape[1]")
        if out is None:
            out = torch.empty(m, dtype=self.dtype, device=A.device)
        _check(_lib.fgemv_modp(self._h, m, n, _ptr(A), A.stride(0), _ptr(x), _ptr(out),
                               _stream(stream)), "fgemv_modp")
        return out

    def gemm(self, A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
        self._need(A, "A")
        self._need(B, "B")
        M, K = A.shape
        K2, N = B.shape
        if K != K2 or A.stride(1) != 1 or B.stride(1) != 1:
            raise ValueError("A and B must be row-major with matching inner dimension")
        if out is None:
            out = torch.empty((M, N), dtype=self.dtype, device=A.device)
        _check(_lib.fgemm_modp(self._h, M, N, K, _ptr(A), A.stride(0), _ptr(B), B.stride(0),
                               _ptr(out), out.stride(0), _stream(stream)), "fgemm_modp")
        return out


# -------------------------------------------------------------------- serving
OPS = {"dot": 0, "gemv": 1, "gemm": 2}


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("reserved", ctypes.c_int32), ("field", _vp),
                ("a", _vp), ("b", _vp), ("out", _vp), ("m", _u64), ("n", _u64), ("k", _u64),
                ("footprint", _u64), ("ready", _vp)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", _u64), ("max_inflight", ctypes.c_uint32),
                ("max_queue", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("fake_device", ctypes.c_uint32),
                ("plain", ctypes.c_uint32), ("exclusive_ns", _u64), ("short_ns", _u64),
                ("matrix_depth", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Timing(ctypes.Structure):
    _fields_ = [("submit_ns", _u64), ("admit_ns", _u64), ("launch_ns", _u64), ("done_ns", _u64),
                ("status", ctypes.c_int32), ("batch_size", ctypes.c_uint32),
                ("stream", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("rejected", _u64), ("launches", _u64),
                ("peak_footprint", _u64), ("peak_inflight", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


_sig("fdot_server_create", [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)])
_sig("fdot_server_submit", [_vp, ctypes.POINTER(Request), ctypes.POINTER(_u64)])
_sig("fdot_server_poll", [_vp, _u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Timing)])
_sig("fdot_server_drain", [_vp, _u64])
_sig("fdot_server_replay", [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_double), _sz,
                            ctypes.POINTER(Timing)])
_sig("fdot_server_stats", [_vp, ctypes.POINTER(ServerStats)])
_sig("fdot_server_destroy", [_vp])


def make_request(op: str, field: "Field", a, b, out, m: int = 0, n: int = 0, k: int = 0,
                 footprint: int = 0, ready=None) -> Request:
    """A request on device tensors (a, b, out) of field's dtype; a/b/out may
    also be raw device addresses (ints).  ready: an optional torch.cuda.Event
    recorded after the operands were written; the launch waits for it."""
    addr = lambda t: t if isinstance(t, int) else t.data_ptr()  # noqa: E731
    ev = None if ready is None else (ready.cuda_event if hasattr(ready, "cuda_event") else int(ready))
    return Request(OPS[op], 0, field.handle, addr(a), addr(b), addr(out), m, n, k, footprint, ev)


class Server:
    """The continuous-batching request server of libfdot (one GPU)."""

    def __init__(self, hbm_budget: int = 0, max_inflight: int = 0, max_queue: int = 0,
                 streams: int = 0, max_batch: int = 0, fake_device: bool = False,
                 plain: bool = False, exclusive_ns: int = 0, short_ns: int = 0,
                 matrix_depth: int = 0):
        cfg = ServerConfig(hbm_budget, max_inflight, max_queue, streams, max_batch,
                           1 if fake_device else 0, 1 if plain else 0, exclusive_ns, short_ns,
                           matrix_depth, 0)
        h = _vp()
        _check(_lib.fdot_server_create(ctypes.byref(cfg), ctypes.byref(h)), "fdot_server_create")
        self._h = h

    def close(self, _destroy=_lib.fdot_server_destroy):
        if getattr(self, "_h", None) is not None and self._h.value:
            _destroy(self._h)
            self._h = None

    __del__ = close

    def submit(self, req: Request) -> int:
        t = _u64()
        _check(_lib.fdot_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
               "fdot_server_submit")
        return t.value

    def try_submit(self, req: Request):
        """(status, ticket) without raising."""
        t = _u64()
        st = _lib.fdot_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        return st, t.value

    def poll(self, ticket: int):
        done = ctypes.c_int()
        tm = Timing()
        _check(_lib.fdot_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(tm)),
               "fdot_server_poll")
        return bool(done.value), tm

    def drain(self, timeout_ms: int = 600000) -> None:
        _check(_lib.fdot_server_drain(self._h, timeout_ms), "fdot_server_drain")

    def replay(self, reqs, arrivals):
        """Submit reqs[i] at arrivals[i] seconds after the call; returns the
        timings (structured numpy array, nanoseconds)."""
        import numpy as np
        n = len(reqs)
        arr = (Request * max(n, 1))(*reqs)
        at = (ctypes.c_double * max(n, 1))(*[float(x) for x in arrivals])
        tm = (Timing * max(n, 1))()
        _check(_lib.fdot_server_replay(self._h, arr, at, n, tm), "fdot_server_replay")
        dt = np.dtype([("submit_ns", np.uint64), ("admit_ns", np.uint64), ("launch_ns", np.uint64),
                       ("done_ns", np.uint64), ("status", np.int32), ("batch_size", np.uint32),
                       ("stream", np.uint32), ("reserved", np.uint32)])
        return np.frombuffer(bytes(tm), dtype=dt, count=n).copy()

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib.fdot_server_stats(self._h, ctypes.byref(s)), "fdot_server_stats")
        return {name: getattr(s, name) for name, _ in s._fields_ if name != "reserved"}
