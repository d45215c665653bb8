"""Shared helpers of the GPU parity tests: seeded inputs in each
representation's storage domain (from the shared generator) and host/device
transfers.  Nothing here computes a field operation."""
import numpy as np
import torch

import synth

NP_DTYPES = {"zpz": np.uint32, "mont": np.uint32, "fp64": np.float64, "zech": np.uint16,
             "centred": np.int8}
TORCH_DTYPES = {"zpz": torch.uint32, "mont": torch.uint32, "fp64": torch.float64,
                "zech": torch.uint16, "centred": torch.int8}
ELEM_BYTES = {"zpz": 4, "mont": 4, "fp64": 8, "zech": 2, "centred": 1}


def storage_range(p, rep):
    """(size, low) of the canonical stored values of rep: every representation
    is a bijection onto GF(p), so uniform stored values are uniform field
    elements."""
    if rep == "centred":
        h = (p - 1) // 2
        return 2 * h + 1, -h
    return p, 0


def stored(p, rep, n, seed, stream, pattern="random"):
    if pattern == "random":
        m, lo = storage_range(p, rep)
        v = synth.uniform_int(seed, stream, n, m, lo)
    elif pattern == "maxprod":  # every element is p-1 (or its code): products (p-1)^2
        v = np.full(n, max_element(p, rep), dtype=np.int64)
    else:
        raise ValueError(pattern)
    return v.astype(NP_DTYPES[rep])


def max_element(p, rep):
    """Stored value of the field element p-1 = -1."""
    if rep in ("zpz", "fp64"):
        return p - 1
    if rep == "mont":
        return ((p - 1) << 32) % p
    if rep == "centred":
        return -1
    if rep == "zech":
        import oracle
        return int(oracle.encode(p, "zech", [p - 1])[0])
    raise ValueError(rep)


def to_dev(a, rep=None):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return a.shape == b.shape and a.tobytes() == b.tobytes()
