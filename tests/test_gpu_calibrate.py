"""The measured-peak kernels: the read kernel's sum of words against numpy's
(every word read exactly once, whatever the grid, unroll and ragged size),
the matrix loops' accumulators against their closed form iters * K * a * b,
and the refusal of malformed arguments."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_cs_0404008_amd")


@pytest.mark.parametrize("words", [0, 4, 1024, 4 * 100003, 1 << 22])
@pytest.mark.parametrize("blocks,unroll", [(0, 8), (0, 4), (7, 8), (300, 4)])
def test_read_sum(words, blocks, unroll):
    x = synth.uniform_int(80, words % 7, words, 1 << 32).astype(np.uint32)
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    out = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    fd.calib_read(xd, out, blocks=blocks, unroll=unroll)
    got = int(out.cpu().numpy().view(np.uint64)[0])
    assert got == int(x.astype(np.uint64).sum(dtype=np.uint64))


def test_read_sum_repeated_calls_restart_from_zero():
    x = torch.ones(4096, dtype=torch.int32, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    for _ in range(3):
        fd.calib_read(x, out)
        assert int(out.item()) == 4096


@pytest.mark.parametrize("a,b,iters", [(3, -5, 100), (-128, 127, 1), (1, 1, 0), (127, 127, 2000)])
def test_mfma_i8_loop(a, b, iters):
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    ops = fd.calib_mfma("i8", iters, a, b, out, blocks=3)
    want = (iters * 32 * a * b + (1 << 31)) % (1 << 32) - (1 << 31)  # int32 wrap
    assert int(out[0].item()) == want
    assert int(out[1].item()) == 0
    assert ops == 3 * 8 * iters * 4 * 2 * 32 ** 3


def _lowbias32(x):
    """The lowbias32 integer hash (C. Wellons), on Python integers."""
    x &= 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def _sbytes(word):
    return [((word >> (8 * j)) & 0xFF) - (256 if (word >> (8 * j)) & 0x80 else 0) for j in range(4)]


@pytest.mark.parametrize("seed,iters", [(0, 1), (12345, 3), (4294967295, 1000)])
def test_mfma_i8_random_operand_loop(seed, iters):
    """Element 0 of the first accumulator = iters x (bytewise dot of lanes 0
    and 32 of chain 0's left operand with the right operand), int32 wrap."""
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    ops = fd.calib_mfma("i8_random", iters, seed, 0, out, blocks=5)
    per = 0
    for lane in (0, 32):
        for w in range(4):
            a = _lowbias32(seed ^ _lowbias32(lane * 256 + w))
            b = _lowbias32(seed ^ _lowbias32(lane * 256 + 128 + w))
            per += sum(x * y for x, y in zip(_sbytes(a), _sbytes(b)))
    want = (iters * per + (1 << 31)) % (1 << 32) - (1 << 31)
    assert int(out[0].item()) == want
    assert ops == 5 * 8 * iters * 4 * 2 * 32 ** 3


@pytest.mark.parametrize("a,b,iters", [(1.5, 2.0, 1000), (-0.25, 8.0, 7)])
def test_mfma_f64_loop(a, b, iters):
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    ops = fd.calib_mfma("f64", iters, a, b, out)
    assert float(out[0].item()) == iters * 4 * a * b
    assert ops == fd.calib_mfma("f64", 1, a, b, torch.zeros(2, dtype=torch.float64,
                                                            device="cuda")) * iters


def test_calib_rejects_bad_arguments():
    x = torch.zeros(64, dtype=torch.int32, device="cuda")
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(fd.FdotError):
        fd.calib_read(x, out, unroll=5)
    with pytest.raises(fd.FdotError):
        fd.calib_read(x[1:61], out)          # not 16-byte aligned
    with pytest.raises(fd.FdotError):
        fd.calib_mfma("i8", 1, 200, 1, out.view(torch.int32))
    with pytest.raises(fd.FdotError):
        fd.calib_mfma("i8", 1, 0.5, 1, out.view(torch.int32))
    with pytest.raises(fd.FdotError):
        fd.calib_mfma("i8_random", 1, -1, 0, out.view(torch.int32))
    with pytest.raises(KeyError):
        fd.calib_mfma("bf16", 1, 1, 1, out)
