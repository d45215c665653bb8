"""The shared seeded input generator (host side)."""
import os

import numpy as np

import synth
from tests.conftest import GOLDEN


def test_splitmix64_published_vector():
    want = [int(line) for line in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if line.strip() and not line.startswith("#")]
    # sequential SplitMix64 from seed s: output i = mix64(s + (i+1) * gamma)
    got = [synth.mix64_int(1234567 + (i + 1) * int(synth.GAMMA)) for i in range(len(want))]
    assert got == want
    # the vectorised finaliser agrees with the scalar one
    z = np.array([1234567 + (i + 1) * int(synth.GAMMA) for i in range(5)], dtype=object)
    z = np.array([int(v) % (1 << 64) for v in z], dtype=np.uint64)
    assert [int(v) for v in synth._mix64(z)] == want


def test_counter_form_and_offsets():
    a = synth.raw_u64(3, 4, 1000)
    b = synth.raw_u64(3, 4, 400, offset=600)
    assert np.array_equal(a[600:], b)
    k = synth.key(3, 4)
    assert int(a[0]) == synth.mix64_int(k + int(synth.GAMMA))
    assert not np.array_equal(a, synth.raw_u64(3, 5, 1000))


def test_ranges():
    for m in [1, 2, 251, 32749, 4294967291, 1 << 32]:
        u = synth.uniform_int(1, 0, 20000, m)
        assert u.min() >= 0 and u.max() < m
    c = synth.uniform_int(1, 1, 20000, 251, lo=-125)
    assert c.min() == -125 and c.max() == 125
    f = synth.uniform_float(1, 2, 10000)
    assert f.min() >= 0.0 and f.max() < 1.0
    n = synth.log_uniform_lengths(2, 0, 4096, 3.0, 6.0)
    assert n.min() >= 1000 and n.max() < 1000000
