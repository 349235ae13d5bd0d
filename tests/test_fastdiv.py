"""The block-index decode of the kernels divides by invariant divisors with a
multiply-high and a shift; this replays that arithmetic (32-bit, as written in
the library's common.hpp) against exact integer division."""
import numpy as np


def magic(d):
    s = 0
    while (1 << s) < d:
        s += 1
    m = ((((1 << s) - d) << 32) // d + 1) & 0xFFFFFFFF
    return m, s


def fastdiv(n, d):
    m, s = magic(d)
    hi = (n.astype(np.uint64) * np.uint64(m)) >> np.uint64(32)
    return ((hi + n.astype(np.uint64)) >> np.uint64(s)).astype(np.uint64)


def test_fastdiv_matches_integer_division():
    rng = np.random.default_rng(0)
    divisors = list(range(1, 300)) + [511, 512, 513, 4095, 4096, 4097, 65535, 65536, 1 << 20, (1 << 30) + 7]
    for d in divisors:
        n = np.concatenate([np.arange(0, 5000, dtype=np.uint64),
                            rng.integers(0, 1 << 31, size=20000, dtype=np.uint64),
                            np.array([(1 << 31) - 1, (1 << 31) - 2, d * 12345 % (1 << 31)], dtype=np.uint64)])
        assert np.array_equal(fastdiv(n, d), n // np.uint64(d)), d
