"""The multiply-high division used to decode lattice node indices on the GPU
(q = (umulhi(n, m) + n) >> s, s = ceil(log2 d), m = floor(2^32 (2^s - d)/d) + 1)
is exact for every divisor and numerator the preconditioner uses."""
import numpy as np


def magic(d):
    s = 0
    while (1 << s) < d:
        s += 1
    return ((1 << 32) * ((1 << s) - d)) // d + 1, s


def fdiv(n, d):
    m, s = magic(d)
    n = np.asarray(n, np.uint64)
    hi = (n * np.uint64(m)) >> np.uint64(32)
    return ((hi + n) >> np.uint64(s)).astype(np.int64)


def test_fastdiv_exact():
    rng = np.random.default_rng(0)
    for R in list(range(2, 300)) + [512, 1000, 1024]:
        for d in (R, R * R):
            n_max = min(R ** 3, 1 << 31)
            n = np.concatenate([np.arange(min(n_max, 70000)), rng.integers(0, n_max, 20000),
                                np.arange(max(0, n_max - 5000), n_max)])
            q = fdiv(n, d)
            np.testing.assert_array_equal(q, n // d)
            m, _ = magic(d)
            assert m < (1 << 32)
