"""The 32-bit division-by-constant formula used by the elementwise kernels'
index math: with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
floor(x / d) == (floor(x * m / 2^32) + x) >> l for every 32-bit x.
Checked against integer division (a wrong quotient would index out of
bounds on the device)."""
import numpy as np


def fastdiv(x, d):
    l = 0
    while (1 << l) < d:
        l += 1
    m = ((1 << 32) * ((1 << l) - d)) // d + 1
    assert 0 < m < (1 << 32) or d == 1
    return (((x * m) >> 32) + x) >> l


def test_fastdiv_exact():
    rng = np.random.default_rng(0)
    ds = list(range(1, 2050)) + [4095, 4096, 4097, 8191, 8192, 65535, 65536, 1 << 20,
                                 (1 << 31) - 1, 1 << 31, (1 << 32) - 1]
    xs_fixed = [0, 1, 2, (1 << 31) - 1, 1 << 31, (1 << 32) - 1, (1 << 32) - 2]
    for d in ds:
        xs = xs_fixed + [int(v) for v in rng.integers(0, 1 << 32, size=200)]
        xs += [d * q + r for q in (1, 2, 1000) for r in (-1, 0, 1) if 0 <= d * q + r < (1 << 32)]
        for x in xs:
            assert fastdiv(x, d) == x // d, (x, d)
