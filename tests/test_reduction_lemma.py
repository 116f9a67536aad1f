"""The binary64 reduction lemma the GPU kernels rely on (host check).

For an integer x with |x| < 2^53 and an odd modulus 2 < p < 2^24, with
pinv = fl(1/p) and q = floor(fl(x * pinv)), the remainder r = x - q*p lies in
[-p, 2p), so a single correction step (r += p if r < 0; r -= p if r >= p)
yields the canonical residue.  x - q*p is an exact small integer, so a fused
multiply-add computes it without rounding.  The check below computes q with
IEEE binary64 arithmetic (numpy) and r with Python integers.
"""
import numpy as np
import pytest

from paper_0707_2347_amd import inputs


def _check(xs, p):
    pinv = np.float64(1.0) / np.float64(p)
    for x in xs:
        q = int(np.floor(np.float64(x) * pinv))
        r = x - q * p
        assert -p <= r < 2 * p, (x, p, r)
        r = r + p if r < 0 else (r - p if r >= p else r)
        assert r == x % p


@pytest.mark.parametrize("p", inputs.PRIMES + (3, 65537, 16777213))
def test_one_correction_suffices(p):
    top = 2**53 - 1
    xs = [0, 1, -1, p, -p, top, -top, top - 1, -(top - 1)]
    for t in (1, 2, 3, 7, 1000, 2**20, 2**30, top // p - 1, top // p):
        for e in (-2, -1, 0, 1, 2):
            for s in (1, -1):
                x = s * (t * p + e)
                if abs(x) <= top:
                    xs.append(x)
    rng = np.random.default_rng(p)
    xs += [int(v) for v in rng.integers(-top, top, size=20000)]
    _check(xs, p)
