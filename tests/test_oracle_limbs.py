"""Pins for oracle O4: balanced base-256 digits of centred residues.

* split then join is the identity on every residue of 65521 and on random
  residues of the larger primes; every digit lies in [-128, 127];
* the digit-product assembly equals oracle O1 (pinned by brute force);
* each weight class of digit products stays below the int32 range at the
  largest inner dimension used (3 * k * 2**14 < 2**31 for k <= 2**15).
"""
import numpy as np
import pytest

from oracle import limbs, ref
from paper_0707_2347_amd import inputs


def test_roundtrip_every_residue_small_prime():
    p = 65521
    x = np.arange(p, dtype=np.int64)
    d = limbs.split(x, p)
    assert all(int(t.min()) >= -128 and int(t.max()) <= 127 for t in d)
    assert np.array_equal(limbs.join(d, p), x)
    c = limbs.centre(x, p)
    assert int(np.abs(c).max()) == (p - 1) // 2


@pytest.mark.parametrize("p", [1048573, 8388593])
def test_roundtrip_random_and_edges(p):
    rng = np.random.default_rng(p)
    x = np.concatenate([rng.integers(0, p, size=200000),
                        np.array([0, 1, p - 1, (p - 1) // 2, (p + 1) // 2, p - 2])])
    d = limbs.split(x, p)
    assert all(int(t.min()) >= -128 and int(t.max()) <= 127 for t in d)
    assert np.array_equal(limbs.join(d, p), x % p)


def test_three_digits_cover_the_stated_range():
    """127*(1+2^8+2^16) = 8,355,711 is the largest positive value, so every
    centred residue of a prime up to 16,711,423 has three digits."""
    top = 127 * (1 + 2**8 + 2**16)
    assert top == 8_355_711
    p = 2 * top + 1                      # 16,711,423: (p-1)/2 == top
    d = limbs.split(np.array([top, p - top, 0, 1, p - 1], dtype=np.int64), p)
    assert np.array_equal(limbs.join(d, p), np.array([top, p - top, 0, 1, p - 1]) % p)
    with pytest.raises(ValueError):
        limbs.split(np.array([top + 1], dtype=np.int64), 2 * top + 5)


@pytest.mark.parametrize("p", inputs.PRIMES)
@pytest.mark.parametrize("shape", [(17, 33, 9), (64, 64, 64), (5, 300, 7)])
def test_digit_product_equals_plain_product(p, shape):
    m, k, n = shape
    A, B, _ = inputs.uniform(21, m, k, n, p)
    got, worst = limbs.matmul_mod_p(A, B, p)
    assert np.array_equal(got, ref.matmul_mod_p(A, B, None, 1, 0, p))
    assert worst <= 3 * k * 2**14


def test_weight_class_bound_is_reached_and_safe():
    """Digits all -128 give digit products of exactly k * 2^14 per pair; with
    three pairs in the middle weight, 3 * k * 2^14, below 2^31 for k = 2^15."""
    k = 2**15
    assert 3 * k * 2**14 < 2**31
    p = 16_843_009 + 2                   # room for the all--128 centred value
    c = -128 * (1 + 256 + 65536)
    x = np.full((1, 64), c % p, dtype=np.int64)
    y = np.full((64, 1), c % p, dtype=np.int64)
    got, worst = limbs.matmul_mod_p(x, y, p)
    assert worst == 3 * 64 * 2**14
    assert int(got[0, 0]) == (64 * c * c) % p
