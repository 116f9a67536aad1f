"""Oracle O4: a product over Z/pZ rebuilt from signed 8-bit digit products.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An exact integer product can be assembled from products of small digits: a
residue x in [0, p) is first centred, c = x - p when x > (p-1)/2, so that
|c| <= (p-1)/2, and then written in balanced base 256,

    c = d0 + 256*d1 + 65536*d2,   every digit d_i in [-128, 127].

Three digits reach every centred residue of a prime below 16,711,423
(127*(1 + 2**8 + 2**16) = 8,355,711 on the positive side).  Then

    A*B = sum_{i,j} 2**(8*(i+j)) * (A_i @ B_j),

and each digit product A_i @ B_j has entries of magnitude at most k*2**14,
so the products of one weight w = i+j (at most three of them) sum to less
than 3*k*2**14 -- below 2**31 for k up to 2**15.  Reducing each weight class
mod p and recombining with the residues 2**(8w) mod p gives the value of
oracle O1.  This module writes that out plainly with int64 numpy arrays.
"""
import numpy as np

NDIGITS = 3


def centre(x, p):
    """Centred representative of canonical residues x in [0, p)."""
    x = np.asarray(x, dtype=np.int64)
    return np.where(x > (p - 1) // 2, x - p, x)


def split(x, p, ndigits=NDIGITS):
    """Balanced base-256 digits (list of int64 arrays) of the centred x."""
    c = centre(x, p)
    digits = []
    for _ in range(ndigits):
        d = ((c + 128) % 256) - 128
        digits.append(d)
        c = (c - d) // 256
    if np.any(c != 0):
        raise ValueError("residue does not fit in %d balanced digits" % ndigits)
    return digits


def join(digits, p):
    """Canonical residue from balanced digits (inverse of split)."""
    acc = np.zeros_like(digits[0])
    for i, d in enumerate(digits):
        acc = acc + d * (256 ** i)
    return acc % p


def matmul_mod_p(A, B, p, ndigits=NDIGITS):
    """(A @ B) mod p assembled from digit products, plus the largest magnitude
    reached by any weight-class accumulation (to compare with 2**31)."""
    Ad = split(A, p, ndigits)
    Bd = split(B, p, ndigits)
    m, n = Ad[0].shape[0], Bd[0].shape[1]
    out = np.zeros((m, n), dtype=np.int64)
    worst = 0
    for w in range(2 * ndigits - 1):
        acc = np.zeros((m, n), dtype=np.int64)
        for i in range(ndigits):
            j = w - i
            if 0 <= j < ndigits:
                acc = acc + Ad[i] @ Bd[j]
        if acc.size:
            worst = max(worst, int(np.abs(acc).max()))
        out = (out + (pow(256, w, p) * (acc % p)) % p) % p
    return out, worst
