"""Pins for oracle O2's counters: arithmetic and memory against the paper.

The replays count element additions, base-case operations, peak extra memory
and total allocated memory.  These are compared with

* the arithmetic recurrences of Theorem 3 and Theorem 1, with a classical base
  case at the cut-off (W(n0) = 2n0^3 - n0^2, W_acc(n0) = 2n0^3, which is the
  paper's W(1) = 1, W_acc(1) = 2 at n0 = 1),
* their closed forms at full recursion (Table 10, Theorem 1), including the
  two printed forms that do not solve their recurrences (recorded below),
* Eq. (1), Eq. (2), Lemma 1 and the extra-memory bounds of Sections 5-6,
* the allocation recurrences of Theorem 3 (Table 10's column),
* Section 7.2's R_t(n) and extra memory of the blocked accumulation.
"""
import math
from fractions import Fraction

import pytest

from oracle.schedules import blocked_parts, fp64_chunk, replay, replay_shape


# ----------------------------------------------------------- recurrences
def W1(n, l):
    """Table 1 (and Tables 3, 5): 7 products, 15 additions."""
    return 2 * n**3 - n**2 if l == 0 else 7 * W1(n // 2, l - 1) + 15 * (n // 2) ** 2


def W1r(m, k, n, l):
    """Table 1 on an m x k by k x n product: 4 S, 4 T and 7 U additions."""
    if l == 0:
        return m * n * (2 * k - 1)
    h, kk, w = m // 2, k // 2, n // 2
    return 7 * W1r(h, kk, w, l - 1) + 4 * h * kk + 4 * kk * w + 7 * h * w


def W2(n, l):
    """Table 2: 5 accumulating calls, 2 plain calls, 14 additions."""
    if l == 0:
        return 2 * n**3
    return 5 * W2(n // 2, l - 1) + 2 * W1(n // 2, l - 1) + 14 * (n // 2) ** 2


def W2r(m, k, n, l):
    if l == 0:
        return 2 * m * n * k
    h, kk, w = m // 2, k // 2, n // 2
    return 5 * W2r(h, kk, w, l - 1) + 2 * W1r(h, kk, w, l - 1) + 4 * h * kk + 4 * kk * w + 6 * h * w


def W6(n, l):
    """Table 6: 4 AcLR calls, 3 IP calls, 17 additions."""
    if l == 0:
        return 2 * n**3
    return 4 * W6(n // 2, l - 1) + 3 * W1(n // 2, l - 1) + 17 * (n // 2) ** 2


def W7(n, l):
    """Table 7: 4 AccR, 1 IP, 2 OvR calls and 17 additions (the table has 17
    addition rows; Theorem 3 prints 16, which does not give its own closed form)."""
    if l == 0:
        return 2 * n**3
    return 4 * W7(n // 2, l - 1) + W1(n // 2, l - 1) + 2 * W1(n // 2, l - 1) + 17 * (n // 2) ** 2


def W9(n, l):
    """Table 9: 4 Acc, 1 T1, 1 AcLR, 1 AccR calls and 17 additions."""
    if l == 0:
        return 2 * n**3
    h = n // 2
    return 4 * W9(h, l - 1) + W1(h, l - 1) + W6(h, l - 1) + W7(h, l - 1) + 17 * h**2


def G(s, k, L, d=0):
    """Theorem 1's recurrence with the depth reading of Algorithm 2."""
    if d == L:
        return s * s * (2 * k - 1)
    h = s // 2
    K = min(h, k)
    lev = L - d
    return (3 * W1r(h, K, h, lev) + 3 * (k // K - 1) * W2r(h, K, h, lev)
            + G(h, k, L, d + 1))


# ----------------------------------------------------------- arithmetic
SQUARE = [(n, l) for n in (2, 4, 8, 16, 32, 64) for l in range(0, n.bit_length())]


@pytest.mark.parametrize("n,l", SQUARE)
def test_arithmetic_recurrences(n, l):
    want = {"t1": W1(n, l), "ip": W1(n, l), "ovr": W1(n, l), "hl": W2(n, l),
            "aclr": W6(n, l), "accr": W7(n, l), "acc": W9(n, l)}
    for s, w in want.items():
        r = replay_shape(s, n, n, n, levels=l, beta_nonzero=s in ("hl", "aclr", "accr", "acc"))
        assert r.ops == w, s


@pytest.mark.parametrize("shape,l", [((64, 32, 128), 2), ((128, 64, 32), 3),
                                     ((32, 64, 16), 2), ((16, 16, 64), 4)])
def test_rectangular_recurrences(shape, l):
    m, k, n = shape
    assert replay_shape("t1", m, k, n, levels=l).ops == W1r(m, k, n, l)
    assert replay_shape("hl", m, k, n, levels=l, beta_nonzero=True).ops == W2r(m, k, n, l)


@pytest.mark.parametrize("e", range(1, 7))
def test_closed_forms_full_recursion(e):
    n = 2**e
    f7, f4 = 7**e, 4**e                     # n^log2(7) and n^2, exactly
    assert replay_shape("t1", n, n, n, levels=e).ops == 6 * f7 - 5 * f4
    assert replay_shape("ip", n, n, n, levels=e).ops == 6 * f7 - 5 * f4
    assert replay_shape("ovr", n, n, n, levels=e).ops == 6 * f7 - 5 * f4
    assert replay_shape("hl", n, n, n, levels=e, beta_nonzero=True).ops == 6 * f7 - 4 * f4
    half = Fraction(f4 * e, 2)
    assert replay_shape("aclr", n, n, n, levels=e, beta_nonzero=True).ops == 6 * f7 - 4 * f4 + half
    assert replay_shape("accr", n, n, n, levels=e, beta_nonzero=True).ops == 6 * f7 - 4 * f4 + half
    acc = replay_shape("acc", n, n, n, levels=e, beta_nonzero=True).ops
    # The recurrence of Theorem 3 for Table 9 solves to this form ...
    assert acc == 6 * f7 - 4 * f4 + Fraction(f4, 8) * (e * e + 7 * e)
    # ... and not to the printed one (Table 10 / Theorem 3), except by accident.
    printed = 6 * f7 - 4 * f4 + Fraction(4, 3) * f4 * (e - Fraction(10, 3)) + Fraction(4, 9)
    if e > 1:
        assert acc != printed


@pytest.mark.parametrize("e", range(1, 7))
def test_ipmm_theorem1_closed_form(e):
    """G(n, n) = 7.2 n^log7 - 13 n^2 + 6.8 n, and the general
    G(n, k) = 7.2 k n^(log7 - 1) - 12 k n - n^2 + 34 k / 5, at full recursion."""
    n = 2**e
    for k in (n, 2 * n, 4 * n):
        got = replay_shape("ipmm", n, k, n, levels=e - 1).ops
        want = (Fraction(36, 5) * k * Fraction(7**e, 2**e) - 12 * k * n - n * n
                + Fraction(34 * k, 5))
        assert got == want, k
        if k == n:
            assert got == Fraction(36, 5) * 7**e - 13 * 4**e + Fraction(34, 5) * 2**e


@pytest.mark.parametrize("shape,L", [((64, 64, 64), 1), ((64, 64, 64), 3), ((64, 32, 64), 2),
                                     ((128, 256, 128), 2), ((64, 16, 64), 2)])
def test_ipmm_recurrence_with_cutoff(shape, L):
    m, k, n = shape
    assert replay_shape("ipmm", m, k, n, levels=L).ops == G(n, k, L)


# ----------------------------------------------------------------- memory
def sum_quarters(g, l):
    """sum_{i=1..l} g / 4^i, exact (Eq. (1) and Eq. (2) summed to depth l)."""
    return sum(Fraction(g, 4**i) for i in range(1, l + 1))


@pytest.mark.parametrize("shape,l", [((64, 64, 64), 1), ((64, 64, 64), 4), ((64, 32, 128), 3),
                                     ((128, 64, 32), 2), ((32, 128, 64), 3)])
def test_peak_eq1_eq2(shape, l):
    m, k, n = shape
    assert replay_shape("t1", m, k, n, levels=l).peak == sum_quarters(m * max(k, n) + k * n, l)
    assert replay_shape("hl", m, k, n, levels=l, beta_nonzero=True).peak == \
        sum_quarters(m * k + k * n + m * n, l)


@pytest.mark.parametrize("n,l", [(n, l) for n in (4, 16, 64) for l in range(1, n.bit_length())])
def test_peak_square_schedules(n, l):
    two = 2 * sum_quarters(n * n, l)            # two temporaries: (2/3) n^2 (1 - 4^-l)
    assert two == Fraction(2, 3) * n * n * (1 - Fraction(1, 4**l))
    assert replay_shape("t1", n, n, n, levels=l).peak == two
    assert replay_shape("aclr", n, n, n, levels=l, beta_nonzero=True).peak == two
    assert replay_shape("accr", n, n, n, levels=l, beta_nonzero=True).peak == two
    assert replay_shape("acc", n, n, n, levels=l, beta_nonzero=True).peak == two
    assert replay_shape("ovr", n, n, n, levels=l).peak == sum_quarters(n * n, l)
    assert replay_shape("hl", n, n, n, levels=l, beta_nonzero=True).peak == 3 * sum_quarters(n * n, l)
    assert replay_shape("ip", n, n, n, levels=l).peak == 0
    assert replay_shape("ipmm", n, n, n, levels=l - 1).peak == 0


@pytest.mark.parametrize("m,k,n", [(8, 16, 32), (32, 8, 16), (16, 16, 16)])
def test_lemma1_full_recursion(m, k, n):
    M = min(m, k, n)
    l = M.bit_length() - 1
    g = m * max(k, n) + k * n
    assert replay_shape("t1", m, k, n, levels=l).peak == Fraction(1, 3) * (1 - Fraction(1, M * M)) * g


def test_workload_temporary_bytes():
    """Peak extra bytes (8-byte entries) of the named workloads, from Eq. (1)
    and the two-temporary bound of Sections 5-6."""
    b = lambda r: int(r.peak) * 8
    assert b(replay_shape("t1", 512, 512, 512, levels=1)) == 1_048_576
    assert b(replay_shape("acc", 4096, 4096, 4096, levels=3, beta_nonzero=True)) == 88_080_384
    assert b(replay_shape("aclr", 4096, 4096, 4096, levels=3, beta_nonzero=True)) == 88_080_384
    assert b(replay_shape("hl", 4096, 4096, 4096, levels=3, beta_nonzero=True)) == 132_120_576
    for l, want in zip((1, 2, 3, 4), (201_326_592, 251_658_240, 264_241_152, 267_386_880)):
        assert b(replay_shape("t1", 8192, 4096, 8192, levels=l)) == want
    assert b(replay_shape("ipmm", 8192, 4096, 8192, levels=2)) == 0
    for l, want in zip((1, 2, 3), (1_073_741_824, 1_342_177_280, 1_409_286_144)):
        assert b(replay_shape("t1", 16384, 16384, 16384, levels=l)) == want


# ------------------------------------------------------------ allocations
def A1(n, l):
    return 0 if l == 0 else 2 * (n // 2) ** 2 + 7 * A1(n // 2, l - 1)


def A5(n, l):
    return 0 if l == 0 else (n // 2) ** 2 + 4 * A5(n // 2, l - 1)


def A6(n, l):
    return 0 if l == 0 else 2 * (n // 2) ** 2 + 4 * A6(n // 2, l - 1)


def A7(n, l):
    return 0 if l == 0 else 2 * (n // 2) ** 2 + 4 * A7(n // 2, l - 1) + 2 * A5(n // 2, l - 1)


def A2(n, l):
    return 0 if l == 0 else 3 * (n // 2) ** 2 + 5 * A2(n // 2, l - 1) + 2 * A1(n // 2, l - 1)


def A9(n, l):
    h = n // 2
    return 0 if l == 0 else 2 * h * h + 4 * A9(h, l - 1) + A1(h, l - 1) + A6(h, l - 1) + A7(h, l - 1)


@pytest.mark.parametrize("e", range(1, 7))
def test_allocation_totals(e):
    n = 2**e
    f = lambda s: replay_shape(s, n, n, n, levels=e,
                               beta_nonzero=s in ("hl", "aclr", "accr", "acc")).allocated
    assert f("t1") == A1(n, e) == Fraction(2, 3) * (7**e - 4**e)
    assert f("ovr") == A5(n, e) == Fraction(4**e * e, 4)
    assert f("aclr") == A6(n, e) == Fraction(4**e * e, 2)          # Table 10's form
    assert f("hl") == A2(n, e) == Fraction(2, 3) * 7**e + 5**e - Fraction(5, 3) * 4**e
    assert f("accr") == A7(n, e)
    assert f("acc") == A9(n, e)
    assert f("ip") == 0
    assert replay_shape("ipmm", n, n, n, levels=e - 1).allocated == 0


# ------------------------------------------------------ magnitude bound
@pytest.mark.parametrize("p", [65521, 1048573, 8388593])
def test_fp64_delayed_reduction_bound(p):
    kc = fp64_chunk(p)
    assert kc * (p - 1) ** 2 + (p - 1) < 2**53
    assert (kc + 1) * (p - 1) ** 2 + (p - 1) >= 2**53
    if kc > 4096:
        return
    # All entries p-1 reach the bound exactly in the first chunk.
    import numpy as np
    k = kc + 3
    A = np.full((2, k), p - 1, dtype=np.int64)
    B = np.full((k, 3), p - 1, dtype=np.int64)
    r = replay("classical", A, B, None, 1, 0, p, 0)
    assert r.max_partial == kc * (p - 1) ** 2
    assert np.all(r.C == k % p)


def test_chunk_values():
    assert fp64_chunk(65521) == 2_098_176
    assert fp64_chunk(1048573) == 8192
    assert fp64_chunk(8388593) == 128


# ------------------------------------------- Section 7.2: blocked accumulation
@pytest.mark.parametrize("t", [1, 2, 3, 4])
@pytest.mark.parametrize("e", range(1, 5))
def test_blocked_rt_closed_form(t, e):
    """R_t(n) = t^2 * t * W_acc(n/t) = 6 t^(3 - log7) n^log7 - 4 t n^2 at full
    recursion of Table 2 on the (n/t)-blocks; with n = t 2^e,
    t^(3 - log7) n^log7 = t^3 7^e exactly."""
    n = t * 2**e
    got = replay_shape("blocked", n, n, n, levels=e, beta_nonzero=True, blocks=t).ops
    assert got == 6 * t**3 * 7**e - 4 * t * n * n
    log7 = math.log2(7)
    assert got == pytest.approx(6 * t ** (3 - log7) * n ** log7 - 4 * t * n * n, rel=1e-12)
    assert got == t**3 * W2(n // t, e)


def test_blocked_rt_constants():
    """The leading constants quoted for t = 2 and t = 3 (6.857 and 7.414)."""
    log7 = math.log2(7)
    assert round(6 * 2 ** (3 - log7), 3) == 6.857
    assert round(6 * 3 ** (3 - log7), 3) == 7.414


@pytest.mark.parametrize("t,n", [(2, 64), (3, 48), (4, 64), (3, 96)])
def test_blocked_classical_base_keeps_cubic_count(t, n):
    """With no Winograd level the blocks are classical accumulations: the
    t^3 calls of 2 (n/t)^3 operations give the classical 2 n^3."""
    assert replay_shape("blocked", n, n, n, levels=0, beta_nonzero=True, blocks=t).ops == 2 * n**3
    assert replay_shape("blocked_acc", n, n, n, levels=0, beta_nonzero=True, blocks=t).ops == 2 * n**3


@pytest.mark.parametrize("t,e", [(2, 1), (2, 3), (3, 2), (3, 4), (4, 3)])
def test_blocked_acc_base_count(t, e):
    """Table 9 as the base: t^3 calls of Table 9 on (n/t)-blocks.  Table 9's
    own rows give 6 m^log7 - 4 m^2 + m^2 (log^2 m + 7 log m) / 8 per call; the
    extra term printed in Section 7.2 for this variant,
    t^(2 - log3) n^log6 - t n^2 (t^3 (m^log6 - m^2)), is a different function
    of m, like the printed Table 9 form checked above."""
    n = t * 2**e
    got = replay_shape("blocked_acc", n, n, n, levels=e, beta_nonzero=True, blocks=t).ops
    assert got == t**3 * W9(n // t, e)
    f7, f4 = 7**e, 4**e
    own = t**3 * (6 * f7 - 4 * f4 + Fraction(f4, 8) * (e * e + 7 * e))
    assert got == own
    printed = t**3 * (6 * f7 - 4 * f4) + t**3 * (6**e - f4)
    assert got != printed


@pytest.mark.parametrize("t", [2, 3, 4])
@pytest.mark.parametrize("l", [1, 2, 3])
def test_blocked_extra_memory(t, l):
    """One call's temporaries at a time: Table 2 on an (n/t)-block needs
    3 (n/t)^2 (1 - 4^-l) / 3 = (n/t)^2 (1 - 4^-l), below the one chunk of
    (n/t)^2 (n^2/4 for t = 2, n^2/9 for t = 3); Table 9 needs two thirds of
    that, below 2 n^2 / (3 t^2)."""
    n = t * 32
    b = n // t
    hl = replay_shape("blocked", n, n, n, levels=l, beta_nonzero=True, blocks=t).peak
    assert hl == 3 * sum_quarters(b * b, l) == b * b * (1 - Fraction(1, 4**l))
    assert hl < Fraction(n * n, t * t)
    acc = replay_shape("blocked_acc", n, n, n, levels=l, beta_nonzero=True, blocks=t).peak
    assert acc == 2 * sum_quarters(b * b, l)
    assert acc < Fraction(2 * n * n, 3 * t * t)
    # the unblocked schedules need t^2 times more
    assert replay_shape("hl", n, n, n, levels=l, beta_nonzero=True).peak == t * t * hl
    assert replay_shape("acc", n, n, n, levels=l, beta_nonzero=True).peak == t * t * acc


def test_blocked_parts():
    """The split of one dimension: n/t when t divides it, else ceil(n/t)
    rounded up to a multiple of 2^L."""
    assert blocked_parts(4096, 2, 3) == [2048, 2048]
    assert blocked_parts(3000, 2, 3) == [1500, 1500]
    assert blocked_parts(4096, 3, 3) == [1368, 1368, 1360]
    assert blocked_parts(10, 3, 2) == [4, 4, 2]
    assert blocked_parts(5, 3, 3) == [5]
    assert blocked_parts(0, 3, 1) == []
    for d in range(1, 70):
        for t in (1, 2, 3, 5):
            for L in (0, 1, 3):
                parts = blocked_parts(d, t, L)
                assert sum(parts) == d and 1 <= len(parts) <= t and min(parts) > 0
                assert all(x % 2**L == 0 for x in parts[:-1]) or d % t == 0


def test_blocked_workload_bytes():
    """Extra bytes of the accumulating 4096^3 product with three levels: t = 2
    and t = 3 blocks over Table 2 or Table 9, against the unblocked Table 9."""
    b = lambda s, t: int(replay_shape(s, 4096, 4096, 4096, levels=3, beta_nonzero=True,
                                      blocks=t).peak) * 8
    assert b("blocked", 2) == 3 * (1024**2 + 512**2 + 256**2) * 8 == 33_030_144
    assert b("blocked_acc", 2) == 2 * (1024**2 + 512**2 + 256**2) * 8 == 22_020_096
    # parts 1368, 1368, 1360: the temporaries of the largest block
    assert b("blocked", 3) == 3 * (684**2 + 342**2 + 171**2) * 8 == 14_737_464
    assert b("acc", 2) == 88_080_384


# ------------------------------ the rectangular overwrite family (Section 5.3)
def W8r(m, k, n, l):
    """Table 8: five accumulating calls, two Table 1 calls, 16 additions
    (8 on C-sized blocks, 4 on S blocks, 4 on T blocks)."""
    if l == 0:
        return 2 * m * n * k
    h, kk, w = m // 2, k // 2, n // 2
    return (5 * W8r(h, kk, w, l - 1) + 2 * W1r(h, kk, w, l - 1) + 4 * h * kk + 4 * kk * w
            + 8 * h * w)


def E1r(m, k, n, l):
    """Eq. (1) summed to depth l."""
    if l == 0:
        return 0
    h, kk, w = m // 2, k // 2, n // 2
    return h * max(kk, w) + kk * w + E1r(h, kk, w, l - 1)


def E8r(m, k, n, l):
    """Section 5.3's extra memory of Table 8: X = max(m/2, k/2) n/2, Y = m/2 k/2,
    plus the larger of its callees (Table 8 or Table 1) one level down."""
    if l == 0:
        return 0
    h, kk, w = m // 2, k // 2, n // 2
    return max(h, kk) * w + h * kk + max(E8r(h, kk, w, l - 1), E1r(h, kk, w, l - 1))


@pytest.mark.parametrize("n,l", [(n, l) for n in (2, 8, 32) for l in range(0, n.bit_length())])
def test_ovl_arithmetic_and_memory(n, l):
    """Table 4 performs Table 1's arithmetic (7 products, 15 additions) with
    one (n/2)^2 temporary per level: M(n) = (n/2)^2 + M(n/2) -> n^2/3."""
    r = replay_shape("ovl", n, n, n, levels=l)
    assert r.ops == W1(n, l)
    assert r.peak == sum_quarters(n * n, l)


@pytest.mark.parametrize("e", range(1, 7))
def test_ovl_closed_forms(e):
    """At full recursion: 6n^log7 - 5n^2 operations, at most n^2/3 extra
    memory, and A(n) = (n/2)^2 + 4A(n/2) = n^2 log2(n) / 4 allocations."""
    n = 2**e
    r = replay_shape("ovl", n, n, n, levels=e)
    assert r.ops == 6 * 7**e - 5 * 4**e
    assert r.peak == Fraction(n * n, 3) * (1 - Fraction(1, 4**e)) < Fraction(n * n, 3)
    assert r.allocated == Fraction(n * n * e, 4)


@pytest.mark.parametrize("shape,l", [((32, 32, 32), 3), ((64, 32, 128), 2), ((128, 64, 32), 3),
                                     ((32, 128, 64), 2), ((16, 64, 32), 4), ((64, 16, 16), 2)])
def test_acr_arithmetic_and_memory(shape, l):
    m, k, n = shape
    r = replay_shape("acr", m, k, n, levels=l, beta_nonzero=True)
    assert r.ops == W8r(m, k, n, l)
    assert r.peak == E8r(m, k, n, l)


@pytest.mark.parametrize("e", range(1, 7))
def test_acr_square_closed_forms(e):
    """Square Table 8 at full recursion: W(n) = 5W(n/2) + 2W1(n/2) + 16(n/2)^2
    gives 6n^log7 + 2n^log5 - 6n^2; its extra memory stays within 2n^2/3."""
    n = 2**e
    r = replay_shape("acr", n, n, n, levels=e, beta_nonzero=True)
    assert r.ops == 6 * 7**e + 2 * 5**e - 6 * 4**e
    assert r.peak <= Fraction(2 * n * n, 3)


@pytest.mark.parametrize("shape", [(16, 32, 64), (32, 16, 64), (64, 32, 16), (64, 64, 16),
                                   (16, 64, 32), (32, 64, 16)])
def test_acr_rectangular_memory_bounds(shape):
    """Section 5.3: if m < k < n or k < m < n Table 8 needs less than Table 1;
    otherwise it needs less than (max(m, k) n + m k) / 3."""
    m, k, n = shape
    l = min(shape).bit_length() - 1
    e8 = replay_shape("acr", m, k, n, levels=l, beta_nonzero=True).peak
    if (m < k < n) or (k < m < n):
        assert e8 < replay_shape("t1", m, k, n, levels=l).peak
    else:
        assert e8 < Fraction(max(m, k) * n + m * k, 3)


@pytest.mark.parametrize("shape,l", [((64, 128, 32), 2), ((96, 64, 32), 1), ((32, 96, 32), 3),
                                     ((64, 32, 32), 2), ((32, 32, 32), 5), ((128, 256, 64), 6)])
def test_ip0vmm_arithmetic_and_no_memory(shape, l):
    """Algorithm 1 allocates nothing; its operations are those of its calls:
    m0 Table 1/4 products and m0 (k0 - 1) Table 2 accumulations of n x n
    squares, or (m0 = 1) one Table 3 product and k0 - 1 Table 6 ones."""
    m, k, n = shape
    r = replay_shape("ip0vmm", m, k, n, levels=l)
    assert r.peak == 0 and r.allocated == 0
    m0, k0 = m // n, k // n
    if m0 == 1:
        assert r.ops == W1(n, l) + (k0 - 1) * W6(n, l)
    else:
        assert r.ops == m0 * W1(n, l) + m0 * (k0 - 1) * W2(n, l)
    if l == n.bit_length() - 1 and m0 > 1:                      # full recursion
        assert r.ops == m0 * (6 * 7**l - 5 * 4**l) + m0 * (k0 - 1) * (6 * 7**l - 4 * 4**l)


def G9(s, k, L, d=0):
    """Theorem 1's recurrence with Table 9 for the accumulating chunks."""
    if d == L:
        return s * s * (2 * k - 1)
    h = s // 2
    K = min(h, k)
    lev = L - d
    return 3 * W1r(h, K, h, lev) + 3 * (k // K - 1) * W9(h, lev) + G9(h, k, L, d + 1)


@pytest.mark.parametrize("shape,L", [((64, 64, 64), 1), ((64, 64, 64), 3), ((64, 32, 64), 2),
                                     ((128, 256, 128), 2), ((32, 128, 32), 3)])
def test_ipmm_acc_recurrence(shape, L):
    """Algorithm 2 with Table 9 accumulations: Theorem 1's recurrence with
    W9 in place of W2, no extra memory; never cheaper than with Table 2."""
    m, k, n = shape
    r = replay_shape("ipmm_acc", m, k, n, levels=L)
    assert r.ops == G9(n, k, L)
    assert r.peak == 0
    assert r.ops >= replay_shape("ipmm", m, k, n, levels=L).ops


@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_blocked_makes_t_cubed_calls(t):
    """Section 7.2: with C in four blocks the product takes 8 calls of the
    base schedule; in general t^2 blocks of t calls each."""
    n = 8 * t
    r = replay_shape("blocked", n, n, n, levels=0, beta_nonzero=True, blocks=t)
    assert r.calls["hl"] == t**3 and r.calls["blocked"] == 1
    r = replay_shape("blocked_acc", n, n, n, levels=0, beta_nonzero=True, blocks=t)
    assert r.calls["acc"] == t**3
