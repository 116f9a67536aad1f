"""Pins for oracle O2, the per-schedule replays of Winograd's algorithm.

* The value: each schedule must equal oracle O1 (itself pinned by brute force),
  with garbage injected into every temporary and every operand an overwriting
  callee may destroy -- a row reading a dead location then fails.
* A planted mistake (two rows of Table 3 swapped) is caught by garbage mode.
* Inputs: read-only schedules leave A and B unchanged; Table 5 and Table 7
  leave A unchanged.
* The final state of overwritten inputs after one level is written out from
  Section 2's definitions of S, T, P and U, independently of the replay.
"""
import zlib

import numpy as np
import pytest

from oracle import ref
from oracle.schedules import Winograd, quads, replay
from paper_0707_2347_amd import inputs

P = 65521


def o1(A, B, C, a, b, p):
    return ref.matmul_mod_p(A, B, C, a, b, p)


CASES = [
    # schedule, shape, levels, accumulates
    ("t1", (64, 64, 64), 1, False), ("t1", (64, 64, 64), 3, False),
    ("t1", (64, 32, 128), 2, False), ("t1", (128, 64, 32), 2, False),
    ("t1", (37, 50, 29), 2, False), ("t1", (33, 33, 33), 3, False),
    ("hl", (64, 64, 64), 2, True), ("hl", (32, 64, 16), 2, True),
    ("hl", (45, 22, 31), 1, True),
    ("acc", (64, 64, 64), 1, True), ("acc", (64, 64, 64), 3, True),
    ("acc", (41, 41, 41), 2, True),
    ("ip", (64, 64, 64), 1, False), ("ip", (64, 64, 64), 4, False),
    ("ovr", (32, 32, 32), 3, False),
    ("aclr", (64, 64, 64), 2, True), ("aclr", (16, 16, 16), 4, True),
    ("accr", (32, 32, 32), 3, True),
    ("ipmm", (64, 64, 64), 1, False), ("ipmm", (64, 64, 64), 3, False),
    ("ipmm", (64, 32, 64), 2, False), ("ipmm", (64, 128, 64), 2, False),
    ("ipmm", (64, 16, 64), 2, False),
    ("classical", (13, 17, 19), 0, True),
]


@pytest.mark.parametrize("p", [P, 8388593])
@pytest.mark.parametrize("schedule,shape,levels,accumulates", CASES)
def test_schedule_value_with_garbage(schedule, shape, levels, accumulates, p):
    m, k, n = shape
    A, B, C = inputs.uniform(zlib.crc32(repr((schedule, shape, levels)).encode()), m, k, n, p, True)
    for seed, (alpha, beta) in enumerate([(1, 1), (3, p - 2), (p - 1, 5), (7, 0)]):
        if not accumulates:
            beta = 0
        r = replay(schedule, A, B, C, alpha, beta, p, levels, garbage_seed=seed)
        assert np.array_equal(r.C, o1(A, B, C, alpha, beta, p)), (alpha, beta)


@pytest.mark.parametrize("schedule", ["t1", "hl", "acc", "ipmm", "classical", "ovr", "accr"])
def test_inputs_left_intact(schedule):
    n = 32
    A, B, C = inputs.uniform(5, n, n, n, P, True)
    beta = 3 if schedule in ("hl", "acc", "accr", "classical") else 0
    r = replay(schedule, A, B, C, 2, beta, P, 2, garbage_seed=1)
    assert np.array_equal(r.A, A)
    if schedule not in ("ovr", "accr"):
        assert np.array_equal(r.B, B)


def test_acc_with_beta_zero_ignores_garbage_c():
    n = 32
    A, B, _ = inputs.uniform(6, n, n, n, P)
    r = replay("acc", A, B, None, 5, 0, P, 2, garbage_seed=3)
    assert np.array_equal(r.C, o1(A, B, None, 5, 0, P))


def _sp(A, B, C, a, b, p):
    """Section 2's blocks, formed directly from their definitions."""
    A11, A12, A21, A22 = quads(A)
    B11, B12, B21, B22 = quads(B)
    C11, C12, C21, C22 = quads(C)
    S1 = (A21 + A22) % p
    S2 = (S1 - A11) % p
    S4 = (A12 - S2) % p
    T1 = (B12 - B11) % p
    T2 = (B22 - T1) % p
    T3 = (B22 - B12) % p
    T4 = (T2 - B21) % p
    prod = lambda X, Y: o1(X, Y, None, a, 0, p)
    P = {1: prod(A11, B11), 2: prod(A12, B21), 3: prod(S4, B22), 4: prod(A22, T4),
         5: prod(S1, T1), 6: prod(S2, T2)}
    return dict(A21=A21, A22=A22, B11=B11, B21=B21, B22=B22, A11=A11, A12=A12,
                S2=S2, S4=S4, T2=T2, T3=T3, P=P, C12=C12)


def _blocks(M):
    M11, M12, M21, M22 = quads(M)
    return [M11, M12, M21, M22]


def test_ip_final_inputs_one_level():
    """Table 3 at one level ends with A = [[P5, P3], [P4, S4]] and
    B = [[T2, T3], [B21, B22]]."""
    n, a = 32, 7
    A, B, _ = inputs.uniform(11, n, n, n, P)
    r = replay("ip", A, B, None, a, 0, P, 1)
    d = _sp(A, B, np.zeros((n, n), np.int64), a, 0, P)
    Pp = d["P"]
    for got, want in zip(_blocks(r.A), [Pp[5], Pp[3], Pp[4], d["S4"]]):
        assert np.array_equal(got, want)
    for got, want in zip(_blocks(r.B), [d["T2"], d["T3"], d["B21"], d["B22"]]):
        assert np.array_equal(got, want)


def test_aclr_final_inputs_one_level():
    """Table 6 at one level ends with A = [[A11, A12], [S2, S4]] and
    B = [[B11, T2], [B21, B22]]."""
    n, a, b = 32, 5, 9
    A, B, C = inputs.uniform(12, n, n, n, P, True)
    r = replay("aclr", A, B, C, a, b, P, 1)
    d = _sp(A, B, C, a, b, P)
    for got, want in zip(_blocks(r.A), [d["A11"], d["A12"], d["S2"], d["S4"]]):
        assert np.array_equal(got, want)
    for got, want in zip(_blocks(r.B), [d["B11"], d["T2"], d["B21"], d["B22"]]):
        assert np.array_equal(got, want)


def test_ovr_final_inputs_one_level():
    """Table 5 at one level ends with B = [[S4, P2], [B21, B22]]."""
    n, a = 32, 3
    A, B, _ = inputs.uniform(13, n, n, n, P)
    r = replay("ovr", A, B, None, a, 0, P, 1)
    d = _sp(A, B, np.zeros((n, n), np.int64), a, 0, P)
    for got, want in zip(_blocks(r.B), [d["S4"], d["P"][2], d["B21"], d["B22"]]):
        assert np.array_equal(got, want)
    assert np.array_equal(r.A, A)


def test_accr_final_inputs_one_level():
    """Table 7 at one level ends with B = [[B11, T2], [U4 + b*C12, B22]]
    where U4 = P1 + P6 + P5."""
    n, a, b = 32, 4, 6
    A, B, C = inputs.uniform(14, n, n, n, P, True)
    r = replay("accr", A, B, C, a, b, P, 1)
    d = _sp(A, B, C, a, b, P)
    Pp = d["P"]
    u4 = (Pp[1] + Pp[6] + Pp[5] + b * d["C12"]) % P
    for got, want in zip(_blocks(r.B), [d["B11"], d["T2"], u4, d["B22"]]):
        assert np.array_equal(got, want)


def test_overwrite_final_state_is_deterministic():
    n = 64
    A, B, C = inputs.uniform(15, n, n, n, P, True)
    for s in ("ip", "aclr"):
        r1 = replay(s, A, B, C, 2, 3 if s == "aclr" else 0, P, 3)
        r2 = replay(s, A, B, C, 2, 3 if s == "aclr" else 0, P, 3)
        assert np.array_equal(r1.A, r2.A) and np.array_equal(r1.B, r2.B)


class _SwappedIP(Winograd):
    """Table 3 with rows 6 and 7 exchanged: S2 = S1 - A11 is formed after the
    product P1 has been allowed to destroy A11."""

    def ip(self, A, B, C, a, lev):
        if lev == 0:
            self.leaf(A, B, C, a, 0, False)
            self.destroy(A, B)
            return
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        self.sub(C11, A11, A21)
        self.add(A21, A21, A22)
        self.sub(C22, B12, B11)
        self.sub(B12, B22, B12)
        self.ip(C11, B12, C21, a, lev - 1)
        self.ip(A11, B11, C11, a, lev - 1)        # row 7 moved up
        self.sub(C12, A21, A11)                   # row 6 now reads a dead A11
        self.sub(B11, B22, C22)
        self.ip(A21, C22, A11, a, lev - 1)
        self.sub(C22, B11, B21)
        self.ip(A22, C22, A21, a, lev - 1)
        self.sub(A22, A12, C12)
        self.ip(C12, B11, C22, a, lev - 1)
        self.add(C22, C11, C22)
        self.ip(A12, B21, C12, a, lev - 1)
        self.add(C11, C11, C12)
        self.add(C12, C22, A11)
        self.add(C22, C22, C21)
        self.sub(C21, C22, A21)
        self.add(C22, C22, A11)
        self.ip(A22, B22, A12, a, lev - 1)
        self.add(C12, C12, A12)
        self.destroy(A, B)


def test_garbage_mode_catches_a_planted_mistake():
    n = 32
    A, B, _ = inputs.uniform(16, n, n, n, P)
    want = o1(A, B, None, 1, 0, P)
    w = _SwappedIP(P, garbage_seed=0)
    Ac, Bc, C = A.copy(), B.copy(), np.zeros((n, n), np.int64)
    w.ip(Ac, Bc, C, 1, 1)
    assert not np.array_equal(C, want)
    # The unmodified schedule passes under the same garbage.
    w = Winograd(P, garbage_seed=0)
    Ac, Bc, C = A.copy(), B.copy(), np.zeros((n, n), np.int64)
    w.ip(Ac, Bc, C, 1, 1)
    assert np.array_equal(C, want)


def test_rejects_unsupported_shapes():
    A, B, C = inputs.uniform(17, 12, 12, 12, P, True)
    with pytest.raises(ValueError):
        replay("ip", A, B, None, 1, 0, P, 3)        # 12 not divisible by 8
    with pytest.raises(ValueError):
        replay("t1", A, B, C, 1, 1, P, 1)           # t1 has no beta
    A2, B2, _ = inputs.uniform(18, 12, 8, 16, P)
    with pytest.raises(ValueError):
        replay("aclr", A2, B2, np.zeros((12, 16), np.int64), 1, 1, P, 1)


# ------------------------------------------- Section 7.2: blocked accumulation
BLOCKED = [
    # schedule, shape, levels, t
    ("blocked", (64, 64, 64), 2, 2), ("blocked", (96, 96, 96), 1, 3),
    ("blocked", (64, 32, 128), 2, 2), ("blocked", (37, 50, 29), 1, 3),
    ("blocked", (100, 100, 100), 2, 3), ("blocked", (33, 17, 65), 2, 4),
    ("blocked", (32, 32, 32), 2, 1), ("blocked", (5, 70, 3), 1, 3),
    ("blocked_acc", (64, 64, 64), 2, 2), ("blocked_acc", (96, 96, 96), 2, 3),
    ("blocked_acc", (90, 90, 90), 2, 3), ("blocked_acc", (64, 64, 64), 1, 4),
]


@pytest.mark.parametrize("p", [P, 8388593])
@pytest.mark.parametrize("schedule,shape,levels,t", BLOCKED)
def test_blocked_value_with_garbage(schedule, shape, levels, t, p):
    m, k, n = shape
    A, B, C = inputs.uniform(zlib.crc32(repr((schedule, shape, t)).encode()), m, k, n, p, True)
    for seed, (alpha, beta) in enumerate([(1, 1), (3, p - 2), (p - 1, 5), (7, 0)]):
        r = replay(schedule, A, B, C, alpha, beta, p, levels, garbage_seed=seed, blocks=t)
        assert np.array_equal(r.C, o1(A, B, C, alpha, beta, p)), (alpha, beta)
        assert np.array_equal(r.A, A) and np.array_equal(r.B, B)


def test_blocked_empty_inner_dimension_scales_c():
    A, B, C = inputs.uniform(21, 9, 0, 7, P, True)
    r = replay("blocked", A, B, C, 4, 6, P, 1, blocks=3)
    assert np.array_equal(r.C, 6 * C % P)


class _BetaEveryCall(Winograd):
    """A planted mistake: every inner block product applies beta again."""

    def blocked(self, core, A, B, C, a, b, t, L):
        from oracle.schedules import blocked_parts
        m, k = A.shape
        n = B.shape[1]
        cut = lambda d: np.cumsum([0] + blocked_parts(d, t, L))
        ri, kl, cj = cut(m), cut(k), cut(n)
        for i in range(len(ri) - 1):
            for j in range(len(cj) - 1):
                for l in range(len(kl) - 1):
                    core(A[ri[i]:ri[i + 1], kl[l]:kl[l + 1]], B[kl[l]:kl[l + 1], cj[j]:cj[j + 1]],
                         C[ri[i]:ri[i + 1], cj[j]:cj[j + 1]], a, b, L)


def test_blocked_planted_mistake_is_caught():
    n = 32
    A, B, C = inputs.uniform(22, n, n, n, P, True)
    want = o1(A, B, C, 1, 3, P)
    w = _BetaEveryCall(P, garbage_seed=0)
    Cw = C.copy()
    w.blocked(w.hl, A.copy(), B.copy(), Cw, 1, 3, 2, 1)
    assert not np.array_equal(Cw, want)
    w = Winograd(P, garbage_seed=0)
    Cw = C.copy()
    w.blocked(w.hl, A.copy(), B.copy(), Cw, 1, 3, 2, 1)
    assert np.array_equal(Cw, want)


def test_blocked_rejects_bad_blocks():
    A, B, C = inputs.uniform(23, 12, 12, 12, P, True)
    with pytest.raises(ValueError):
        replay("blocked", A, B, C, 1, 1, P, 1, blocks=0)
    with pytest.raises(ValueError):
        replay("blocked_acc", A, B, C, 1, 1, P, 1, blocks=5)     # 12 not divisible by 5
    A2, B2, C2 = inputs.uniform(24, 12, 8, 12, P, True)
    with pytest.raises(ValueError):
        replay("blocked_acc", A2, B2, C2, 1, 1, P, 1, blocks=2)  # not square


# ------------------------------ the rectangular overwrite family (Section 5.3)
OVERWRITE_FAMILY = [
    # schedule, shape, levels, accumulates
    ("ovl", (32, 32, 32), 1, False), ("ovl", (64, 64, 64), 3, False),
    ("ovl", (16, 16, 16), 4, False),
    ("acr", (32, 32, 32), 2, True), ("acr", (64, 32, 128), 2, True),
    ("acr", (128, 64, 32), 3, True), ("acr", (32, 128, 64), 2, True),
    ("acr", (48, 16, 80), 1, True),
    ("ip0vmm", (64, 128, 32), 2, False), ("ip0vmm", (96, 64, 32), 1, False),
    ("ip0vmm", (32, 96, 32), 3, False), ("ip0vmm", (64, 32, 32), 2, False),
    ("ip0vmm", (32, 32, 32), 2, False), ("ip0vmm", (128, 128, 64), 2, False),
]


@pytest.mark.parametrize("p", [P, 8388593])
@pytest.mark.parametrize("schedule,shape,levels,accumulates", OVERWRITE_FAMILY)
def test_overwrite_family_value_with_garbage(schedule, shape, levels, accumulates, p):
    m, k, n = shape
    A, B, C = inputs.uniform(zlib.crc32(repr((schedule, shape, levels)).encode()), m, k, n, p, True)
    for seed, (alpha, beta) in enumerate([(1, 1), (3, p - 2), (p - 1, 5), (7, 0)]):
        if not accumulates:
            beta = 0
        r = replay(schedule, A, B, C, alpha, beta, p, levels, garbage_seed=seed)
        assert np.array_equal(r.C, o1(A, B, C, alpha, beta, p)), (alpha, beta)
        if schedule == "acr":
            assert np.array_equal(r.A, A)                      # Table 8 overwrites B only
        if schedule == "ovl":
            assert np.array_equal(r.B, B)                      # Table 4 overwrites A only
        if schedule == "ip0vmm" and m > n:
            assert np.array_equal(r.B, B)                      # Tables 1, 4, 2 leave B


def test_ovl_final_inputs_one_level():
    """Table 4 at one level ends with A = [[T4, A12], [P4, A22]] and B intact."""
    n, a = 32, 6
    A, B, _ = inputs.uniform(25, n, n, n, P)
    r = replay("ovl", A, B, None, a, 0, P, 1)
    d = _sp(A, B, np.zeros((n, n), np.int64), a, 0, P)
    t4 = (d["T2"] - d["B21"]) % P
    for got, want in zip(_blocks(r.A), [t4, d["A12"], d["P"][4], d["A22"]]):
        assert np.array_equal(got, want)
    assert np.array_equal(r.B, B)


def test_acr_final_inputs_one_level():
    """Table 8 at one level ends with B = [[B11, T2], [B21, B22]] and A intact."""
    n, a, b = 32, 4, 10
    A, B, C = inputs.uniform(26, n, n, n, P, True)
    r = replay("acr", A, B, C, a, b, P, 1)
    d = _sp(A, B, C, a, b, P)
    for got, want in zip(_blocks(r.B), [d["B11"], d["T2"], d["B21"], d["B22"]]):
        assert np.array_equal(got, want)
    assert np.array_equal(r.A, A)


def test_ip0vmm_final_state_is_deterministic():
    for shape in [(64, 128, 32), (32, 96, 32)]:
        m, k, n = shape
        A, B, _ = inputs.uniform(27, m, k, n, P)
        r1 = replay("ip0vmm", A, B, None, 2, 0, P, 2)
        r2 = replay("ip0vmm", A, B, None, 2, 0, P, 2)
        assert np.array_equal(r1.A, r2.A) and np.array_equal(r1.B, r2.B)


class _OvlReadsDeadA11(Winograd):
    """Table 4 with rows 3 and 5 exchanged: S2 = S1 - A11 is formed after P1
    has been allowed to destroy A11."""

    def ovl(self, A, B, C, a, lev):
        if lev == 0:
            self.leaf(A, B, C, a, 0, False)
            self.destroy(A)
            return
        n = C.shape[0]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((n // 2, n // 2)) as (X,):
            self.sub(C22, A11, A21)
            self.add(A21, A21, A22)
            self.sub(C21, B12, B11)
            self.ovl(A11, B11, C11, a, lev - 1)       # row 5 moved up
            self.sub(C12, A21, A11)                   # row 3 now reads a dead A11
            self.sub(A11, B22, B12)
            self.ip(C22, A11, X, a, lev - 1)
            self.sub(A11, B22, C21)
            self.ip(A21, C21, C22, a, lev - 1)
            self.sub(C21, A12, C12)
            self.ovl(C21, B22, A21, a, lev - 1)
            self.ovl(C12, A11, C21, a, lev - 1)
            self.sub(A11, A11, B21)
            self.add(C21, C11, C21)
            self.add(C12, C21, C22)
            self.add(C21, C21, X)
            self.add(C22, C21, C22)
            self.add(C12, C12, A21)
            self.ovl(A12, B21, X, a, lev - 1)
            self.add(C11, C11, X)
            self.ip(A22, A11, A21, a, lev - 1)
            self.sub(C21, C21, A21)
        self.destroy(A)


def test_garbage_mode_catches_a_planted_mistake_in_table4():
    n = 32
    A, B, _ = inputs.uniform(28, n, n, n, P)
    want = o1(A, B, None, 1, 0, P)
    w = _OvlReadsDeadA11(P, garbage_seed=0)
    C = np.zeros((n, n), np.int64)
    w.ovl(A.copy(), B.copy(), C, 1, 1)
    assert not np.array_equal(C, want)
    w = Winograd(P, garbage_seed=0)
    C = np.zeros((n, n), np.int64)
    w.ovl(A.copy(), B.copy(), C, 1, 1)
    assert np.array_equal(C, want)


def test_overwrite_family_rejects_unsupported_shapes():
    A, B, C = inputs.uniform(29, 24, 24, 24, P, True)
    with pytest.raises(ValueError):
        replay("ovl", A, B, C, 1, 1, P, 1)            # Table 4 has no beta
    with pytest.raises(ValueError):
        replay("acr", A, B, C, 1, 1, P, 4)            # 24 not divisible by 16
    A2, B2, C2 = inputs.uniform(30, 48, 32, 32, P, True)
    with pytest.raises(ValueError):
        replay("ip0vmm", A2, B2, None, 1, 0, P, 1)    # n = 32 does not divide m = 48
    A3, B3, _ = inputs.uniform(31, 32, 64, 64, P)
    with pytest.raises(ValueError):
        replay("ip0vmm", A3, B3, None, 1, 0, P, 1)    # n is not the smallest dimension


# ------------------- Algorithm 2 with Table 9 accumulations (end of Section 7.1)
@pytest.mark.parametrize("p", [P, 8388593])
@pytest.mark.parametrize("shape,levels", [((64, 64, 64), 1), ((64, 64, 64), 3), ((64, 128, 64), 2),
                                          ((32, 64, 32), 2), ((64, 32, 64), 2)])
def test_ipmm_acc_value_with_garbage(shape, levels, p):
    m, k, n = shape
    A, B, _ = inputs.uniform(zlib.crc32(repr(("ipmm_acc", shape, levels)).encode()), m, k, n, p)
    for seed, alpha in enumerate([1, 3, p - 1]):
        r = replay("ipmm_acc", A, B, None, alpha, 0, p, levels, garbage_seed=seed)
        assert np.array_equal(r.C, o1(A, B, None, alpha, 0, p))
        assert np.array_equal(r.A, A) and np.array_equal(r.B, B)
        assert r.peak == 0 and r.allocated == 0


def test_ipmm_acc_needs_square_chunks():
    A, B, _ = inputs.uniform(32, 64, 16, 64, P)
    with pytest.raises(ValueError):
        replay("ipmm_acc", A, B, None, 1, 0, P, 2)        # k < n/2: chunks are not square
