"""Symbolic check of every schedule replay of oracle O2 (the validator half of
the pebble game of Section 4).

The replays run on matrices of formal symbols instead of residues: every entry
of A, B and C is an atom, a product of two values is the bilinear expansion
into pairs (A-side atom, B-side atom), and coefficients live in Z/pZ.  Every
freshly allocated temporary and every operand that an overwriting callee may
destroy is filled with a new junk atom.  A schedule is then correct exactly
when the final C equals alpha*A*B + beta*C as a formal expression -- an
identity over every ring, not a sample -- and it reads no dead location
exactly when no junk atom survives into C.  Read-only schedules must leave
the atoms of A and B in place.

This pins the table transcriptions of oracle/schedules.py to the definition
of the product, independently of oracle O1 and of any random input.
"""
import itertools

import numpy as np
import pytest

from oracle import schedules as S
from oracle.schedules import Winograd

from .test_oracle_schedules import _SwappedIP, _OvlReadsDeadA11

P = 65521


class Sym:
    """A formal Z/pZ-combination of atoms and of products of atoms."""

    __slots__ = ("t",)

    def __init__(self, t=None):
        self.t = t if t is not None else {}

    @staticmethod
    def atom(key):
        return Sym({key: 1})

    def _comb(self, other, sign):
        if isinstance(other, (int, np.integer)):
            if int(other) % P:
                raise TypeError("a nonzero constant entered a symbolic replay")
            return self
        t = dict(self.t)
        for k, v in other.t.items():
            c = (t.get(k, 0) + sign * v) % P
            if c:
                t[k] = c
            else:
                t.pop(k, None)
        return Sym(t)

    def __add__(self, other):
        return self._comb(other, 1)

    __radd__ = __add__

    def __sub__(self, other):
        return self._comb(other, -1)

    def __rsub__(self, other):
        return (self * -1)._comb(other, 1)

    def __mul__(self, other):
        if isinstance(other, (int, np.integer)):
            c = int(other) % P
            return Sym({k: v * c % P for k, v in self.t.items() if v * c % P})
        t = {}
        for (k1, v1), (k2, v2) in itertools.product(self.t.items(), other.t.items()):
            key = ("*", k1, k2)
            c = (t.get(key, 0) + v1 * v2) % P
            if c:
                t[key] = c
            else:
                t.pop(key, None)
        return Sym(t)

    def __rmul__(self, other):
        return self * other

    def __mod__(self, p):
        assert p == P
        return self

    def __eq__(self, other):
        return isinstance(other, Sym) and self.t == other.t

    __hash__ = None

    def has_junk(self):
        def junk(key):
            return key[0] == "junk" or (key[0] == "*" and (junk(key[1]) or junk(key[2])))
        return any(junk(k) for k in self.t)


def _symbols(name, r, c):
    M = np.empty((r, c), dtype=object)
    for i, j in np.ndindex(r, c):
        M[i, j] = Sym.atom((name, i, j))
    return M


def _replay(schedule, m, k, n, levels, alpha, beta, blocks=2, cls=Winograd):
    count = itertools.count()
    w = cls(P, junk=lambda: Sym.atom(("junk", next(count))))
    A, B, C = _symbols("a", m, k), _symbols("b", k, n), _symbols("c", m, n)
    A0, B0, C0 = A.copy(), B.copy(), C.copy()
    S._check(schedule, m, k, n, P, beta, levels, blocks)
    if beta % P == 0:
        w._garbage(C)                       # C is output only
    S._run(w, schedule, A, B, C, alpha, beta, levels, blocks)
    return (A0, B0, C0), (A, B, C)


def _expected(A, B, C, alpha, beta):
    m, k = A.shape
    n = B.shape[1]
    E = np.empty((m, n), dtype=object)
    for i, j in np.ndindex(m, n):
        e = Sym()
        for l in range(k):
            e = e + A[i, l] * B[l, j]
        e = e * alpha
        if beta % P:
            e = e + C[i, j] * beta
        E[i, j] = e
    return E


CASES = [
    ("classical", (4, 3, 5), 0),
    ("t1", (2, 2, 2), 1), ("t1", (4, 4, 4), 2), ("t1", (4, 2, 6), 1), ("t1", (3, 3, 3), 1),
    ("hl", (2, 2, 2), 1), ("hl", (4, 4, 4), 2), ("hl", (4, 2, 6), 1), ("hl", (3, 5, 3), 1),
    ("acc", (2, 2, 2), 1), ("acc", (4, 4, 4), 2), ("acc", (5, 5, 5), 2),
    ("ip", (2, 2, 2), 1), ("ip", (4, 4, 4), 2), ("ip", (8, 8, 8), 3),
    ("ovl", (2, 2, 2), 1), ("ovl", (4, 4, 4), 2), ("ovl", (8, 8, 8), 3),
    ("ovr", (2, 2, 2), 1), ("ovr", (4, 4, 4), 2), ("ovr", (8, 8, 8), 3),
    ("aclr", (2, 2, 2), 1), ("aclr", (4, 4, 4), 2), ("aclr", (8, 8, 8), 3),
    ("accr", (2, 2, 2), 1), ("accr", (4, 4, 4), 2), ("accr", (8, 8, 8), 3),
    ("acr", (2, 2, 2), 1), ("acr", (4, 4, 4), 2), ("acr", (4, 2, 8), 1), ("acr", (8, 4, 4), 2),
    ("ipmm", (4, 4, 4), 1), ("ipmm", (8, 8, 8), 2), ("ipmm", (4, 8, 4), 1),
    ("ipmm_acc", (4, 4, 4), 1), ("ipmm_acc", (8, 8, 8), 2), ("ipmm_acc", (4, 8, 4), 1),
    ("ip0vmm", (4, 4, 2), 1), ("ip0vmm", (2, 6, 2), 1), ("ip0vmm", (6, 4, 2), 1),
    ("ip0vmm", (8, 16, 4), 2), ("ip0vmm", (4, 4, 4), 2),
]
READ_ONLY = ("classical", "t1", "hl", "acc", "ipmm", "ipmm_acc", "blocked", "blocked_acc")
PLAIN = ("t1", "ip", "ovr", "ovl", "ipmm", "ipmm_acc", "ip0vmm")


def _verify(schedule, shape, levels, blocks=2):
    m, k, n = shape
    for alpha, beta in [(1, 1), (3, 5), (2, 0), (P - 1, P - 2)]:
        if schedule in PLAIN:
            beta = 0
        (A0, B0, C0), (A, B, C) = _replay(schedule, m, k, n, levels, alpha, beta, blocks)
        want = _expected(A0, B0, C0, alpha, beta)
        for idx in np.ndindex(m, n):
            assert not C[idx].has_junk(), (alpha, beta, idx)
            assert C[idx] == want[idx], (alpha, beta, idx)
        if schedule in READ_ONLY:
            assert all(A[i] == A0[i] for i in np.ndindex(A.shape))
            assert all(B[i] == B0[i] for i in np.ndindex(B.shape))


@pytest.mark.parametrize("schedule,shape,levels", CASES)
def test_schedule_is_the_product_symbolically(schedule, shape, levels):
    _verify(schedule, shape, levels)


@pytest.mark.parametrize("schedule,shape,levels,t", [
    ("blocked", (4, 4, 4), 1, 2), ("blocked", (6, 6, 6), 1, 3), ("blocked", (5, 3, 7), 1, 2),
    ("blocked", (8, 8, 8), 2, 2), ("blocked_acc", (4, 4, 4), 1, 2), ("blocked_acc", (6, 6, 6), 1, 3),
    ("blocked_acc", (8, 8, 8), 1, 4)])
def test_blocked_is_the_product_symbolically(schedule, shape, levels, t):
    _verify(schedule, shape, levels, t)


@pytest.mark.parametrize("cls,schedule", [(_SwappedIP, "ip"), (_OvlReadsDeadA11, "ovl")])
def test_planted_dead_read_leaves_junk(cls, schedule):
    """Rows taken out of order read a location whose value is dead: junk
    reaches C."""
    (A0, B0, C0), (A, B, C) = _replay(schedule, 4, 4, 4, 1, 1, 0, cls=cls)
    assert any(C[idx].has_junk() for idx in np.ndindex(4, 4))


def test_symbols_follow_ring_rules():
    """The symbolic ring itself: distributivity, additive inverses, and no
    commutation of the two factors of a product."""
    a, b, c = Sym.atom(("a", 0, 0)), Sym.atom(("b", 0, 0)), Sym.atom(("c", 0, 0))
    assert (a + c) * b == a * b + c * b
    assert a * (b + c) == a * b + a * c
    assert (a - a) == Sym() and (a * b - a * b) == Sym()
    assert a * b != b * a
    assert (a * 3 + a * (P - 3)) == Sym()
