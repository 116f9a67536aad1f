"""Pins for the final contents of inputs that an overwriting schedule destroys,
at any depth, written without the replay.

A schedule that overwrites its inputs (Tables 3-8, Algorithm 1) leaves every
quadrant of A and B in one of three states:

* a value it stored there last: a Section 2 block (S1..S4, T1..T4), a product
  P1..P7 (alpha times the product, reduced), or a post-addition U_i;
* an operand block it never touched;
* the operand of its last destroying sub-call, which at the next level down
  leaves that quadrant in *that* callee's final state.

So the final state at depth L is the one-level form of the table with the
third kind of quadrant replaced by the callee's final state at depth L-1 on
the same operands; at depth 0 (the classical base) nothing is destroyed.  The
functions below write these recursions out from Section 2's definitions of
S, T, P and U and from which sub-call of each table last consumes each
quadrant; products come from oracle O1 (pinned by brute force elsewhere).
Nothing here calls the replay's schedule code: the replay is only the thing
compared.

Algorithm 1 also lends the block A_11 of A to the temporaries of its later
calls (the quadtree placement: slots top-left, bottom-left, top-right for the
first, second and third temporary of a call, the bottom-right quadrant for
its callees).  Its final contents are then the last temporaries stored at
each depth of that quadtree, and the original (or already overwritten)
entries wherever no temporary ever landed.
"""
import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay
from paper_0707_2347_amd import inputs


def q(M):
    """Quadrants M11, M12, M21, M22 (half the rows, half the columns)."""
    r, c = M.shape[0] // 2, M.shape[1] // 2
    return M[:r, :c], M[:r, c:], M[r:, :c], M[r:, c:]


def join(M11, M12, M21, M22):
    return np.block([[M11, M12], [M21, M22]])


class Blocks:
    """Section 2's blocks of one call on operands X (A-role) and Y (B-role)."""

    def __init__(self, X, Y, a, p):
        self.p, self.a = p, a
        self.X11, self.X12, self.X21, self.X22 = q(X)
        self.Y11, self.Y12, self.Y21, self.Y22 = q(Y)
        self.S1 = (self.X21 + self.X22) % p
        self.S2 = (self.S1 - self.X11) % p
        self.S3 = (self.X11 - self.X21) % p
        self.S4 = (self.X12 - self.S2) % p
        self.T1 = (self.Y12 - self.Y11) % p
        self.T2 = (self.Y22 - self.T1) % p
        self.T3 = (self.Y22 - self.Y12) % p
        self.T4 = (self.T2 - self.Y21) % p

    def prod(self, U, V):
        return ref.matmul_mod_p(U, V, None, self.a, 0, self.p)

    @property
    def P1(self):
        return self.prod(self.X11, self.Y11)

    @property
    def P2(self):
        return self.prod(self.X12, self.Y21)

    @property
    def P3(self):
        return self.prod(self.S4, self.Y22)

    @property
    def P4(self):
        return self.prod(self.X22, self.T4)

    @property
    def P5(self):
        return self.prod(self.S1, self.T1)

    @property
    def P6(self):
        return self.prod(self.S2, self.T2)

    @property
    def P7(self):
        return self.prod(self.S3, self.T3)


# ---------------------------------------------------- final-state recursions
# Each takes the operands of one call (X in the A role, Y in the B role) and
# the depth L, and returns the final contents of the operand it destroys.

def ip_a(X, Y, a, p, L):
    """Table 3, A: P5 and P3 on top, P4 and the operand S4 of the last call
    (P3 = S4 B22) below."""
    if L == 0:
        return X
    d = Blocks(X, Y, a, p)
    return join(d.P5, d.P3, d.P4, ip_a(d.S4, d.Y22, a, p, L - 1))


def ip_b(X, Y, a, p, L):
    """Table 3, B: each quadrant is the B operand of the last call reading it:
    P6 = S2 T2, P7 = S3 T3, P2 = A12 B21, P3 = S4 B22."""
    if L == 0:
        return Y
    d = Blocks(X, Y, a, p)
    return join(ip_b(d.S2, d.T2, a, p, L - 1), ip_b(d.S3, d.T3, a, p, L - 1),
                ip_b(d.X12, d.Y21, a, p, L - 1), ip_b(d.S4, d.Y22, a, p, L - 1))


def ovl_a(X, Y, a, p, L):
    """Table 4, A: T4 (then both operands of P4 = A22 T4, a Table 3 call),
    A12 (operand of P2, a Table 4 call), the product P4."""
    if L == 0:
        return X
    d = Blocks(X, Y, a, p)
    return join(ip_b(d.X22, d.T4, a, p, L - 1), ovl_a(d.X12, d.Y21, a, p, L - 1),
                d.P4, ip_a(d.X22, d.T4, a, p, L - 1))


def ovr_b(X, Y, a, p, L):
    """Table 5, B: S4 and B22 (operands of P3, a Table 3 call), the product
    P2, B21 (operand of P2, a Table 5 call)."""
    if L == 0:
        return Y
    d = Blocks(X, Y, a, p)
    return join(ip_a(d.S4, d.Y22, a, p, L - 1), d.P2,
                ovr_b(d.X12, d.Y21, a, p, L - 1), ip_b(d.S4, d.Y22, a, p, L - 1))


def aclr_a(X, Y, a, p, L):
    """Table 6, A: operands of P1 (Table 3), P2 (Table 6), P6 and P3 (Table 3)."""
    if L == 0:
        return X
    d = Blocks(X, Y, a, p)
    return join(ip_a(d.X11, d.Y11, a, p, L - 1), aclr_a(d.X12, d.Y21, a, p, L - 1),
                ip_a(d.S2, d.T2, a, p, L - 1), ip_a(d.S4, d.Y22, a, p, L - 1))


def aclr_b(X, Y, a, p, L):
    """Table 6, B: operands of P1, P6 (Table 3), P2 (Table 6), P3 (Table 3)."""
    if L == 0:
        return Y
    d = Blocks(X, Y, a, p)
    return join(ip_b(d.X11, d.Y11, a, p, L - 1), ip_b(d.S2, d.T2, a, p, L - 1),
                aclr_b(d.X12, d.Y21, a, p, L - 1), ip_b(d.S4, d.Y22, a, p, L - 1))


def accr_b(X, Y, C, a, b, p, L):
    """Table 7, B: operands of P1 and P6 (Table 5 calls), U4 + b*C12 (stored
    last into B21), operand of P3 (Table 3)."""
    if L == 0:
        return Y
    d = Blocks(X, Y, a, p)
    u4 = (d.P1 + d.P6 + d.P5 + b * q(C)[1]) % p
    return join(ovr_b(d.X11, d.Y11, a, p, L - 1), ovr_b(d.S2, d.T2, a, p, L - 1), u4,
                ip_b(d.S4, d.Y22, a, p, L - 1))


def acr_b(X, Y, a, p, L):
    """Table 8, B: B11 and B22 only read; T2 and B21 consumed by Table 8 calls
    (U2 = S2 T2 + P1 and P2 = A12 B21)."""
    if L == 0:
        return Y
    d = Blocks(X, Y, a, p)
    return join(d.Y11, acr_b(d.S2, d.T2, a, p, L - 1), acr_b(d.X12, d.Y21, a, p, L - 1), d.Y22)


# --------------------------------------------------------------- Algorithm 1
def _overlay_chain(R, L, temps_of, first):
    """Write the temporaries of a chain of calls into the quadtree of R: the
    call at depth d (level L - d) stores its temporaries in the top-left,
    bottom-left and top-right quadrants of R's bottom-right quadrant taken d
    times; temps_of(state) returns those blocks and the next call's state."""
    state = first
    for _ in range(L):
        temps, state = temps_of(state)
        r11, r12, r21, r22 = q(R)
        for slot, T in zip((r11, r21, r12), temps):
            slot[:T.shape[0], :T.shape[1]] = T
        R = r22


def ip0vmm_final(A, B, a, p, L):
    """Final A and B of Algorithm 1 (n = min(m, k, n) dividing m and k)."""
    m, k = A.shape
    s = B.shape[1]
    m0, k0 = m // s, k // s
    A, B = A.copy(), B.copy()
    Ab = lambda i, j: A[i * s:(i + 1) * s, j * s:(j + 1) * s]
    Bb = lambda j: B[j * s:(j + 1) * s]
    if m0 == 1:
        # Table 3 on the first block column, then Table 6 on each further one
        # with its temporaries in the freed A_11.
        A0, B0 = Ab(0, 0).copy(), Bb(0).copy()
        acc = ref.matmul_mod_p(A0, B0, None, a, 0, p)
        Ab(0, 0)[...] = ip_a(A0, B0, a, p, L)
        Bb(0)[...] = ip_b(A0, B0, a, p, L)
        for j in range(1, k0):
            X, Y = Ab(0, j).copy(), Bb(j).copy()
            Ab(0, j)[...] = aclr_a(X, Y, a, p, L)
            Bb(j)[...] = aclr_b(X, Y, a, p, L)
            if j == k0 - 1:
                # Table 6's temporaries end as X = U4 + b*C12 (b = 1 here) and
                # Y = P1; its last callee with temporaries is row 16's
                # P2 + b*C11 on (A12, B21, C11).
                def temps(st):
                    Xc, Yc, Cc = st
                    d = Blocks(Xc, Yc, a, p)
                    x = (d.P1 + d.P6 + d.P5 + q(Cc)[1]) % p
                    return (x, d.P1), (d.X12, d.Y21, q(Cc)[0])
                _overlay_chain(Ab(0, 0), L, temps, (X, Y, acc))
            acc = (acc + ref.matmul_mod_p(X, Y, None, a, 0, p)) % p
        return A, B
    # m0 > 1: Table 1 on A_11 (temporaries in C), A_11 freed; Table 4 down the
    # first block column, Table 2 (read-only) for the other block columns.
    last_col0 = Ab(m0 - 1, 0).copy()
    for i in range(1, m0):
        Ab(i, 0)[...] = ovl_a(Ab(i, 0).copy(), Bb(0), a, p, L)
    if k0 > 1:
        # Last call: Table 2 on (A_{m0-1,k0-1}, B_{k0-1}); its temporaries end
        # as S3, T3 and U3 = P1 + P6 + P7, its last callee with temporaries is
        # row 19's on (S3, T3).
        def temps(st):
            d = Blocks(st[0], st[1], a, p)
            return (d.S3, d.T3, (d.P1 + d.P6 + d.P7) % p), (d.S3, d.T3)
        _overlay_chain(Ab(0, 0), L, temps, (Ab(m0 - 1, k0 - 1).copy(), Bb(k0 - 1)))
    else:
        # Last call: Table 4 on (A_{m0-1,0}, B_0) (its original operand); its
        # temporary ends as P2, its last callee with a temporary is row 19's
        # P2 on (A12, B21).
        def temps(st):
            d = Blocks(st[0], st[1], a, p)
            return (d.P2,), (d.X12, d.Y21)
        _overlay_chain(Ab(0, 0), L, temps, (last_col0, Bb(0)))
    return A, B


# ---------------------------------------------------------------------- tests
P = 65521
LEVELS = [1, 2, 3]


def _inputs(seed, m, k, n, p, with_c=False):
    return inputs.uniform(seed, m, k, n, p, with_c=with_c)


@pytest.mark.parametrize("L", LEVELS)
@pytest.mark.parametrize("p", [P, 8388593])
def test_table3_final_inputs(L, p):
    n, a = 32, 7
    A, B, _ = _inputs(100 + L, n, n, n, p)
    r = replay("ip", A, B, None, a, 0, p, L)
    assert np.array_equal(r.A, ip_a(A, B, a, p, L))
    assert np.array_equal(r.B, ip_b(A, B, a, p, L))


@pytest.mark.parametrize("L", LEVELS)
def test_table4_final_inputs(L):
    n, a = 32, 6
    A, B, _ = _inputs(110 + L, n, n, n, P)
    r = replay("ovl", A, B, None, a, 0, P, L)
    assert np.array_equal(r.A, ovl_a(A, B, a, P, L))
    assert np.array_equal(r.B, B)


@pytest.mark.parametrize("L", LEVELS)
def test_table5_final_inputs(L):
    n, a = 32, 3
    A, B, _ = _inputs(120 + L, n, n, n, P)
    r = replay("ovr", A, B, None, a, 0, P, L)
    assert np.array_equal(r.B, ovr_b(A, B, a, P, L))
    assert np.array_equal(r.A, A)


@pytest.mark.parametrize("L", LEVELS)
@pytest.mark.parametrize("p", [P, 8388593])
def test_table6_final_inputs(L, p):
    n, a, b = 32, 5, 9
    A, B, C = _inputs(130 + L, n, n, n, p, True)
    r = replay("aclr", A, B, C, a, b, p, L)
    assert np.array_equal(r.A, aclr_a(A, B, a, p, L))
    assert np.array_equal(r.B, aclr_b(A, B, a, p, L))


@pytest.mark.parametrize("L", LEVELS)
def test_table7_final_inputs(L):
    n, a, b = 32, 4, 6
    A, B, C = _inputs(140 + L, n, n, n, P, True)
    r = replay("accr", A, B, C, a, b, P, L)
    assert np.array_equal(r.B, accr_b(A, B, C, a, b, P, L))
    assert np.array_equal(r.A, A)


@pytest.mark.parametrize("L", LEVELS)
@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 32, 128), (128, 64, 32), (32, 128, 64)])
def test_table8_final_inputs(L, shape):
    m, k, n = shape
    a, b = 4, 10
    A, B, C = _inputs(150 + L + m, m, k, n, P, True)
    r = replay("acr", A, B, C, a, b, P, L)
    assert np.array_equal(r.B, acr_b(A, B, a, P, L))
    assert np.array_equal(r.A, A)


@pytest.mark.parametrize("L", LEVELS)
@pytest.mark.parametrize("shape", [(32, 64, 32), (32, 96, 32), (32, 32, 32)])
def test_algorithm1_one_block_row_final_inputs(L, shape):
    """m = n: Table 3, then Table 6 on each further block column, with the
    Table 6 temporaries in the freed A_11."""
    m, k, n = shape
    a = 3
    A, B, _ = _inputs(160 + L + k, m, k, n, P)
    r = replay("ip0vmm", A, B, None, a, 0, P, L)
    wa, wb = ip0vmm_final(A, B, a, P, L)
    assert np.array_equal(r.A, wa)
    assert np.array_equal(r.B, wb)


@pytest.mark.parametrize("L", LEVELS)
@pytest.mark.parametrize("shape", [(64, 128, 32), (96, 64, 32), (128, 128, 64)])
def test_algorithm1_several_block_rows_final_inputs(L, shape):
    """n < m: Table 1 on the first block, Table 4 down the first block column
    and Table 2 elsewhere, all later temporaries in the freed A_11; B intact."""
    m, k, n = shape
    a = 5
    A, B, _ = _inputs(170 + L + m + k, m, k, n, P)
    r = replay("ip0vmm", A, B, None, a, 0, P, L)
    wa, wb = ip0vmm_final(A, B, a, P, L)
    assert np.array_equal(r.A, wa)
    assert np.array_equal(r.B, B)


@pytest.mark.parametrize("L", LEVELS)
@pytest.mark.parametrize("shape", [(64, 32, 32), (128, 32, 32)])
def test_algorithm1_one_block_column_final_inputs(L, shape):
    m, k, n = shape
    a = 2
    A, B, _ = _inputs(180 + L + m, m, k, n, P)
    r = replay("ip0vmm", A, B, None, a, 0, P, L)
    wa, wb = ip0vmm_final(A, B, a, P, L)
    assert np.array_equal(r.A, wa)
    assert np.array_equal(r.B, B)


def test_recursions_reduce_to_the_one_level_forms():
    """At one level the recursions are the one-level forms: a mistake in a
    recursion's quadrant order shows here against Section 2's blocks."""
    n, a, b = 16, 3, 4
    A, B, C = _inputs(190, n, n, n, P, True)
    d = Blocks(A, B, a, P)
    assert np.array_equal(ip_a(A, B, a, P, 1), join(d.P5, d.P3, d.P4, d.S4))
    assert np.array_equal(ip_b(A, B, a, P, 1), join(d.T2, d.T3, d.Y21, d.Y22))
    assert np.array_equal(ovl_a(A, B, a, P, 1), join(d.T4, d.X12, d.P4, d.X22))
    assert np.array_equal(ovr_b(A, B, a, P, 1), join(d.S4, d.P2, d.Y21, d.Y22))
    assert np.array_equal(aclr_a(A, B, a, P, 1), join(d.X11, d.X12, d.S2, d.S4))
    assert np.array_equal(aclr_b(A, B, a, P, 1), join(d.Y11, d.T2, d.Y21, d.Y22))
    assert np.array_equal(acr_b(A, B, a, P, 1), join(d.Y11, d.T2, d.Y21, d.Y22))
    u4 = (d.P1 + d.P6 + d.P5 + b * q(C)[1]) % P
    assert np.array_equal(accr_b(A, B, C, a, b, P, 1), join(d.Y11, d.T2, u4, d.Y22))
