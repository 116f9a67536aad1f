"""Oracle O2: Winograd's algorithm replayed under each memory schedule.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code, table or helper
with the GPU library: the schedules below are written from the paper directly.

What it is for
--------------
Every schedule computes the same value as the plain product (oracle O1) --
Winograd's identity is exact in any ring -- so the value itself is pinned by
O1.  This replay adds what O1 cannot see:

* the *memory placement* of each table: every row writes exactly the location
  named in the table's "loc." column, sub-products go through the callee
  schedule the table names, and temporaries come from an arena that records
  the peak extra memory and the total number of allocated elements;
* the final contents of the inputs after a schedule that overwrites them
  (needed to compare such schedules bit for bit);
* the number of element additions and base-case operations, to compare with
  the paper's arithmetic recurrences (Theorem 1, Theorem 3);
* the largest unreduced partial sum seen in the base case, to compare with
  the exactness bound of a delayed reduction in binary64 (2**53).

A "garbage" mode fills freshly allocated temporaries, and the operands an
overwriting callee is allowed to destroy, with random residues.  A schedule
that reads a dead value then returns a wrong product, which the tests catch.

The final contents of inputs an overwriting schedule destroys (Tables 3-8,
Algorithm 1) are pinned at every depth by closed-form recursions written from
Section 2's block definitions, independently of this replay.

Notation (Section 2): A is m x k, B is k x n, C is m x n, each split into
quadrants X11, X12, X21, X22 of half the rows and half the columns.
S1..S4 / T1..T4 are the pre-additions, P1..P7 the seven products and
U1..U7 the post-additions.  All arithmetic is exact in int64 and every stored
value is a canonical residue in [0, p).

Readings of the paper taken here (where it is silent or garbled):
* alpha is applied at the base case (linearity); beta where the rows say.
  "-beta" means the residue p - beta.
* The "operation" column names the beta-free value; the row is executed with
  the location semantics that reproduce alpha*A*B + beta*C (for instance
  Table 9 row 10 stores P5 + beta*Z1 plus what is already in C12).
* Table 6 prints two row numbers twice; the rows are taken in table order,
  left column 1-12 then right column 13-24.
* Table 9 row 24 is executed as an AccR call with -alpha and beta' = 1 into
  C21 (U3 - alpha*A22*T4), which is the same value without a negation pass.
* At the base case an "overwriting" callee is a plain classical product and
  leaves its operands unchanged (so the final state of overwritten inputs is
  fully determined by the tables).
* Section 7.2 (blocked accumulation) with a block count t: A, B and C are
  cut along every dimension into t consecutive parts (the paper's n/t when t
  divides the dimension; otherwise parts of ceil(d/t) rounded up to a multiple
  of 2**L, the last one shorter).  Block C_ij accumulates the products
  A_il B_lj for l = 1..t in order, the first with beta and the others with 1,
  each by one call of the base schedule (Table 2, or Table 9 for square
  blocks).  Only one call's temporaries exist at a time.
* Table 8's X holds a T block (k/2 x n/2) and then products (m/2 x n/2), so it
  is max(m/2, k/2) x n/2; Y holds S blocks (m/2 x k/2).  Its two plain
  products (rows 12 and 22) are Table 1 calls.
* Algorithm 1 (IP0vMM) as its section describes it, with the loop bounds and
  the accumulation read as C_i <- A_ij B_j + C_i (the printed indices are
  garbled): n = min(m, k, n) must divide m and k, and A, B, C are cut into
  n x n squares A_ij (m0 x k0 of them), B_j and C_i.  With m0 >= 2: C_1 by
  Table 1 with its temporaries in C_2, then A_11 is free space; C_i for
  i >= 2 by Table 4 (overwriting A_i1) and then C_i += A_ij B_j for j >= 2
  by Table 2, all with temporaries in A_11.  With m0 = 1 (m = n <= k, the
  shapes the paper times): C by Table 3 from A_1 and B_1, then C += A_j B_j
  by Table 6 with temporaries in the freed A_1.  Temporaries in a free
  square are laid out as in Algorithm 2 (quadrants, recursion in the
  bottom-right one).
* Algorithm 2 with Table 9 for the accumulating chunks (the remark closing
  Section 7.1, square case): every chunk after the first runs Table 9 instead
  of Table 2, which needs square chunk products (k >= n/2, so K = s/2 at every
  depth); Table 9's two temporaries take the top-left and bottom-left
  quadrants of the lent region.
* Algorithm 2 with the depth parameter L: at depth d < L the three quadrant
  products are Winograd calls of depth L - d, with inner dimension cut in
  chunks of K = min(s/2, k); at depth L the remaining corner is a classical
  product over the whole inner dimension.  Temporaries of those calls are
  quadrants of C22: X in the top-left, Y in the bottom-left, Z (Table 2 only)
  in the top-right, and the callee's own temporaries in the bottom-right.
"""
from collections import Counter
from contextlib import contextmanager

import numpy as np

SCHEDULES = ("classical", "t1", "hl", "ip", "ovr", "aclr", "accr", "acc", "ipmm",
             "blocked", "blocked_acc", "ovl", "acr", "ip0vmm", "ipmm_acc")
OVERWRITES = {"ip": "AB", "ovr": "B", "aclr": "AB", "accr": "B", "ovl": "A", "acr": "B",
              "ip0vmm": "AB"}


def quads(M):
    """The four quadrant views (Section 2's natural block decomposition)."""
    r, c = M.shape[0] // 2, M.shape[1] // 2
    return M[:r, :c], M[:r, c:], M[r:, :c], M[r:, c:]


def fp64_chunk(p: int) -> int:
    """Largest t with t*(p-1)**2 + (p-1) < 2**53 (exact binary64 sums)."""
    q = (p - 1) * (p - 1)
    return max(1, (2 ** 53 - 1 - (p - 1)) // q) if q else 2 ** 53


class Winograd:
    """One replay: state (counters, arena) plus one method per schedule."""

    def __init__(self, p, *, dry=False, garbage_seed=None, kc=None, junk=None):
        self.p = int(p)
        self.dry = dry
        self.rng = None if garbage_seed is None else np.random.default_rng(garbage_seed)
        # Symbolic replays: ``junk()`` returns a fresh unknown value; then every
        # matrix is an object array and dead values are junk, not residues.
        self.junk = junk
        self.kc = int(kc) if kc else fp64_chunk(self.p)
        self.adds = 0            # element additions, one per element per addition row
        self.leaf_ops = 0        # classical base-case operations
        self.leaf_calls = 0
        self.cur = 0             # extra memory currently allocated (elements)
        self.peak = 0            # high-water mark of extra memory (elements)
        self.allocated = 0       # total elements ever allocated (the paper's A)
        self.calls = Counter()
        self.max_partial = 0     # largest unreduced base-case partial sum
        self._regions = []       # regions of C lent as temporary space (Alg. 2)

    # ---------------------------------------------------------------- storage
    def _garbage(self, V):
        if self.junk is not None and V.size:
            for idx in np.ndindex(V.shape):
                V[idx] = self.junk()
        elif self.rng is not None and not self.dry and V.size:
            V[...] = self.rng.integers(0, self.p, size=V.shape, dtype=np.int64)

    @contextmanager
    def frame(self, *shapes):
        """Temporaries of one schedule call, released when the call returns."""
        if self._regions:
            R = self._regions[-1]
            q11, q12, q21, q22 = quads(R)
            slots = (q11, q21, q12)
            if len(shapes) > len(slots):
                raise AssertionError("region cannot host this many temporaries")
            views = []
            for (r, c), q in zip(shapes, slots):
                if r > q.shape[0] or c > q.shape[1]:
                    raise AssertionError("temporary %dx%d does not fit a %dx%d quadrant"
                                         % (r, c, q.shape[0], q.shape[1]))
                views.append(q[:r, :c])
            for V in views:
                self._garbage(V)
            self._regions.append(q22)
            try:
                yield views
            finally:
                self._regions.pop()
            return
        views = []
        total = 0
        for r, c in shapes:
            if self.dry:
                V = np.lib.stride_tricks.as_strided(np.zeros(1, np.int64),
                                                    shape=(r, c), strides=(0, 0))
            else:
                V = np.zeros((r, c), dtype=object if self.junk else np.int64)
                self._garbage(V)
            views.append(V)
            total += r * c
        self.cur += total
        self.allocated += total
        self.peak = max(self.peak, self.cur)
        try:
            yield views
        finally:
            self.cur -= total

    def destroy(self, *views):
        """An overwriting callee returned: its destroyed operands are dead."""
        for V in views:
            self._garbage(V)

    # ------------------------------------------------------------- arithmetic
    def add(self, dst, x, y):
        self.adds += dst.size
        if not self.dry:
            dst[...] = (x + y) % self.p

    def sub(self, dst, x, y):
        self.adds += dst.size
        if not self.dry:
            dst[...] = (x - y) % self.p

    def lin(self, dst, x, cx, y, cy):
        """One addition row with scalings: dst <- cx*x + cy*y."""
        self.adds += dst.size
        if not self.dry:
            dst[...] = (int(cx) % self.p * x + int(cy) % self.p * y) % self.p

    def leaf(self, A, B, C, a, b, accumulate):
        """Classical base case: C <- a*A*B + b*C (C not read when b == 0 mod p).

        Operation count: m*n*(2k-1) for a plain product, 2*m*n*k when the call
        accumulates (the paper's W(1) = 1 and W_acc(1) = 2 per element)."""
        m, k = A.shape
        n = B.shape[1]
        self.leaf_calls += 1
        self.leaf_ops += 2 * m * n * k if accumulate else m * n * max(2 * k - 1, 0)
        if self.dry:
            return
        p = self.p
        s = np.zeros((m, n), dtype=np.int64)
        for l0 in range(0, k, self.kc):
            s = s + A[:, l0:l0 + self.kc] @ B[l0:l0 + self.kc, :]
            if s.size:
                if s.dtype != object:
                    self.max_partial = max(self.max_partial, int(np.abs(s).max()))
            s %= p
        r = (int(a) % p) * s % p
        if int(b) % p:
            r = (r + (int(b) % p) * C) % p
        C[...] = r

    # ---------------------------------------------------------- Table 1 (T1)
    def t1(self, A, B, C, a, lev):
        """Table 1: C <- a*A*B with two temporaries X (m/2 x max(k/2,n/2)) and
        Y (k/2 x n/2); A and B are read only."""
        self.calls["t1"] += 1
        if lev == 0:
            return self.leaf(A, B, C, a, 0, False)
        m, k = A.shape
        n = B.shape[1]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((m // 2, max(k // 2, n // 2)), (k // 2, n // 2)) as (X, Y):
            XS = X[:, :k // 2]          # X holding an S block
            XP = X[:, :n // 2]          # X holding a product
            self.sub(XS, A11, A21)               # 1  S3
            self.sub(Y, B22, B12)                # 2  T3
            self.t1(XS, Y, C21, a, lev - 1)      # 3  P7 = S3 T3
            self.add(XS, A21, A22)               # 4  S1
            self.sub(Y, B12, B11)                # 5  T1
            self.t1(XS, Y, C22, a, lev - 1)      # 6  P5 = S1 T1
            self.sub(XS, XS, A11)                # 7  S2 = S1 - A11
            self.sub(Y, B22, Y)                  # 8  T2 = B22 - T1
            self.t1(XS, Y, C12, a, lev - 1)      # 9  P6 = S2 T2
            self.sub(XS, A12, XS)                # 10 S4 = A12 - S2
            self.t1(XS, B22, C11, a, lev - 1)    # 11 P3 = S4 B22
            self.t1(A11, B11, XP, a, lev - 1)    # 12 P1
            self.add(C12, XP, C12)               # 13 U2 = P1 + P6
            self.add(C21, C12, C21)              # 14 U3 = U2 + P7
            self.add(C12, C12, C22)              # 15 U4 = U2 + P5
            self.add(C22, C21, C22)              # 16 U7 = U3 + P5
            self.add(C12, C12, C11)              # 17 U5 = U4 + P3
            self.sub(Y, Y, B21)                  # 18 T4 = T2 - B21
            self.t1(A22, Y, C11, a, lev - 1)     # 19 P4 = A22 T4
            self.sub(C21, C21, C11)              # 20 U6 = U3 - P4
            self.t1(A12, B21, C11, a, lev - 1)   # 21 P2
            self.add(C11, XP, C11)               # 22 U1 = P1 + P2

    # ---------------------------------------------------------- Table 2 (HL)
    def hl(self, A, B, C, a, b, lev):
        """Table 2: C <- a*A*B + b*C with three temporaries X (m/2 x k/2),
        Y (k/2 x n/2), Z (m/2 x n/2); A and B are read only."""
        self.calls["hl"] += 1
        if lev == 0:
            return self.leaf(A, B, C, a, b, True)
        m, k = A.shape
        n = B.shape[1]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((m // 2, k // 2), (k // 2, n // 2), (m // 2, n // 2)) as (X, Y, Z):
            self.add(X, A21, A22)                # 1  S1
            self.sub(Y, B12, B11)                # 2  T1
            self.t1(X, Y, Z, a, lev - 1)         # 3  P5 = a S1 T1
            self.lin(C22, Z, 1, C22, b)          # 4  C22 = P5 + b C22
            self.lin(C12, Z, 1, C12, b)          # 5  C12 = P5 + b C12
            self.sub(X, X, A11)                  # 6  S2
            self.sub(Y, B22, Y)                  # 7  T2
            self.t1(A11, B11, Z, a, lev - 1)     # 8  P1 = a A11 B11
            self.lin(C11, Z, 1, C11, b)          # 9  C11 = P1 + b C11
            self.hl(X, Y, Z, a, 1, lev - 1)      # 10 U2 = a S2 T2 + P1
            self.hl(A12, B21, C11, a, 1, lev - 1)  # 11 U1 = a A12 B21 + C11
            self.sub(X, A12, X)                  # 12 S4
            self.sub(Y, Y, B21)                  # 13 T4
            self.hl(X, B22, C12, a, 1, lev - 1)  # 14 C12 = a S4 B22 + C12
            self.add(C12, Z, C12)                # 15 U5 = U2 + C12
            self.hl(A22, Y, C21, a, -b, lev - 1)  # 16 C21 = a A22 T4 - b C21
            self.sub(X, A11, A21)                # 17 S3
            self.sub(Y, B22, B12)                # 18 T3
            self.hl(X, Y, Z, a, 1, lev - 1)      # 19 U3 = a S3 T3 + U2
            self.add(C22, Z, C22)                # 20 U7 = U3 + C22
            self.sub(C21, Z, C21)                # 21 U6 = U3 - C21

    # ---------------------------------------------------------- Table 3 (IP)
    def ip(self, A, B, C, a, lev):
        """Table 3: C <- a*A*B with no temporary; overwrites A and B."""
        self.calls["ip"] += 1
        if lev == 0:
            self.leaf(A, B, C, a, 0, False)
            self.destroy(A, B)
            return
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        self.sub(C11, A11, A21)                  # 1  S3
        self.add(A21, A21, A22)                  # 2  S1
        self.sub(C22, B12, B11)                  # 3  T1
        self.sub(B12, B22, B12)                  # 4  T3
        self.ip(C11, B12, C21, a, lev - 1)       # 5  P7 = S3 T3
        self.sub(C12, A21, A11)                  # 6  S2 = S1 - A11
        self.ip(A11, B11, C11, a, lev - 1)       # 7  P1
        self.sub(B11, B22, C22)                  # 8  T2 = B22 - T1
        self.ip(A21, C22, A11, a, lev - 1)       # 9  P5 = S1 T1
        self.sub(C22, B11, B21)                  # 10 T4 = T2 - B21
        self.ip(A22, C22, A21, a, lev - 1)       # 11 P4 = A22 T4
        self.sub(A22, A12, C12)                  # 12 S4 = A12 - S2
        self.ip(C12, B11, C22, a, lev - 1)       # 13 P6 = S2 T2
        self.add(C22, C11, C22)                  # 14 U2 = P1 + P6
        self.ip(A12, B21, C12, a, lev - 1)       # 15 P2
        self.add(C11, C11, C12)                  # 16 U1 = P1 + P2
        self.add(C12, C22, A11)                  # 17 U4 = U2 + P5
        self.add(C22, C22, C21)                  # 18 U3 = U2 + P7
        self.sub(C21, C22, A21)                  # 19 U6 = U3 - P4
        self.add(C22, C22, A11)                  # 20 U7 = U3 + P5
        self.ip(A22, B22, A12, a, lev - 1)       # 21 P3 = S4 B22
        self.add(C12, C12, A12)                  # 22 U5 = U4 + P3
        self.destroy(A, B)

    # --------------------------------------------------------- Table 4 (OvL)
    def ovl(self, A, B, C, a, lev):
        """Table 4: C <- a*A*B with one temporary X ((n/2)^2); overwrites A."""
        self.calls["ovl"] += 1
        if lev == 0:
            self.leaf(A, B, C, a, 0, False)
            self.destroy(A)
            return
        n = C.shape[0]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((n // 2, n // 2)) as (X,):
            self.sub(C22, A11, A21)              # 1  S3
            self.add(A21, A21, A22)              # 2  S1
            self.sub(C12, A21, A11)              # 3  S2 = S1 - A11
            self.sub(C21, B12, B11)              # 4  T1
            self.ovl(A11, B11, C11, a, lev - 1)  # 5  P1
            self.sub(A11, B22, B12)              # 6  T3
            self.ip(C22, A11, X, a, lev - 1)     # 7  P7 = S3 T3
            self.sub(A11, B22, C21)              # 8  T2 = B22 - T1
            self.ip(A21, C21, C22, a, lev - 1)   # 9  P5 = S1 T1
            self.sub(C21, A12, C12)              # 10 S4 = A12 - S2
            self.ovl(C21, B22, A21, a, lev - 1)  # 11 P3 = S4 B22
            self.ovl(C12, A11, C21, a, lev - 1)  # 12 P6 = S2 T2
            self.sub(A11, A11, B21)              # 13 T4 = T2 - B21
            self.add(C21, C11, C21)              # 14 U2 = P1 + P6
            self.add(C12, C21, C22)              # 15 U4 = U2 + P5
            self.add(C21, C21, X)                # 16 U3 = U2 + P7
            self.add(C22, C21, C22)              # 17 U7 = U3 + P5
            self.add(C12, C12, A21)              # 18 U5 = U4 + P3
            self.ovl(A12, B21, X, a, lev - 1)    # 19 P2
            self.add(C11, C11, X)                # 20 U1 = P1 + P2
            self.ip(A22, A11, A21, a, lev - 1)   # 21 P4 = A22 T4
            self.sub(C21, C21, A21)              # 22 U6 = U3 - P4
        self.destroy(A)

    # --------------------------------------------------------- Table 5 (OvR)
    def ovr(self, A, B, C, a, lev):
        """Table 5: C <- a*A*B with one temporary X ((n/2)^2); overwrites B."""
        self.calls["ovr"] += 1
        if lev == 0:
            self.leaf(A, B, C, a, 0, False)
            self.destroy(B)
            return
        n = C.shape[0]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((n // 2, n // 2)) as (X,):
            self.sub(C22, A11, A21)              # 1  S3
            self.add(C21, A21, A22)              # 2  S1
            self.sub(C12, B12, B11)              # 3  T1
            self.ovr(A11, B11, C11, a, lev - 1)  # 4  P1
            self.sub(B11, C21, A11)              # 5  S2 = S1 - A11
            self.sub(B12, B22, B12)              # 6  T3
            self.ip(C22, B12, X, a, lev - 1)     # 7  P7 = S3 T3
            self.sub(B12, B22, C12)              # 8  T2 = B22 - T1
            self.ip(C21, C12, C22, a, lev - 1)   # 9  P5 = S1 T1
            self.sub(C12, B12, B21)              # 10 T4 = T2 - B21
            self.ovr(B11, B12, C21, a, lev - 1)  # 11 P6 = S2 T2
            self.ovr(A22, C12, B12, a, lev - 1)  # 12 P4 = A22 T4
            self.sub(B11, A12, B11)              # 13 S4 = A12 - S2
            self.add(C21, C11, C21)              # 14 U2 = P1 + P6
            self.add(C12, C21, C22)              # 15 U4 = U2 + P5
            self.add(C21, C21, X)                # 16 U3 = U2 + P7
            self.add(C22, C21, C22)              # 17 U7 = U3 + P5
            self.sub(C21, C21, B12)              # 18 U6 = U3 - P4
            self.ip(B11, B22, B12, a, lev - 1)   # 19 P3 = S4 B22
            self.add(C12, C12, B12)              # 20 U5 = U4 + P3
            self.ovr(A12, B21, B12, a, lev - 1)  # 21 P2
            self.add(C11, C11, B12)              # 22 U1 = P1 + P2
        self.destroy(B)

    # -------------------------------------------------------- Table 6 (AcLR)
    def aclr(self, A, B, C, a, b, lev):
        """Table 6: C <- a*A*B + b*C with two temporaries ((n/2)^2 each);
        overwrites A and B."""
        self.calls["aclr"] += 1
        if lev == 0:
            self.leaf(A, B, C, a, b, True)
            self.destroy(A, B)
            return
        n = C.shape[0]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((n // 2, n // 2), (n // 2, n // 2)) as (X, Y):
            self.sub(C22, C22, C12)                  # 1  Z1
            self.add(X, A21, A22)                    # 2  S1
            self.sub(Y, B12, B11)                    # 3  T1
            self.sub(C21, C21, C22)                  # 4  Z2 = C21 - Z1
            self.sub(B12, B22, B12)                  # 5  T3
            self.sub(A21, A11, A21)                  # 6  S3
            self.aclr(A21, B12, C22, a, b, lev - 1)  # 7  P7 + b Z1
            self.sub(A21, X, A11)                    # 8  S2 = S1 - A11
            self.sub(B12, B22, Y)                    # 9  T2 = B22 - T1
            self.aclr(X, Y, C12, a, b, lev - 1)      # 10 P5 + b C12
            self.ip(A11, B11, Y, a, lev - 1)         # 11 P1
            self.sub(X, B12, B21)                    # 12 T4 = T2 - B21
            self.aclr(A22, X, C21, a, -b, lev - 1)   # 13 P4 - b Z2
            self.sub(A22, A12, A21)                  # 14 S4 = A12 - S2
            self.ip(A21, B12, X, a, lev - 1)         # 15 P6 = S2 T2
            self.aclr(A12, B21, C11, a, b, lev - 1)  # 16 P2 + b C11
            self.add(C11, Y, C11)                    # 17 U1 = P1 + P2
            self.add(X, Y, X)                        # 18 U2 = P1 + P6
            self.add(C22, X, C22)                    # 19 U3 = U2 + P7
            self.add(X, X, C12)                      # 20 U4 = U2 + P5
            self.sub(C21, C22, C21)                  # 21 U6 = U3 - P4
            self.add(C22, C22, C12)                  # 22 U7 = U3 + P5
            self.ip(A22, B22, C12, a, lev - 1)       # 23 P3 = S4 B22
            self.add(C12, X, C12)                    # 24 U5 = U4 + P3
        self.destroy(A, B)

    # -------------------------------------------------------- Table 7 (AccR)
    def accr(self, A, B, C, a, b, lev):
        """Table 7: C <- a*A*B + b*C with two temporaries ((n/2)^2 each);
        overwrites B only."""
        self.calls["accr"] += 1
        if lev == 0:
            self.leaf(A, B, C, a, b, True)
            self.destroy(B)
            return
        n = C.shape[0]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((n // 2, n // 2), (n // 2, n // 2)) as (X, Y):
            self.sub(C22, C22, C12)                  # 1  Z1
            self.sub(X, B12, B11)                    # 2  T1
            self.sub(C21, C21, C22)                  # 3  Z2 = C21 - Z1
            self.sub(B12, B22, B12)                  # 4  T3
            self.sub(Y, A11, A21)                    # 5  S3
            self.accr(Y, B12, C22, a, b, lev - 1)    # 6  P7 + b Z1
            self.add(Y, A21, A22)                    # 7  S1
            self.sub(B12, B22, X)                    # 8  T2 = B22 - T1
            self.accr(Y, X, C12, a, b, lev - 1)      # 9  P5 + b C12
            self.sub(X, B12, B21)                    # 10 T4 = T2 - B21
            self.accr(A22, X, C21, a, -b, lev - 1)   # 11 P4 - b Z2
            self.ovr(A11, B11, X, a, lev - 1)        # 12 P1
            self.accr(A12, B21, C11, a, b, lev - 1)  # 13 P2 + b C11
            self.sub(Y, Y, A11)                      # 14 S2 = S1 - A11
            self.ovr(Y, B12, B21, a, lev - 1)        # 15 P6 = S2 T2
            self.sub(Y, A12, Y)                      # 16 S4 = A12 - S2
            self.add(B21, X, B21)                    # 17 U2 = P1 + P6
            self.add(C22, B21, C22)                  # 18 U3 = U2 + P7
            self.add(B21, B21, C12)                  # 19 U4 = U2 + P5
            self.sub(C21, C22, C21)                  # 20 U6 = U3 - P4
            self.add(C11, X, C11)                    # 21 U1 = P1 + P2
            self.add(C22, C22, C12)                  # 22 U7 = U3 + P5
            self.ip(Y, B22, C12, a, lev - 1)         # 23 P3 = S4 B22
            self.add(C12, B21, C12)                  # 24 U5 = U4 + P3
        self.destroy(B)

    # --------------------------------------------------------- Table 8 (AcR)
    def acr(self, A, B, C, a, b, lev):
        """Table 8: C <- a*A*B + b*C for any even shape with two temporaries,
        X (max(m/2, k/2) x n/2) and Y (m/2 x k/2); overwrites B only; five
        accumulating calls and two Table 1 calls."""
        self.calls["acr"] += 1
        if lev == 0:
            self.leaf(A, B, C, a, b, True)
            self.destroy(B)
            return
        m, k = A.shape
        n = B.shape[1]
        h, kk, w = m // 2, k // 2, n // 2
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((max(h, kk), w), (h, kk)) as (X, Y):
            XT, XP = X[:kk], X[:h]                   # X holding a T block, then a product
            self.sub(C22, C22, C12)                  # 1  Z1
            self.sub(XT, B12, B11)                   # 2  T1
            self.sub(C21, C21, C22)                  # 3  Z2 = C21 - Z1
            self.sub(B12, B22, B12)                  # 4  T3
            self.sub(Y, A11, A21)                    # 5  S3
            self.acr(Y, B12, C22, a, b, lev - 1)     # 6  P7 + b Z1
            self.add(Y, A21, A22)                    # 7  S1
            self.sub(B12, B22, XT)                   # 8  T2 = B22 - T1
            self.acr(Y, XT, C12, a, b, lev - 1)      # 9  P5 + b C12
            self.sub(XT, B12, B21)                   # 10 T4 = T2 - B21
            self.acr(A22, XT, C21, a, -b, lev - 1)   # 11 P4 - b Z2
            self.t1(A11, B11, XP, a, lev - 1)        # 12 P1
            self.acr(A12, B21, C11, a, b, lev - 1)   # 13 P2 + b C11
            self.add(C11, XP, C11)                   # 14 U1 = P1 + P2
            self.sub(Y, Y, A11)                      # 15 S2 = S1 - A11
            self.acr(Y, B12, XP, a, 1, lev - 1)      # 16 U2 = a S2 T2 + P1
            self.add(C22, XP, C22)                   # 17 U3 = U2 + P7
            self.sub(C21, C22, C21)                  # 18 U6 = U3 - P4
            self.add(C22, C22, C12)                  # 19 U7 = U3 + P5
            self.add(XP, XP, C12)                    # 20 U4 = U2 + P5
            self.sub(Y, A12, Y)                      # 21 S4 = A12 - S2
            self.t1(Y, B22, C12, a, lev - 1)         # 22 P3 = S4 B22
            self.add(C12, XP, C12)                   # 23 U5 = U4 + P3
        self.destroy(B)

    # --------------------------------------------------------- Table 9 (Acc)
    def acc(self, A, B, C, a, b, lev):
        """Table 9: C <- a*A*B + b*C with two temporaries ((n/2)^2 each);
        A and B are read only (T2 is formed twice)."""
        self.calls["acc"] += 1
        if lev == 0:
            return self.leaf(A, B, C, a, b, True)
        n = C.shape[0]
        A11, A12, A21, A22 = quads(A)
        B11, B12, B21, B22 = quads(B)
        C11, C12, C21, C22 = quads(C)
        with self.frame((n // 2, n // 2), (n // 2, n // 2)) as (X, Y):
            self.sub(C22, C22, C12)                  # 1  Z1
            self.sub(C12, C12, C21)                  # 2  Z3
            self.add(X, A21, A22)                    # 3  S1
            self.sub(Y, B12, B11)                    # 4  T1
            self.acc(X, Y, C12, a, b, lev - 1)       # 5  P5 + b Z3
            self.sub(X, X, A11)                      # 6  S2
            self.sub(Y, B22, Y)                      # 7  T2
            self.acc(X, Y, C21, a, b, lev - 1)       # 8  P6 + b C21
            self.sub(X, A12, X)                      # 9  S4
            self.lin(C22, C12, 1, C22, b)            # 10 W1 = P5 + b Z1 (+ what C12 holds)
            self.acc(X, B22, C12, a, 1, lev - 1)     # 11 P3 + P5
            self.t1(A11, B11, X, a, lev - 1)         # 12 P1
            self.add(C21, C21, X)                    # 13 U2 = P6 + P1
            self.acc(A12, B21, C11, a, b, lev - 1)   # 14 P2 + b C11
            self.add(C11, X, C11)                    # 15 U1 = P1 + P2
            self.add(C12, C21, C12)                  # 16 U5 = U2 + P3
            self.sub(X, A11, A21)                    # 17 S3
            self.sub(Y, B22, B12)                    # 18 T3
            self.aclr(X, Y, C21, a, 1, lev - 1)      # 19 U3 = a S3 T3 + U2
            self.add(C22, C21, C22)                  # 20 U7 = U3 + W1
            self.sub(Y, B12, B11)                    # 21 T1'
            self.sub(Y, B22, Y)                      # 22 T2'
            self.sub(Y, Y, B21)                      # 23 T4
            self.accr(A22, Y, C21, -a, 1, lev - 1)   # 24 U6 = U3 - a A22 T4

    # ------------------------------------------------------ Algorithm 2 (IPMM)
    def ipmm(self, A, B, C, a, L, d=0, acc_base=False):
        """Algorithm 2: C <- a*A*B with no extra memory and A, B read only.
        The three quadrant products run as Table 1 (first inner chunk) and
        Table 2 (remaining chunks; Table 9 with ``acc_base``) calls whose
        temporaries live in C22; C22 itself is then computed by the same
        algorithm."""
        self.calls["ipmm"] += 1
        s = C.shape[0]
        k = A.shape[1]
        if d == L or s < 2 or k == 0:
            return self.leaf(A, B, C, a, 0, False)
        h = s // 2
        K = min(h, k)
        accumulate = self.acc if acc_base else self.hl
        if k % K:
            raise AssertionError("inner dimension is not a multiple of the chunk")
        C11, C12, C21, C22 = quads(C)
        A1, A2 = A[:h], A[h:]
        B1, B2 = B[:, :h], B[:, h:]
        lev = L - d
        self._regions.append(C22)
        try:
            for i in range(k // K):
                a1 = A1[:, i * K:(i + 1) * K]
                a2 = A2[:, i * K:(i + 1) * K]
                b1 = B1[i * K:(i + 1) * K]
                b2 = B2[i * K:(i + 1) * K]
                if i == 0:
                    self.t1(a1, b1, C11, a, lev)
                    self.t1(a1, b2, C12, a, lev)
                    self.t1(a2, b1, C21, a, lev)
                else:
                    accumulate(a1, b1, C11, a, 1, lev)
                    accumulate(a1, b2, C12, a, 1, lev)
                    accumulate(a2, b1, C21, a, 1, lev)
        finally:
            self._regions.pop()
        self.ipmm(A2, B2, C22, a, L, d + 1, acc_base)

    # ------------------------------------------------------ Algorithm 1 (IP0vMM)
    def ip0vmm(self, A, B, C, a, lev):
        """Algorithm 1 and the cutting into squares around it: C <- a*A*B with
        no extra memory, n = min(m, k, n) dividing m and k.  Overwrites A (and
        B when m = n); temporaries live in C_2 and then in the freed A_11."""
        self.calls["ip0vmm"] += 1
        m, k = A.shape
        s = B.shape[1]
        m0, k0 = m // s, k // s
        Ab = lambda i, j: A[i * s:(i + 1) * s, j * s:(j + 1) * s]
        Bb = lambda j: B[j * s:(j + 1) * s]
        Cb = lambda i: C[i * s:(i + 1) * s]
        if m0 == 1:
            self.ip(Ab(0, 0), Bb(0), Cb(0), a, lev)
            self._regions.append(Ab(0, 0))
            try:
                for j in range(1, k0):
                    self.aclr(Ab(0, j), Bb(j), Cb(0), a, 1, lev)
            finally:
                self._regions.pop()
            return
        self._regions.append(Cb(1))
        try:
            self.t1(Ab(0, 0), Bb(0), Cb(0), a, lev)
        finally:
            self._regions.pop()
        self.destroy(Ab(0, 0))
        self._regions.append(Ab(0, 0))
        try:
            for i in range(1, m0):
                self.ovl(Ab(i, 0), Bb(0), Cb(i), a, lev)
            for j in range(1, k0):
                for i in range(m0):
                    self.hl(Ab(i, j), Bb(j), Cb(i), a, 1, lev)
        finally:
            self._regions.pop()

    # --------------------------------------- Section 7.2 (blocked accumulation)
    def blocked(self, core, A, B, C, a, b, t, L):
        """Section 7.2: C <- a*A*B + b*C as a t x t grid of blocks; block C_ij
        receives the t products A_il B_lj one after the other, each by one
        accumulating call of ``core`` (Table 2 or Table 9) with depth L.  The
        calls run one at a time, so the extra memory is that of one call on
        an (n/t)-sized block."""
        self.calls["blocked"] += 1
        m, k = A.shape
        n = B.shape[1]
        ri, kl, cj = (_offsets(blocked_parts(d, t, L)) for d in (m, k, n))
        kl = kl or [(0, 0)]             # k == 0: one empty product still scales C by b
        for i0, i1 in ri:
            for j0, j1 in cj:
                Cij = C[i0:i1, j0:j1]
                for l, (l0, l1) in enumerate(kl):
                    bl = b if l == 0 else 1
                    self.peeled(lambda A0, B0, C0, bl=bl: core(A0, B0, C0, a, bl, L),
                                A[i0:i1, l0:l1], B[l0:l1, j0:j1], Cij, a, bl, L, True)

    # ------------------------------------------------------------ peeling
    def peeled(self, core, A, B, C, a, b, L, accumulate):
        """Winograd on the largest leading block whose dimensions are multiples
        of 2**L; the thin remainders are classical products (Section 8's
        remark on peeling).  ``core(A0, B0, C0)`` runs the schedule."""
        m, k = A.shape
        n = B.shape[1]
        q = 2 ** L
        m0, k0, n0 = m - m % q, k - k % q, n - n % q
        if min(m0, k0, n0) == 0:
            return self.leaf(A, B, C, a, b, accumulate)
        core(A[:m0, :k0], B[:k0, :n0], C[:m0, :n0])
        if k0 < k:
            self.leaf(A[:m0, k0:], B[k0:, :n0], C[:m0, :n0], a, 1, True)
        if n0 < n:
            self.leaf(A[:m0, :], B[:, n0:], C[:m0, n0:], a, b, accumulate)
        if m0 < m:
            self.leaf(A[m0:, :], B, C[m0:, :], a, b, accumulate)


class Result:
    def __init__(self, C, A, B, w):
        self.C, self.A, self.B = C, A, B
        self.adds = w.adds
        self.leaf_ops = w.leaf_ops
        self.leaf_calls = w.leaf_calls
        self.ops = w.adds + w.leaf_ops
        self.peak = w.peak
        self.allocated = w.allocated
        self.calls = dict(w.calls)
        self.max_partial = w.max_partial


def blocked_parts(d, t, L):
    """Lengths of the t consecutive parts of a dimension of length d in the
    blocked accumulation of Section 7.2: d/t each when t divides d, otherwise
    ceil(d/t) rounded up to a multiple of 2**L with a shorter last part (and
    fewer parts when d is small)."""
    if d == 0:
        return []
    if d % t == 0:
        return [d // t] * t
    q = 2 ** L
    s = -(-d // t)
    s = -(-s // q) * q
    parts = []
    while d > 0:
        parts.append(min(s, d))
        d -= s
    return parts


def _offsets(parts):
    out, o = [], 0
    for x in parts:
        out.append((o, o + x))
        o += x
    return out


def ip0vmm_shape_ok(m, k, n, L):
    """Shapes Algorithm 1 (with the cutting into n x n squares) runs at depth L."""
    return n > 0 and n <= min(m, k) and m % n == 0 and k % n == 0 and n % (2 ** L) == 0


def ipmm_shape_ok(m, k, n, L):
    """Shapes Algorithm 2 can run with depth L under the chunking above."""
    if m != n or L < 0:
        return False
    s = n
    for d in range(L):
        if s % 2:
            return False
        h = s // 2
        K = min(h, k)
        q = 2 ** (L - d)
        if K == 0 or k % K or h % q or K % q:
            return False
        s = h
    return True


def _check(schedule, m, k, n, p, beta, L, t=2):
    if schedule not in SCHEDULES:
        raise ValueError("unknown schedule %r" % (schedule,))
    if schedule in ("blocked", "blocked_acc") and not 1 <= t <= 64:
        raise ValueError("the block count t must lie in [1, 64]")
    if schedule == "blocked_acc" and (not (m == k == n) or n % t):
        raise ValueError("blocked accumulation over Table 9 needs m == k == n divisible by t")
    if beta % p and schedule in ("t1", "ip", "ovr", "ipmm"):
        raise ValueError("schedule %s computes C = A*B only (beta must be 0)" % schedule)
    if schedule in ("ip", "ovr", "aclr", "accr"):
        if not (m == k == n) or m % (2 ** L):
            raise ValueError("schedule %s needs a square shape divisible by 2**levels"
                             % schedule)
    if schedule == "acc" and not (m == k == n):
        raise ValueError("schedule acc needs a square shape")
    if schedule in ("ipmm", "ipmm_acc") and not ipmm_shape_ok(m, k, n, L):
        raise ValueError("shape not supported by ipmm at this depth")
    if schedule == "ipmm_acc" and 2 * k < n:
        raise ValueError("Table 9 inside Algorithm 2 needs square chunks (k >= n/2)")
    if beta % p and schedule in ("ovl", "ip0vmm", "ipmm_acc"):
        raise ValueError("schedule %s computes C = A*B only (beta must be 0)" % schedule)
    if schedule == "ovl" and (not (m == k == n) or m % (2 ** L)):
        raise ValueError("schedule ovl needs a square shape divisible by 2**levels")
    if schedule == "acr" and (m % (2 ** L) or k % (2 ** L) or n % (2 ** L)):
        raise ValueError("schedule acr needs every dimension divisible by 2**levels")
    if schedule == "ip0vmm" and not ip0vmm_shape_ok(m, k, n, L):
        raise ValueError("schedule ip0vmm needs n = min(m, k, n) dividing m and k, "
                         "and divisible by 2**levels")


def _run(w, schedule, A, B, C, a, b, L, t=2):
    m, k = A.shape
    n = B.shape[1]
    p = w.p
    if schedule == "classical" or m == 0 or n == 0:
        w.leaf(A, B, C, a, b, bool(b % p))
    elif schedule == "t1":
        w.peeled(lambda A0, B0, C0: w.t1(A0, B0, C0, a, L), A, B, C, a, 0, L, False)
    elif schedule == "hl":
        w.peeled(lambda A0, B0, C0: w.hl(A0, B0, C0, a, b, L), A, B, C, a, b, L, True)
    elif schedule == "acc":
        w.peeled(lambda A0, B0, C0: w.acc(A0, B0, C0, a, b, L), A, B, C, a, b, L, True)
    elif schedule == "ip":
        w.ip(A, B, C, a, L)
    elif schedule == "ovr":
        w.ovr(A, B, C, a, L)
    elif schedule == "aclr":
        w.aclr(A, B, C, a, b, L)
    elif schedule == "accr":
        w.accr(A, B, C, a, b, L)
    elif schedule == "ipmm":
        w.ipmm(A, B, C, a, L)
    elif schedule == "ovl":
        w.ovl(A, B, C, a, L)
    elif schedule == "acr":
        w.acr(A, B, C, a, b, L)
    elif schedule == "ip0vmm":
        w.ip0vmm(A, B, C, a, L)
    elif schedule == "ipmm_acc":
        w.ipmm(A, B, C, a, L, acc_base=True)
    elif schedule == "blocked":
        w.blocked(w.hl, A, B, C, a, b, t, L)
    elif schedule == "blocked_acc":
        w.blocked(w.acc, A, B, C, a, b, t, L)


def replay(schedule, A, B, C=None, alpha=1, beta=0, p=65521, levels=1, *,
           garbage_seed=None, kc=None, blocks=2):
    """Run ``schedule`` on copies of the inputs; return a :class:`Result`.

    schedule: one of SCHEDULES.  'classical' is the plain product;
    't1', 'hl' and 'acc' peel remainders ('t1' and 'hl' also take
    rectangular shapes); 'ip', 'ovr', 'aclr', 'accr' need a square shape
    divisible by 2**levels; 'ipmm' needs a square C (see ipmm_shape_ok);
    'blocked' and 'blocked_acc' cut every dimension into ``blocks`` parts
    ('blocked_acc' needs a square shape divisible by ``blocks``)."""
    p = int(p)
    w = Winograd(p, garbage_seed=garbage_seed, kc=kc)
    A = np.array(A, dtype=np.int64, copy=True)
    B = np.array(B, dtype=np.int64, copy=True)
    m, k = A.shape
    n = B.shape[1]
    if C is None:
        C = np.zeros((m, n), dtype=np.int64)
        beta = 0
    else:
        C = np.array(C, dtype=np.int64, copy=True)
    _check(schedule, m, k, n, p, int(beta), int(levels), int(blocks))
    if int(beta) % p == 0:
        w._garbage(C)                   # C is output only: its content is garbage
    _run(w, schedule, A, B, C, int(alpha), int(beta), int(levels), int(blocks))
    return Result(C, A, B, w)


def replay_shape(schedule, m, k, n, p=65521, levels=1, beta_nonzero=False, blocks=2):
    """Follow ``schedule`` on shapes only (no arithmetic): counts and memory."""
    p = int(p)
    w = Winograd(p, dry=True)
    beta = 1 if beta_nonzero else 0
    _check(schedule, m, k, n, p, beta, int(levels), int(blocks))

    def shaped(r, c):
        return np.lib.stride_tricks.as_strided(np.zeros(1, np.int64), (r, c), (0, 0))

    _run(w, schedule, shaped(m, k), shaped(k, n), shaped(m, n), 1, beta, int(levels),
         int(blocks))
    return Result(None, None, None, w)
