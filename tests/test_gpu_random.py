"""GPU parity on a seeded random sweep: every schedule selector, random shapes
(ragged ones where the schedule peels), depths, moduli, alpha and beta, both
storage types and, where its bounds allow, the 8-bit digit base.  The product is compared with oracle O1 element by element, and
the inputs an overwriting schedule leaves behind with oracle O2's replay."""
import numpy as np
import pytest

from oracle import ref
from oracle.schedules import blocked_parts, ip0vmm_shape_ok, ipmm_shape_ok, replay
from paper_0707_2347_amd import capi, inputs

from .gpu_util import call

pytestmark = pytest.mark.gpu

PRIMES = [3, 257, 65521, 1048573, 8388593, 16777213]
ORACLE = {capi.WS_OVR: "ovr", capi.WS_ACCR: "accr", capi.WS_OVL: "ovl", capi.WS_ACR: "acr"}


def _case(rng):
    """One admissible (schedule, m, k, n, levels, beta, blocks, p, oracle name);
    whether the product accumulates is decided by beta mod p, as the library
    decides it."""
    while True:
        p = int(rng.choice(PRIMES))
        sched = int(rng.choice([capi.WS_CLASSICAL, capi.WS_TWO_TEMP, capi.WS_OVERWRITE,
                                capi.WS_READONLY_INPLACE, capi.WS_HL_THREE_TEMP, capi.WS_OVR,
                                capi.WS_ACCR, capi.WS_BLOCKED, capi.WS_BLOCKED_ACC, capi.WS_OVL,
                                capi.WS_ACR, capi.WS_IPMM_ACC]))
        L = int(rng.integers(0, 4))
        q = 2 ** L
        beta = int(rng.integers(0, 2)) * int(rng.integers(1, 1 << 30))
        acc = beta % p != 0
        t = int(rng.integers(1, 5))
        dims = [int(x) for x in rng.integers(1, 260, size=3)]
        if sched in (capi.WS_OVR, capi.WS_OVL, capi.WS_ACCR) or (
                sched == capi.WS_OVERWRITE and rng.random() < 0.4):
            n = q * int(rng.integers(1, max(2, 256 // q)))
            m = k = n
        elif sched == capi.WS_OVERWRITE:
            if acc:
                m, k, n = (q * int(rng.integers(1, max(2, 256 // q))) for _ in range(3))
            else:
                n = q * int(rng.integers(1, max(2, 128 // q)))
                m, k = n * int(rng.integers(1, 4)), n * int(rng.integers(1, 4))
        elif sched == capi.WS_ACR:
            m, k, n = (q * int(rng.integers(1, max(2, 256 // q))) for _ in range(3))
        elif sched in (capi.WS_READONLY_INPLACE, capi.WS_IPMM_ACC):
            n = 2 * q * int(rng.integers(1, max(2, 128 // q)))
            m = n
            k = (n // 2) * int(rng.integers(1, 4))
        elif sched in (capi.WS_TWO_TEMP, capi.WS_BLOCKED_ACC) and acc:
            m = k = n = dims[0] if sched == capi.WS_TWO_TEMP else t * int(rng.integers(1, 80))
        else:
            m, k, n = dims
        if sched in (capi.WS_OVR, capi.WS_OVL, capi.WS_READONLY_INPLACE, capi.WS_IPMM_ACC):
            beta, acc = 0, False
        if sched == capi.WS_OVERWRITE and not (m == k == n) and not acc and \
                not ip0vmm_shape_ok(m, k, n, L):
            continue
        if sched in (capi.WS_READONLY_INPLACE, capi.WS_IPMM_ACC) and not ipmm_shape_ok(m, k, n, L):
            continue
        if sched == capi.WS_BLOCKED_ACC and (not (m == k == n) or n % t):
            continue
        if sched == capi.WS_BLOCKED and not blocked_parts(m, t, L):
            continue
        name = ORACLE.get(sched)
        if sched == capi.WS_OVERWRITE:
            name = ("aclr" if acc else "ip") if m == k == n else ("acr" if acc else "ip0vmm")
        return sched, m, k, n, L, beta, t, p, name


CASES = [_case(np.random.default_rng([77, i])) + (i,) for i in range(300)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "s%d_%dx%dx%d_l%d_b%d" % (
    c[0], c[1], c[2], c[3], c[4], int(c[5] != 0)))
def test_random_case(case):
    sched, m, k, n, L, beta, t, p, name, i = case
    rng = np.random.default_rng([78, i])
    dtype = capi.WS_I64 if i % 3 == 0 else capi.WS_F64
    base = (capi.WS_BASE_I8_LIMBS if i % 4 == 1 and p <= 16711423 and k <= 32768
            else capi.WS_BASE_F64_MFMA)
    alpha = int(rng.integers(-(1 << 40), 1 << 40))
    print("random case", i, sched, (m, k, n), L, beta, t, p, dtype, base, flush=True)
    A, B, C = inputs.uniform(900 + i, m, k, n, p, with_c=True)
    st, C2, A2, B2 = call(sched, A, B, C, alpha, beta, p, L, dtype=dtype, base=base, blocks=t)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p))
    if name is not None:
        r = replay(name, A, B, C, alpha, beta, p, L)
        assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    else:
        assert np.array_equal(A2, A) and np.array_equal(B2, B)


def _digit_case(rng):
    """A schedule on the 8-bit digit base at shapes whose blocks are whole
    128 x 64 tiles at the leaves, where temporaries and input quadrants are
    held as digit planes (sizes up to 1024, so the oracle stays quick)."""
    while True:
        p = int(rng.choice([3, 257, 65521, 65537, 1048573, 8388593, 16711421]))
        sched = int(rng.choice([capi.WS_TWO_TEMP, capi.WS_HL_THREE_TEMP, capi.WS_OVERWRITE,
                                capi.WS_ACCR, capi.WS_ACR, capi.WS_OVR, capi.WS_OVL,
                                capi.WS_READONLY_INPLACE]))
        L = int(rng.integers(1, 3))
        q = 128 << L
        beta = int(rng.integers(0, 2)) * int(rng.integers(1, 1 << 30))
        if sched in (capi.WS_OVR, capi.WS_OVL, capi.WS_READONLY_INPLACE):
            beta = 0
        acc = beta % p != 0
        square = sched in (capi.WS_OVR, capi.WS_OVL, capi.WS_ACCR) or \
            (sched == capi.WS_TWO_TEMP and acc) or (sched == capi.WS_OVERWRITE and acc)
        dims = [q * int(rng.integers(1, 1024 // q + 1)) for _ in range(3)]
        m, k, n = (dims[0],) * 3 if square else dims
        if sched == capi.WS_READONLY_INPLACE:
            m = n = dims[0]
            k = dims[1]
            if not ipmm_shape_ok(m, k, n, L):
                continue
        if sched == capi.WS_OVERWRITE and not acc and not (m == k == n) and \
                not ip0vmm_shape_ok(m, k, n, L):
            continue
        name = ORACLE.get(sched)
        if sched == capi.WS_OVERWRITE:
            name = ("aclr" if acc else "ip") if m == k == n else ("acr" if acc else "ip0vmm")
        return sched, m, k, n, L, beta, p, name


DIGIT_CASES = [_digit_case(np.random.default_rng([79, i])) + (i,) for i in range(60)]


@pytest.mark.parametrize("case", DIGIT_CASES, ids=lambda c: "d%d_%dx%dx%d_l%d_b%d" % (
    c[0], c[1], c[2], c[3], c[4], int(c[5] != 0)))
def test_random_digit_case(case):
    sched, m, k, n, L, beta, p, name, i = case
    rng = np.random.default_rng([80, i])
    dtype = capi.WS_I64 if i % 2 else capi.WS_F64
    alpha = int(rng.integers(-(1 << 40), 1 << 40))
    print("random digit case", i, sched, (m, k, n), L, beta, p, dtype, flush=True)
    A, B, C = inputs.uniform(1900 + i, m, k, n, p, with_c=True)
    st, C2, A2, B2 = call(sched, A, B, C, alpha, beta, p, L, dtype=dtype,
                          base=capi.WS_BASE_I8_LIMBS)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p))
    if name is not None:
        r = replay(name, A, B, C, alpha, beta, p, L)
        assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    else:
        assert np.array_equal(A2, A) and np.array_equal(B2, B)
