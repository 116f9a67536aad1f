"""GPU parity of the 8-bit digit base (centred residues, balanced base-256
digits, int32 matrix-core sums, recombination mod p) against the oracle."""
import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay
from paper_0707_2347_amd import capi, inputs

from .gpu_util import call

pytestmark = pytest.mark.gpu
I8 = capi.WS_BASE_I8_LIMBS


@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("shape", [(1, 1, 1), (16, 64, 16), (17, 33, 9), (100, 257, 130),
                                   (128, 64, 128), (300, 200, 700), (129, 1000, 255),
                                   (1024, 1024, 1024), (4, 0, 6)])
@pytest.mark.parametrize("p", [3, 251, 65521, 1048573, 8388593, 16711421])
def test_digit_base_classical(shape, dtype, p):
    m, k, n = shape
    print("digits", shape, dtype, p, flush=True)
    A, B, C = inputs.uniform(m * 31 + k * 3 + n + p % 97, m, k, n, p, with_c=True)
    for alpha, beta in [(1, 0), (p - 1, 3 % p)]:
        st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, C, alpha, beta, p, 0, dtype=dtype, base=I8)
        assert st == capi.WS_OK, capi.wsmul_last_error()
        assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p)), (alpha, beta)


@pytest.mark.parametrize("shape", [(64, 4096, 48), (32, 16384, 32), (32, 32768, 32)])
@pytest.mark.parametrize("p", [65521, 1048573, 8388593, 16711421])
def test_digit_extremes(p, shape):
    """Residues whose centred value has the largest digits, up to the longest
    inner dimension the digit base accepts (32768, where a weight class of
    three digit products comes within a factor 1.33 of the int32 range)."""
    m, k, n = shape
    print("digit extremes", shape, p, flush=True)
    h = (p - 1) // 2
    rng = np.random.default_rng(p)
    choices = np.array([h, h + 1, p - 1, 1, 0], dtype=np.int64)
    A = choices[rng.integers(0, 5, size=(m, k))]
    B = choices[rng.integers(0, 5, size=(k, n))]
    st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, None, 1, 0, p, 0, base=I8)
    assert st == capi.WS_OK
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, None, 1, 0, p))
    A[:] = h
    B[:] = h + 1
    st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, None, 1, 0, p, 0, base=I8)
    assert np.all(C2 == (k * h * (h + 1)) % p)


@pytest.mark.parametrize("schedule,shape,levels,acc", [
    (capi.WS_TWO_TEMP, (256, 256, 256), 2, False), (capi.WS_TWO_TEMP, (256, 256, 256), 2, True),
    (capi.WS_OVERWRITE, (256, 256, 256), 2, True), (capi.WS_READONLY_INPLACE, (256, 128, 256), 2, False),
    (capi.WS_TWO_TEMP, (300, 260, 190), 1, False)])
def test_digit_base_schedules(schedule, shape, levels, acc):
    m, k, n = shape
    p = 1048573
    A, B, C = inputs.uniform(99 + levels, m, k, n, p, with_c=True)
    beta = 5 if acc else 0
    st, C2, A2, B2 = call(schedule, A, B, C, 3, beta, p, levels, base=I8)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 3, beta, p))
    if schedule == capi.WS_OVERWRITE:
        r = replay("aclr", A, B, C, 3, beta, p, levels)
        assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    s = capi.wsmul_get_stats()
    assert s.base == I8 and s.scratch_bytes > 0


def test_digit_base_limits():
    import torch
    d = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    a = capi.make_args(1, 40000, 1, 65521, d, d, d, 1, 0, capi.WS_CLASSICAL, 0, base=I8)
    assert capi.wsmul_mod_p_ex(a) == capi.WS_ESHAPE
    a = capi.make_args(1, 1, 1, 16711433, d, d, d, 1, 0, capi.WS_CLASSICAL, 0, base=I8)
    assert capi.wsmul_mod_p_ex(a) == capi.WS_EMODULUS


@pytest.mark.parametrize("p", [257, 65521, 65536, 65537])
@pytest.mark.parametrize("schedule,levels", [(capi.WS_CLASSICAL, 0), (capi.WS_TWO_TEMP, 1)])
def test_two_digit_boundary(p, schedule, levels):
    """p <= 65536 runs on two digits, residues above 32639 taken minus p;
    65537 is the smallest modulus on three.  Entries at the centring
    threshold and at the ends of the range, through the classical product
    and through Table 1 with digit-plane temporaries."""
    m = k = n = 512
    print("two-digit boundary", p, schedule, flush=True)
    h = (p - 1) // 2
    pick = np.array(sorted({0, 1, 255, 256, min(32639, p - 1), min(32640, p - 1), h, h + 1, p - 1}),
                    dtype=np.int64)
    rng = np.random.default_rng(p + levels)
    A = pick[rng.integers(0, len(pick), size=(m, k))]
    B = pick[rng.integers(0, len(pick), size=(k, n))]
    st, C2, _, _ = call(schedule, A, B, None, 1, 0, p, levels, base=I8)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, None, 1, 0, p))
