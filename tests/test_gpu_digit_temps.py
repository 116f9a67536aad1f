"""GPU parity of the 8-bit digit base when the schedule's temporaries are
held as digit planes.

On the digit base a temporary that is written by an addition group and then
read only by base products (in one operand role) and by addition groups is
kept as the three digit planes the product reads: the addition kernel writes
and decodes them, the product skips that operand's split.  Each case checks
the result element by element against the oracle, that the inputs are left
as the schedule leaves them (untouched, or as the oracle's replay of an
overwriting table leaves them), and (through the trace counters) that the digit
temporaries were used.  Inputs mix uniform residues with the residues whose
centred digits are extreme; the workspace starts as random bytes.
"""
import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay
from paper_0707_2347_amd import capi, inputs

from .gpu_util import to_dev, to_host, torch

pytestmark = pytest.mark.gpu
I8 = capi.WS_BASE_I8_LIMBS


def _extreme(rng, shape, p, base):
    h = (p - 1) // 2
    pick = np.array([h, h + 1, p - 1, 1, 0, 255, p - 256, 65535 % p], dtype=np.int64)
    mask = rng.random(shape) < 0.5
    return np.where(mask, pick[rng.integers(0, len(pick), size=shape)], base)


def _run(schedule, m, k, n, levels, p, alpha, beta, dtype, seed, misalign=False):
    t = torch()
    A, B, C = inputs.uniform(seed, m, k, n, p, with_c=True)
    rng = np.random.default_rng(seed)
    A, B = _extreme(rng, A.shape, p, A), _extreme(rng, B.shape, p, B)
    dA, dB, dC = to_dev(A, dtype), to_dev(B, dtype), to_dev(C, dtype)
    s = t.cuda.current_stream()
    info = capi.wsmul_plan_info(capi.make_args(m, k, n, p, alpha=alpha, beta=beta,
                                               schedule=schedule, levels=levels, dtype=dtype,
                                               base=I8))
    nb = info.workspace_bytes
    g = t.Generator(device="cuda:0")
    g.manual_seed(seed)
    raw = t.randint(-2 ** 62, 2 ** 62, (nb // 8 + 2,), dtype=t.int64, device="cuda:0", generator=g)
    ws = raw[1:] if misalign else raw          # 8 bytes past an aligned base
    wptr = ws.data_ptr()
    assert wptr % 16 == (8 if misalign else 0)
    capi.wsmul_reset_stats()
    args = capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, schedule, levels, dtype=dtype,
                          base=I8, stream=s, flags=capi.WS_FLAG_TRACE, workspace=wptr,
                          workspace_bytes=nb)
    st = capi.wsmul_mod_p_ex(args)
    t.cuda.synchronize()
    assert st == capi.WS_OK, capi.wsmul_last_error()
    return (A, B, C), (to_host(dA), to_host(dB), to_host(dC)), capi.wsmul_get_trace()


CASES = [
    # schedule, (m, k, n), levels, accumulate
    (capi.WS_TWO_TEMP, (512, 512, 512), 1, False),
    (capi.WS_TWO_TEMP, (1024, 1024, 1024), 2, False),
    (capi.WS_TWO_TEMP, (2048, 2048, 2048), 3, False),
    (capi.WS_TWO_TEMP, (1024, 512, 768), 1, False),
    (capi.WS_TWO_TEMP, (768, 1024, 512), 1, False),
    (capi.WS_TWO_TEMP, (1024, 1024, 1024), 2, True),
    (capi.WS_HL_THREE_TEMP, (1024, 1024, 1024), 1, True),
    (capi.WS_HL_THREE_TEMP, (1024, 1024, 1024), 2, True),
    (capi.WS_HL_THREE_TEMP, (1024, 768, 512), 1, True),
    (capi.WS_ACR, (1024, 1024, 1024), 1, True),
    (capi.WS_ACCR, (512, 512, 512), 1, True),
    (capi.WS_OVERWRITE, (1024, 1024, 1024), 1, True),
]
# schedules that leave A or B overwritten: their final state is the replay's
OVERWRITING = {capi.WS_ACR: "acr", capi.WS_ACCR: "accr", capi.WS_OVERWRITE: "aclr"}


@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("p", [65521, 1048573, 16711421])
@pytest.mark.parametrize("schedule,shape,levels,acc", CASES)
def test_digit_temporaries(schedule, shape, levels, acc, p, dtype):
    m, k, n = shape
    print("digit temporaries", schedule, shape, levels, acc, p, dtype, flush=True)
    alpha, beta = (3, p - 2) if acc else (p - 1, 0)
    (A, B, C), (A2, B2, C2), tr = _run(schedule, m, k, n, levels, p, alpha, beta, dtype,
                                       m + 3 * k + 7 * n + levels + p % 1000)
    want = ref.matmul_mod_p(A, B, C, alpha, beta, p)
    bad = np.argwhere(C2 != want)
    assert bad.size == 0, ("first differing entry", bad[0].tolist(), len(bad))
    if schedule in OVERWRITING:
        r = replay(OVERWRITING[schedule], A, B, C, alpha, beta, p, levels)
        assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    else:
        assert np.array_equal(A2, A) and np.array_equal(B2, B)
    assert tr.digit_adds > 0 and tr.unsplit_operands > 0


def test_table1_uses_digits_for_every_temporary():
    """Table 1, one level, at 2048: A and B are split once each, and all 14
    product operands are read as planes (temporaries in W, input quadrants
    from the whole inputs' planes); five addition groups are digit ones
    (S3/T3, S1/T1, S2/T2, S4, and T4 moved out of P1's epilogue) and one,
    P1's post-additions moved after it, runs on residues."""
    p = 1048573
    (A, B, C), (_, _, C2), tr = _run(capi.WS_TWO_TEMP, 2048, 2048, 2048, 1, p, 1, 0,
                                     capi.WS_F64, 11)
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, None, 1, 0, p))
    assert tr.gemm_launches == 7
    assert tr.split_launches == 2 and tr.unsplit_operands == 14
    assert tr.add_launches == 6 and tr.digit_adds == 5


def test_misaligned_workspace_keeps_residues():
    """A workspace that is not 16-byte aligned runs every temporary as
    residues (no digit planes) and gives the same result."""
    p = 65521
    (A, B, C), (_, _, C2), tr = _run(capi.WS_TWO_TEMP, 512, 512, 512, 1, p, 1, 0,
                                     capi.WS_I64, 12, misalign=True)
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, None, 1, 0, p))
    assert tr.digit_adds == 0 and tr.unsplit_operands == 0 and tr.split_launches == 14
