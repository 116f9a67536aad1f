"""Host-side checks of the digit base's execution list (no GPU).

On the 8-bit digit base the library runs a plan's operations with some
workspace temporaries held as digit planes instead of residues (their view's
form, include/wsmul.h).  wsmul_plan_export returns that list for the digit
base; the numpy stand-in (tests/plan_interp.py) runs it with every
digit-plane block overwritten by a non-residue while the values are kept
aside, so a residue read of such a block, a planes read of a block nobody
encoded, a group rewriting a view in another form, or a planes view the
device could not lay out fails.  The result must equal the oracle and the
final inputs the oracle's replay.
"""
import os

import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay
from paper_0707_2347_amd import capi, inputs

from . import plan_interp

pytestmark = pytest.mark.skipif(not os.path.exists(capi.LIB_PATH),
                                reason="libwsmul.so not built")
I8 = capi.WS_BASE_I8_LIMBS

REPLAY = {
    (capi.WS_TWO_TEMP, False): "t1", (capi.WS_TWO_TEMP, True): "acc",
    (capi.WS_OVERWRITE, False): "ip", (capi.WS_OVERWRITE, True): "aclr",
    (capi.WS_HL_THREE_TEMP, True): "hl", (capi.WS_HL_THREE_TEMP, False): "hl",
    (capi.WS_ACCR, True): "accr", (capi.WS_ACR, True): "acr",
    (capi.WS_READONLY_INPLACE, False): "ipmm",
}


def _export(schedule, m, k, n, p, alpha, beta, levels, base=I8, flags=0):
    args = capi.make_args(m, k, n, p, alpha=alpha, beta=beta, schedule=schedule,
                          levels=levels, base=base, flags=flags)
    return capi.wsmul_plan_info(args), capi.wsmul_plan_export(args)


def _forms(ops):
    views = []
    for op in ops:
        views += [op.in_[i] for i in range(op.nin)] + [op.out[o] for o in range(op.nout)]
        if op.kind == capi.WS_OP_GEMM:
            views += [op.a, op.b]
    return sum(1 for v in views if v.form)


CASES = [
    # schedule, (m, k, n), levels, accumulate, digit forms expected
    (capi.WS_TWO_TEMP, (256, 256, 256), 1, False, True),
    (capi.WS_TWO_TEMP, (512, 512, 512), 2, False, True),
    (capi.WS_TWO_TEMP, (1024, 1024, 1024), 3, False, True),
    (capi.WS_TWO_TEMP, (512, 256, 384), 1, False, True),
    (capi.WS_TWO_TEMP, (384, 512, 256), 1, False, True),
    (capi.WS_TWO_TEMP, (320, 320, 320), 1, False, False),     # 160-row blocks: no whole tiles
    (capi.WS_TWO_TEMP, (512, 512, 512), 2, True, True),
    (capi.WS_TWO_TEMP, (256, 256, 256), 1, True, True),
    (capi.WS_HL_THREE_TEMP, (512, 512, 512), 1, True, True),
    (capi.WS_HL_THREE_TEMP, (512, 512, 512), 2, True, True),
    (capi.WS_HL_THREE_TEMP, (512, 384, 256), 1, True, True),
    (capi.WS_HL_THREE_TEMP, (512, 512, 512), 1, False, True),
    (capi.WS_OVERWRITE, (512, 512, 512), 1, True, True),
    (capi.WS_OVERWRITE, (512, 512, 512), 2, True, True),
    (capi.WS_OVERWRITE, (512, 512, 512), 2, False, False),    # Table 3: no temporaries
    (capi.WS_ACCR, (512, 512, 512), 1, True, True),
    (capi.WS_ACR, (512, 512, 512), 1, True, True),
    (capi.WS_ACR, (512, 256, 768), 1, True, True),
    (capi.WS_READONLY_INPLACE, (512, 512, 512), 1, False, False),
]


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("schedule,shape,levels,acc,digits", CASES)
def test_execution_list_reproduces_oracle(schedule, shape, levels, acc, digits, fuse):
    m, k, n = shape
    p = 1048573 if levels % 2 else 16711421
    alpha, beta = (3, p - 5) if acc else (p - 1, 0)
    seed = m + 3 * k + 7 * n + levels
    A, B, C = inputs.uniform(seed, m, k, n, p, with_c=True)
    info, ops = _export(schedule, m, k, n, p, alpha, beta, levels,
                        flags=0 if fuse else capi.WS_FLAG_NOFUSE)
    assert (_forms(ops) > 0) == digits
    rng = np.random.default_rng(seed)
    W = rng.integers(0, p, size=max(info.workspace_bytes // 8, 1))
    Cg = C.copy() if beta else rng.integers(0, p, size=(m, n))
    bufs = [A.copy().ravel(), B.copy().ravel(), Cg.ravel().copy(), W]
    plan_interp.run(ops, bufs, p)
    assert np.array_equal(bufs[2].reshape(m, n), ref.matmul_mod_p(A, B, C, alpha, beta, p))
    r = replay(REPLAY[(schedule, acc)], A, B, C, alpha, beta, p, levels)
    assert np.array_equal(bufs[0].reshape(m, k), r.A) and np.array_equal(bufs[1].reshape(k, n), r.B)


def test_table1_execution_list():
    """Table 1, one level: every temporary is held as digit planes.  S and T
    blocks are written as planes by the pre-additions (T4 by a group moved
    out of P1's epilogue); the quadrants of A and B are read from planes of
    the whole inputs, split once, by the pre-additions and by the products.
    P1's epilogue (four inputs, three outputs besides P1 itself) moves into a
    group of residues right after it that reads P1 back from X."""
    info, ops = _export(capi.WS_TWO_TEMP, 512, 512, 512, 65521, 1, 0, 1)
    _, plain = _export(capi.WS_TWO_TEMP, 512, 512, 512, 65521, 1, 0, 1,
                       base=capi.WS_BASE_F64_MFMA)
    assert len(ops) == len(plain) + 2 == 13
    gemms = [op for op in ops if op.kind == capi.WS_OP_GEMM]
    # every operand is read as planes: temporaries in W, input quadrants from
    # the planes of the whole A and B (split once)
    assert [(g.a.form, g.b.form) for g in gemms] == [(1, 2)] * 7
    assert [(g.a.buf, g.b.buf) for g in gemms] == [(3, 3), (3, 3), (3, 3), (3, 1), (0, 1),
                                                   (0, 3), (0, 1)]
    assert all(g.nout == 1 for g in gemms[:5])
    adds = [op for op in ops if op.kind == capi.WS_OP_ADD]
    assert len(adds) == 6
    digit = [op for op in adds if any(op.out[o].form for o in range(op.nout))]
    assert len(digit) == 5
    for op in digit:
        assert all(op.out[o].form for o in range(op.nout))
    after_p1 = ops[ops.index(next(o for o in ops if o.kind == capi.WS_OP_GEMM and
                                  (o.a.buf, o.b.buf) == (0, 1))) + 1]
    assert after_p1.kind == capi.WS_OP_ADD and after_p1.nout == 3 and after_p1.nin == 5
    assert after_p1.in_[0].buf == capi.WS_BUF_W and not any(
        after_p1.in_[i].form for i in range(after_p1.nin))
    # the pre-additions read the input quadrants as planes too
    for op in digit:
        assert all(op.in_[i].form for i in range(op.nin))
    assert _forms(plain) == 0


def test_misplaced_planes_are_caught():
    """The stand-in fails when a block holding planes is read as residues
    (the check the tests above rely on): flip one consumer to residues."""
    _, ops = _export(capi.WS_TWO_TEMP, 256, 256, 256, 65521, 1, 0, 1)
    g = next(op for op in ops if op.kind == capi.WS_OP_GEMM and op.a.form)
    g.a.form = 0
    A, B, _ = inputs.uniform(1, 256, 256, 256, 65521, with_c=True)
    bufs = [A.ravel().copy(), B.ravel().copy(), np.zeros(256 * 256, np.int64),
            np.zeros(2 * 128 * 128, np.int64)]
    with pytest.raises(AssertionError, match="holds digit planes"):
        plan_interp.run(ops, bufs, 65521)


@pytest.mark.parametrize("graph", ["table9", "table2"])
@pytest.mark.parametrize("n,levels", [(256, 1), (512, 2)])
def test_row_schedules_on_the_digit_base(graph, n, levels):
    """Schedules given as rows (the §4 search's, tests/golden/acc_search.json)
    run on the digit base's execution list: same result as the oracle, A and
    B untouched, and digit planes in use."""
    import json
    d = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "acc_search.json")))[graph]
    st, sid = capi.wsmul_register_rows([tuple(r) for r in d["library_rows"]], d["temps"])
    assert st == capi.WS_OK
    p = 1048573
    A, B, C = inputs.uniform(n + levels, n, n, n, p, with_c=True)
    args = capi.make_args(n, n, n, p, alpha=5, beta=p - 7, schedule=capi.WS_ROWS, levels=levels,
                          blocks=sid, base=I8)
    info, ops = capi.wsmul_plan_info(args), capi.wsmul_plan_export(args)
    assert _forms(ops) > 0
    rng = np.random.default_rng(n)
    W = rng.integers(0, p, size=max(info.workspace_bytes // 8, 1))
    bufs = [A.copy().ravel(), B.copy().ravel(), C.copy().ravel(), W]
    plan_interp.run(ops, bufs, p)
    assert np.array_equal(bufs[2].reshape(n, n), ref.matmul_mod_p(A, B, C, 5, p - 7, p))
    assert np.array_equal(bufs[0].reshape(n, n), A) and np.array_equal(bufs[1].reshape(n, n), B)
