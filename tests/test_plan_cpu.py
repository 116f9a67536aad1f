"""Host-side checks of the HIP library (no GPU): the C-ABI library loads and
exports every symbol of include/wsmul.h; argument checks return the documented
status codes; the planner's workspace equals each schedule's temporary count
(Eq. (1), Eq. (2), Sections 5-6) and its op list, run by a numpy stand-in,
reproduces the oracle bit for bit, including the final state of inputs the
overwriting schedules destroy."""
import os
import re

import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay, replay_shape
from paper_0707_2347_amd import capi, inputs

from . import plan_interp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(capi.LIB_PATH),
                                reason="libwsmul.so not built")

TABLE_OF = {  # (public schedule, beta != 0) -> oracle schedule
    (capi.WS_CLASSICAL, False): "classical", (capi.WS_CLASSICAL, True): "classical",
    (capi.WS_TWO_TEMP, False): "t1", (capi.WS_TWO_TEMP, True): "acc",
    (capi.WS_OVERWRITE, False): "ip", (capi.WS_OVERWRITE, True): "aclr",
    (capi.WS_READONLY_INPLACE, False): "ipmm",
    (capi.WS_HL_THREE_TEMP, False): "hl", (capi.WS_HL_THREE_TEMP, True): "hl",
    (capi.WS_OVR, False): "ovr", (capi.WS_ACCR, True): "accr",
}


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "wsmul.h")).read()
    names = re.findall(r"WSMUL_API\s+[\w\s\*]*?\b(wsmul_\w+)\s*\(", header)
    assert len(names) >= 14
    lib = capi.lib()
    for name in names:
        assert hasattr(lib, name), name


def test_binding_constants_match_the_header():
    """Every enumerator and size #define of include/wsmul.h has the same
    value in the binding (a kind or schedule added on one side only fails)."""
    header = open(os.path.join(ROOT, "include", "wsmul.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    values = {}
    for name, expr in re.findall(r"\b(WS_[A-Z0-9_]+)\s*=\s*([^,}\n]+)", header):
        expr = expr.strip().replace("1u", "1")
        values[name] = eval(expr, {"__builtins__": {}})
    for name, val in re.findall(r"#define\s+(WS_MAX_\w+)\s+(\d+)", header):
        values[name] = int(val)
    assert len(values) >= 40
    for name, val in values.items():
        assert getattr(capi, name) == val, name


def _interp(schedule, m, k, n, p, alpha, beta, levels, seed, fuse=True, dtype=capi.WS_F64,
            blocks=0):
    A, B, C = inputs.uniform(seed, m, k, n, p, with_c=True)
    args = capi.make_args(m, k, n, p, alpha=alpha, beta=beta, schedule=schedule,
                          levels=levels, dtype=dtype, flags=0 if fuse else capi.WS_FLAG_NOFUSE,
                          blocks=blocks)
    info = capi.wsmul_plan_info(args)
    ops = capi.wsmul_plan_export(args)
    rng = np.random.default_rng(seed + 1)
    W = rng.integers(0, p, size=max(info.workspace_bytes // 8, 1))
    Cg = C.copy() if beta % p else rng.integers(0, p, size=(m, n))   # garbage when beta = 0
    bufs = [A.copy().ravel(), B.copy().ravel(), Cg.ravel().copy(), W]
    plan_interp.run(ops, bufs, p)
    return (A, B, C), (bufs[0].reshape(m, k), bufs[1].reshape(k, n), bufs[2].reshape(m, n)), info


CASES = [
    (capi.WS_CLASSICAL, (33, 47, 29), 0, False),
    (capi.WS_TWO_TEMP, (64, 64, 64), 1, False), (capi.WS_TWO_TEMP, (64, 64, 64), 3, False),
    (capi.WS_TWO_TEMP, (64, 32, 128), 2, False), (capi.WS_TWO_TEMP, (96, 64, 32), 2, False),
    (capi.WS_TWO_TEMP, (37, 50, 29), 2, False), (capi.WS_TWO_TEMP, (45, 45, 45), 3, False),
    (capi.WS_TWO_TEMP, (64, 64, 64), 1, True), (capi.WS_TWO_TEMP, (64, 64, 64), 3, True),
    (capi.WS_TWO_TEMP, (41, 41, 41), 2, True),
    (capi.WS_OVERWRITE, (64, 64, 64), 1, False), (capi.WS_OVERWRITE, (64, 64, 64), 3, False),
    (capi.WS_OVERWRITE, (32, 32, 32), 2, True), (capi.WS_OVERWRITE, (64, 64, 64), 3, True),
    (capi.WS_READONLY_INPLACE, (64, 64, 64), 1, False),
    (capi.WS_READONLY_INPLACE, (64, 64, 64), 3, False),
    (capi.WS_READONLY_INPLACE, (64, 32, 64), 2, False),
    (capi.WS_READONLY_INPLACE, (64, 128, 64), 2, False),
    (capi.WS_HL_THREE_TEMP, (64, 64, 64), 2, True), (capi.WS_HL_THREE_TEMP, (48, 32, 16), 2, True),
    (capi.WS_OVR, (32, 32, 32), 3, False), (capi.WS_ACCR, (32, 32, 32), 3, True),
]


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("schedule,shape,levels,acc", CASES)
def test_plan_reproduces_oracle(schedule, shape, levels, acc, fuse):
    m, k, n = shape
    p = 8388593 if levels % 2 else 65521
    alpha, beta = 5, (7 if acc else 0)
    (A, B, C), (A2, B2, C2), info = _interp(schedule, m, k, n, p, alpha, beta, levels,
                                             seed=m * 7 + k * 3 + n + levels, fuse=fuse)
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p))
    name = TABLE_OF[(schedule, bool(beta))]
    r = replay(name, A, B, C, alpha, beta, p, levels)
    assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    if name not in ("ip", "aclr", "ovr", "accr"):
        assert np.array_equal(A2, A) and np.array_equal(B2, B)
    rs = replay_shape(name, m, k, n, p, levels, beta_nonzero=bool(beta))
    assert info.workspace_bytes == 8 * rs.peak
    assert info.element_additions == rs.adds


BLOCKED = [
    # schedule, shape, levels, t (0 = the default 2), beta
    (capi.WS_BLOCKED, (64, 64, 64), 2, 0, 7), (capi.WS_BLOCKED, (96, 96, 96), 1, 3, 7),
    (capi.WS_BLOCKED, (64, 32, 128), 2, 2, 7), (capi.WS_BLOCKED, (37, 50, 29), 1, 3, 7),
    (capi.WS_BLOCKED, (100, 100, 100), 2, 3, 0), (capi.WS_BLOCKED, (33, 17, 65), 2, 4, 7),
    (capi.WS_BLOCKED, (32, 32, 32), 2, 1, 7), (capi.WS_BLOCKED, (5, 70, 3), 1, 3, 7),
    (capi.WS_BLOCKED_ACC, (64, 64, 64), 2, 2, 7), (capi.WS_BLOCKED_ACC, (96, 96, 96), 2, 3, 7),
    (capi.WS_BLOCKED_ACC, (90, 90, 90), 2, 3, 7), (capi.WS_BLOCKED_ACC, (64, 64, 64), 1, 4, 0),
]


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("schedule,shape,levels,t,beta", BLOCKED)
def test_blocked_plan_reproduces_oracle(schedule, shape, levels, t, beta, fuse):
    """Section 7.2's blocked accumulation: the plan's value, its temporaries
    (one block call's) and its addition count equal the oracle's replay."""
    m, k, n = shape
    p = 8388593 if levels % 2 else 65521
    alpha = 5
    (A, B, C), (A2, B2, C2), info = _interp(schedule, m, k, n, p, alpha, beta, levels,
                                             seed=m * 5 + k + n * 3 + t, fuse=fuse, blocks=t)
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p))
    assert np.array_equal(A2, A) and np.array_equal(B2, B)
    name = "blocked" if schedule == capi.WS_BLOCKED else "blocked_acc"
    rs = replay_shape(name, m, k, n, p, levels, beta_nonzero=True, blocks=t or 2)
    assert info.workspace_bytes == 8 * rs.peak
    assert info.element_additions == rs.adds
    assert capi.wsmul_schedule_name(info.schedule).startswith("section7.2-blocked")


FAMILY = [
    # selector, shape, levels, beta, oracle schedule
    (capi.WS_OVL, (32, 32, 32), 1, 0, "ovl"), (capi.WS_OVL, (64, 64, 64), 3, 0, "ovl"),
    (capi.WS_ACR, (32, 32, 32), 2, 7, "acr"), (capi.WS_ACR, (64, 32, 128), 2, 7, "acr"),
    (capi.WS_ACR, (128, 64, 32), 3, 0, "acr"), (capi.WS_ACR, (48, 16, 80), 1, 7, "acr"),
    (capi.WS_OVERWRITE, (64, 32, 128), 2, 7, "acr"),
    (capi.WS_OVERWRITE, (64, 128, 32), 2, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (96, 64, 32), 1, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (32, 96, 32), 3, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (64, 32, 32), 2, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (128, 128, 64), 2, 0, "ip0vmm"),
    (capi.WS_IPMM_ACC, (64, 64, 64), 3, 0, "ipmm_acc"),
    (capi.WS_IPMM_ACC, (64, 128, 64), 2, 0, "ipmm_acc"),
    (capi.WS_IPMM_ACC, (64, 32, 64), 2, 0, "ipmm_acc"),
]


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("schedule,shape,levels,beta,name", FAMILY)
def test_overwrite_family_plan_reproduces_oracle(schedule, shape, levels, beta, name, fuse):
    """Tables 4 and 8 and Algorithm 1: the plan's product, the final state of
    the inputs it overwrites, its temporaries and its additions equal the
    oracle's replay."""
    m, k, n = shape
    p = 8388593 if levels % 2 else 65521
    alpha = 3
    (A, B, C), (A2, B2, C2), info = _interp(schedule, m, k, n, p, alpha, beta, levels,
                                             seed=m + k * 3 + n * 7 + levels, fuse=fuse)
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p))
    r = replay(name, A, B, C, alpha, beta, p, levels)
    assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    rs = replay_shape(name, m, k, n, p, levels, beta_nonzero=bool(beta))
    assert info.workspace_bytes == 8 * rs.peak
    assert info.element_additions == rs.adds
    assert capi.wsmul_schedule_name(info.schedule).startswith(
        {"ovl": "table4", "acr": "table8", "ip0vmm": "algorithm1",
         "ipmm_acc": "algorithm2-read-only-in-place-table9"}[name])


def test_overwrite_family_argument_errors():
    import ctypes
    s = capi.ws_stats()

    def status(m, k, n, schedule, levels, beta):
        a = capi.make_args(m, k, n, 65521, A=16, B=16, C=16, beta=beta, schedule=schedule,
                           levels=levels)
        return capi.lib().wsmul_plan_info(ctypes.byref(a), ctypes.byref(s))

    assert status(32, 32, 32, capi.WS_OVL, 1, 3) == capi.WS_ESCHEDULE      # Table 4: no beta
    assert status(32, 64, 32, capi.WS_OVL, 1, 0) == capi.WS_ESHAPE         # Table 4: square
    assert status(48, 32, 40, capi.WS_ACR, 4, 1) == capi.WS_ESHAPE         # 48 % 16 != 0
    assert status(48, 64, 32, capi.WS_OVERWRITE, 1, 0) == capi.WS_ESHAPE   # 32 does not divide 48
    assert status(32, 64, 64, capi.WS_OVERWRITE, 1, 0) == capi.WS_ESHAPE   # n is not the smallest
    assert status(64, 128, 32, capi.WS_OVERWRITE, 6, 0) == capi.WS_ESHAPE  # 32 % 64 != 0
    assert status(64, 128, 32, capi.WS_OVERWRITE, 5, 0) == capi.WS_OK
    assert status(64, 128, 32, capi.WS_OVERWRITE, 2, 1) == capi.WS_OK      # Table 8
    assert status(64, 16, 64, capi.WS_IPMM_ACC, 2, 0) == capi.WS_ESHAPE    # k < n/2
    assert status(64, 64, 64, capi.WS_IPMM_ACC, 2, 3) == capi.WS_ESCHEDULE


ALL_SELECTORS = [capi.WS_CLASSICAL, capi.WS_TWO_TEMP, capi.WS_OVERWRITE, capi.WS_READONLY_INPLACE,
                 capi.WS_HL_THREE_TEMP, capi.WS_OVR, capi.WS_ACCR, capi.WS_BLOCKED,
                 capi.WS_BLOCKED_ACC, capi.WS_OVL, capi.WS_ACR, capi.WS_IPMM_ACC]
BETA_FREE = (capi.WS_READONLY_INPLACE, capi.WS_OVR, capi.WS_OVL, capi.WS_IPMM_ACC)


@pytest.mark.parametrize("schedule", ALL_SELECTORS)
@pytest.mark.parametrize("shape", [(0, 5, 7), (6, 0, 7), (6, 5, 0), (0, 0, 0)])
def test_empty_products_under_every_schedule(schedule, shape):
    """m = 0 or n = 0 leaves C alone and k = 0 gives C <- beta*C, whatever the
    schedule (the shape restrictions of the tables do not apply)."""
    m, k, n = shape
    p = 65521
    beta = 0 if schedule in BETA_FREE else 7
    (A, B, C), (A2, B2, C2), info = _interp(schedule, m, k, n, p, 3, beta, 2, seed=5)
    assert info.workspace_bytes == 0
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 3, beta, p))


def test_blocked_workload_bytes():
    """The accumulating 4096^3 product with three levels: t = 2 needs a
    quarter (Table 2) or a sixth (Table 9) of n^2 entries at most."""
    info = lambda s, t: capi.wsmul_plan_info(capi.make_args(
        4096, 4096, 4096, 65521, beta=1, schedule=s, levels=3, blocks=t)).workspace_bytes
    assert info(capi.WS_BLOCKED, 2) == 33_030_144 < 4096 * 4096 * 8 // 4
    assert info(capi.WS_BLOCKED_ACC, 2) == 22_020_096 < 4096 * 4096 * 8 // 6
    assert info(capi.WS_BLOCKED, 3) == 14_737_464
    assert info(capi.WS_BLOCKED_ACC, 4) == 2 * (512**2 + 256**2 + 128**2) * 8
    wb = capi.wsmul_workspace_bytes
    assert wb(4096, 4096, 4096, capi.WS_F64, capi.WS_BLOCKED, 3, 1) == 33_030_144


def test_blocked_argument_errors():
    a = capi.make_args(12, 12, 12, 65521, A=16, B=16, C=16, beta=1, schedule=capi.WS_BLOCKED,
                       levels=1, blocks=65)
    import ctypes
    s = capi.ws_stats()
    assert capi.lib().wsmul_plan_info(ctypes.byref(a), ctypes.byref(s)) == capi.WS_EINVAL
    a.schedule, a.blocks = capi.WS_BLOCKED_ACC, 5                  # 12 not divisible by 5
    assert capi.lib().wsmul_plan_info(ctypes.byref(a), ctypes.byref(s)) == capi.WS_ESHAPE
    a.k, a.blocks = 8, 2                                           # not square
    assert capi.lib().wsmul_plan_info(ctypes.byref(a), ctypes.byref(s)) == capi.WS_ESHAPE
    a.schedule = capi.WS_BLOCKED                                   # Table 2 takes any shape
    assert capi.lib().wsmul_plan_info(ctypes.byref(a), ctypes.byref(s)) == capi.WS_OK


def test_fusion_reduces_launches():
    a = capi.make_args(512, 512, 512, 65521, schedule=capi.WS_TWO_TEMP, levels=1)
    fused = capi.wsmul_plan_info(a)
    a.flags = capi.WS_FLAG_NOFUSE
    plain = capi.wsmul_plan_info(a)
    assert plain.add_launches == 15 and plain.gemm_launches == 7
    assert fused.gemm_launches == 7 and fused.add_launches < 15
    assert fused.rows == plain.rows == 22


@pytest.mark.parametrize("schedule,levels,beta,want", [
    (capi.WS_TWO_TEMP, 1, 0, 1_048_576),
])
def test_small_workload_bytes(schedule, levels, beta, want):
    assert capi.wsmul_workspace_bytes(512, 512, 512, capi.WS_I64, schedule, levels, beta) == want


def test_workload_bytes():
    wb = capi.wsmul_workspace_bytes
    assert wb(4096, 4096, 4096, capi.WS_F64, capi.WS_TWO_TEMP, 3, 1) == 88_080_384
    assert wb(4096, 4096, 4096, capi.WS_F64, capi.WS_OVERWRITE, 3, 1) == 88_080_384
    assert wb(4096, 4096, 4096, capi.WS_F64, capi.WS_HL_THREE_TEMP, 3, 1) == 132_120_576
    assert wb(4096, 4096, 4096, capi.WS_F64, capi.WS_OVERWRITE, 3, 0) == 0
    for l, want in zip((1, 2, 3, 4), (201_326_592, 251_658_240, 264_241_152, 267_386_880)):
        assert wb(8192, 4096, 8192, capi.WS_F64, capi.WS_TWO_TEMP, l, 0) == want
    for l in (1, 2, 3):
        assert wb(8192, 4096, 8192, capi.WS_F64, capi.WS_READONLY_INPLACE, l, 0) == 0
    for l, want in zip((1, 2, 3), (1_073_741_824, 1_342_177_280, 1_409_286_144)):
        assert wb(16384, 16384, 16384, capi.WS_F64, capi.WS_TWO_TEMP, l, 0) == want


def _status(**kw):
    base = dict(m=8, k=8, n=8, p=65521, A=16, B=16, C=16, schedule=capi.WS_TWO_TEMP, levels=1)
    base.update(kw)
    m, k, n, p = base.pop("m"), base.pop("k"), base.pop("n"), base.pop("p")
    a = capi.make_args(m, k, n, p, **base)
    s = capi.ws_stats()
    import ctypes
    return capi.lib().wsmul_plan_info(ctypes.byref(a), ctypes.byref(s))


def test_argument_errors():
    assert _status() == capi.WS_OK
    assert _status(m=-1) == capi.WS_EINVAL
    assert _status(p=1) == capi.WS_EMODULUS
    assert _status(p=1 << 24) == capi.WS_EMODULUS
    assert _status(lda=3) == capi.WS_EINVAL
    assert _status(schedule=99) == capi.WS_ESCHEDULE
    assert _status(schedule=capi.WS_READONLY_INPLACE, beta=3) == capi.WS_ESCHEDULE
    assert _status(schedule=capi.WS_OVERWRITE, m=12, k=12, n=12, levels=3) == capi.WS_ESHAPE
    assert _status(schedule=capi.WS_OVERWRITE, m=8, k=4, n=8, levels=1) == capi.WS_ESHAPE
    assert _status(schedule=capi.WS_TWO_TEMP, beta=1, m=8, k=4, n=8) == capi.WS_ESHAPE
    assert _status(levels=25) == capi.WS_EINVAL
    assert _status(dtype=7) == capi.WS_EINVAL
    assert _status(base=9) == capi.WS_EINVAL
    assert "levels" in capi.wsmul_last_error() or capi.wsmul_last_error()
