"""GPU parity: the HIP path through the C-ABI against the oracle, bit for bit.

Small and ragged shapes run every schedule against the oracle's full product
(and, for schedules that destroy their inputs, against the replayed final
state of A and B).  The named workloads at full size are compared entry by
entry in test_gpu_configs.py.
"""
import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay
from paper_0707_2347_amd import capi, inputs

from .gpu_util import call

pytestmark = pytest.mark.gpu

ORACLE_NAME = {
    (capi.WS_CLASSICAL, False): "classical", (capi.WS_CLASSICAL, True): "classical",
    (capi.WS_TWO_TEMP, False): "t1", (capi.WS_TWO_TEMP, True): "acc",
    (capi.WS_OVERWRITE, False): "ip", (capi.WS_OVERWRITE, True): "aclr",
    (capi.WS_READONLY_INPLACE, False): "ipmm",
    (capi.WS_HL_THREE_TEMP, False): "hl", (capi.WS_HL_THREE_TEMP, True): "hl",
    (capi.WS_OVR, False): "ovr", (capi.WS_ACCR, True): "accr",
}


@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("shape", [(1, 1, 1), (16, 4, 16), (17, 33, 9), (3, 1000, 5),
                                   (100, 257, 130), (64, 64, 64), (300, 200, 700),
                                   (511, 512, 513), (1024, 96, 1024), (0, 5, 3), (4, 0, 6)])
@pytest.mark.parametrize("p", [65521, 8388593])
def test_classical_shapes(shape, dtype, p):
    m, k, n = shape
    print("classical", shape, dtype, p, flush=True)
    A, B, C = inputs.uniform(m * 131 + k * 7 + n, m, k, n, p, with_c=True)
    for alpha, beta in [(1, 0), (3, 1), (p - 1, p - 5)]:
        st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, C, alpha, beta, p, 0, dtype=dtype)
        assert st == capi.WS_OK, capi.wsmul_last_error()
        assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p)), (alpha, beta)


def test_extreme_entries_long_k():
    """All entries p-1 with a long inner dimension: the largest partial sums,
    several folds of the accumulators."""
    p = 8388593
    m, k, n = 96, 5000, 80
    A = np.full((m, k), p - 1, dtype=np.int64)
    B = np.full((k, n), p - 1, dtype=np.int64)
    st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, None, 1, 0, p, 0)
    assert st == capi.WS_OK
    assert np.all(C2 == k % p)


# Whole 32 x 32, 64 x 64 or 128 x 128 tiles and 64-deep inner chunks with
# aligned rows: the pipelined kernels, both storage types, folds included.
@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("shape,p", [((32, 64, 32), 65521), ((96, 640, 160), 8388593),
                                     ((128, 128, 128), 1048573), ((256, 4096, 256), 8388593),
                                     ((64, 2048, 64), 16777213), ((512, 512, 512), 65521),
                                     ((32, 8192, 64), 16777213), ((1024, 1024, 1024), 65521),
                                     ((1024, 512, 1024), 8388593), ((2048, 128, 512), 1048573),
                                     ((1024, 2048, 512), 16777213), ((4096, 256, 2048), 8388593),
                                     ((2048, 1024, 4096), 16777213), ((4096, 512, 2048), 65521)])
def test_whole_tile_products(shape, p, dtype):
    m, k, n = shape
    print("whole-tile", shape, p, dtype, flush=True)
    A, B, C = inputs.uniform(m + 3 * k + 7 * n, m, k, n, p, with_c=True)
    for alpha, beta in [(1, 0), (3, 1), (p - 1, p - 5)]:
        st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, C, alpha, beta, p, 0, dtype=dtype)
        assert st == capi.WS_OK, capi.wsmul_last_error()
        assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p)), (alpha, beta)


@pytest.mark.parametrize("shape", [(256, 4096, 256), (1024, 2048, 1024), (4096, 1024, 2048)])
def test_whole_tile_largest_uncentred_sums(shape):
    """All entries p-1 for p = 8388593, where the pipelined kernels keep the
    operands uncentred and fold the accumulators instead: each fold period
    brings a partial sum within a few p of 2^53."""
    p = 8388593
    m, k, n = shape
    A = np.full((m, k), p - 1, dtype=np.int64)
    B = np.full((k, n), p - 1, dtype=np.int64)
    st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, None, 1, 0, p, 0)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.all(C2 == k % p)


@pytest.mark.parametrize("shape", [(64, 8192, 96), (1024, 2048, 1024), (2048, 1024, 4096)])
def test_whole_tile_largest_centred_sums(shape):
    """Centred operands of the largest magnitude, (p-1)/2 against -(p-1)/2,
    over long inner dimensions: every partial sum needs the periodic folds
    (32 x 32 and 64 x 64 tiles)."""
    p = 16777213
    m, k, n = shape
    A = np.full((m, k), (p - 1) // 2, dtype=np.int64)
    B = np.full((k, n), (p + 1) // 2, dtype=np.int64)
    st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, None, 1, 0, p, 0)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, None, 1, 0, p))


CASES = [
    (capi.WS_TWO_TEMP, (64, 64, 64), 1, False), (capi.WS_TWO_TEMP, (128, 128, 128), 3, False),
    (capi.WS_TWO_TEMP, (128, 64, 256), 2, False), (capi.WS_TWO_TEMP, (192, 128, 64), 2, False),
    (capi.WS_TWO_TEMP, (137, 150, 129), 2, False), (capi.WS_TWO_TEMP, (255, 255, 255), 3, False),
    (capi.WS_TWO_TEMP, (128, 128, 128), 1, True), (capi.WS_TWO_TEMP, (256, 256, 256), 3, True),
    (capi.WS_TWO_TEMP, (161, 161, 161), 2, True),
    (capi.WS_OVERWRITE, (128, 128, 128), 1, False), (capi.WS_OVERWRITE, (256, 256, 256), 3, False),
    (capi.WS_OVERWRITE, (64, 64, 64), 2, True), (capi.WS_OVERWRITE, (256, 256, 256), 3, True),
    (capi.WS_READONLY_INPLACE, (128, 128, 128), 1, False),
    (capi.WS_READONLY_INPLACE, (256, 256, 256), 3, False),
    (capi.WS_READONLY_INPLACE, (256, 128, 256), 2, False),
    (capi.WS_READONLY_INPLACE, (128, 256, 128), 2, False),
    (capi.WS_HL_THREE_TEMP, (128, 128, 128), 2, True), (capi.WS_HL_THREE_TEMP, (96, 64, 32), 2, True),
    (capi.WS_OVR, (128, 128, 128), 3, False), (capi.WS_ACCR, (128, 128, 128), 3, True),
]


@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("schedule,shape,levels,acc", CASES)
def test_schedules(schedule, shape, levels, acc, dtype):
    m, k, n = shape
    print("schedule", schedule, shape, levels, acc, dtype, flush=True)
    p = 8388593 if levels % 2 else 65521
    A, B, C = inputs.uniform(m * 11 + k * 5 + n * 3 + levels, m, k, n, p, with_c=True)
    alpha, beta = 7, (11 if acc else 0)
    st, C2, A2, B2 = call(schedule, A, B, C, alpha, beta, p, levels, dtype=dtype)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, alpha, beta, p))
    name = ORACLE_NAME[(schedule, acc)]
    r = replay(name, A, B, C, alpha, beta, p, levels)
    assert np.array_equal(C2, r.C)
    assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)


def test_unfused_equals_fused():
    p = 65521
    A, B, C = inputs.uniform(77, 256, 256, 256, p, with_c=True)
    outs = []
    for flags in (0, capi.WS_FLAG_NOFUSE):
        st, C2, A2, B2 = call(capi.WS_TWO_TEMP, A, B, C, 3, 4, p, 3, flags=flags)
        assert st == capi.WS_OK
        outs.append((C2, A2, B2))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_t1_512_int64_full():
    """C = A*B mod 65521, 512^3, one level of Table 1, int64 storage."""
    w = inputs.WORKLOADS["t1_512_p65521_l1_i64"]
    A, B, _ = inputs.uniform(w["seed"], w["m"], w["k"], w["n"], w["p"])
    st, C2, A2, B2 = call(capi.WS_TWO_TEMP, A, B, None, 1, 0, w["p"], 1, dtype=capi.WS_I64)
    assert st == capi.WS_OK
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, None, 1, 0, w["p"]))
    assert np.array_equal(A2, A) and np.array_equal(B2, B)
    s = capi.wsmul_get_stats()
    assert s.workspace_bytes == 1_048_576


BLOCKED = [
    # schedule, shape, levels, t, beta
    (capi.WS_BLOCKED, (256, 256, 256), 2, 2, 11), (capi.WS_BLOCKED, (384, 384, 384), 2, 3, 11),
    (capi.WS_BLOCKED, (300, 200, 100), 1, 3, 11), (capi.WS_BLOCKED, (256, 128, 512), 1, 4, 0),
    (capi.WS_BLOCKED_ACC, (256, 256, 256), 3, 2, 11), (capi.WS_BLOCKED_ACC, (384, 384, 384), 2, 3, 11),
    (capi.WS_BLOCKED_ACC, (270, 270, 270), 1, 3, 11), (capi.WS_BLOCKED_ACC, (128, 128, 128), 1, 1, 0),
]


@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("schedule,shape,levels,t,beta", BLOCKED)
def test_blocked_schedules(schedule, shape, levels, t, beta, dtype):
    """Section 7.2's blocked accumulation (ragged parts and blocks included)."""
    m, k, n = shape
    print("blocked", schedule, shape, levels, t, beta, dtype, flush=True)
    p = 8388593 if levels % 2 else 65521
    A, B, C = inputs.uniform(m * 13 + k * 7 + n + t, m, k, n, p, with_c=True)
    st, C2, A2, B2 = call(schedule, A, B, C, 5, beta, p, levels, dtype=dtype, blocks=t)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 5, beta, p))
    name = "blocked" if schedule == capi.WS_BLOCKED else "blocked_acc"
    r = replay(name, A, B, C, 5, beta, p, levels, blocks=t)
    assert np.array_equal(C2, r.C)
    assert np.array_equal(A2, A) and np.array_equal(B2, B)


FAMILY = [
    # selector, shape, levels, beta, oracle schedule
    (capi.WS_OVL, (128, 128, 128), 1, 0, "ovl"), (capi.WS_OVL, (256, 256, 256), 3, 0, "ovl"),
    (capi.WS_ACR, (256, 128, 512), 2, 11, "acr"), (capi.WS_ACR, (512, 256, 128), 3, 11, "acr"),
    (capi.WS_ACR, (192, 64, 320), 1, 0, "acr"), (capi.WS_ACR, (256, 256, 256), 2, 11, "acr"),
    (capi.WS_OVERWRITE, (256, 512, 128), 2, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (384, 256, 128), 1, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (128, 384, 128), 3, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (256, 128, 128), 2, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (512, 512, 256), 2, 0, "ip0vmm"),
    (capi.WS_OVERWRITE, (256, 128, 512), 2, 11, "acr"),
    (capi.WS_IPMM_ACC, (256, 256, 256), 3, 0, "ipmm_acc"),
    (capi.WS_IPMM_ACC, (256, 512, 256), 2, 0, "ipmm_acc"),
    (capi.WS_IPMM_ACC, (256, 128, 256), 1, 0, "ipmm_acc"),
]


@pytest.mark.parametrize("dtype", [capi.WS_F64, capi.WS_I64])
@pytest.mark.parametrize("schedule,shape,levels,beta,name", FAMILY)
def test_overwrite_family(schedule, shape, levels, beta, name, dtype):
    """Tables 4 and 8, Algorithm 1 and Algorithm 2 with Table 9: the product, and the final state of the
    inputs they overwrite, against the oracle's replay."""
    m, k, n = shape
    print("family", schedule, shape, levels, beta, dtype, flush=True)
    p = 8388593 if levels % 2 else 65521
    A, B, C = inputs.uniform(m * 3 + k * 5 + n * 11 + levels, m, k, n, p, with_c=True)
    st, C2, A2, B2 = call(schedule, A, B, C, 9, beta, p, levels, dtype=dtype)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 9, beta, p))
    r = replay(name, A, B, C, 9, beta, p, levels)
    assert np.array_equal(C2, r.C)
    assert np.array_equal(A2, r.A) and np.array_equal(B2, r.B)
    assert capi.wsmul_get_stats().workspace_bytes == 8 * int(r.peak)


@pytest.mark.parametrize("schedule", [capi.WS_TWO_TEMP, capi.WS_OVERWRITE, capi.WS_READONLY_INPLACE,
                                      capi.WS_OVR, capi.WS_ACCR, capi.WS_BLOCKED, capi.WS_BLOCKED_ACC,
                                      capi.WS_OVL, capi.WS_ACR, capi.WS_IPMM_ACC])
@pytest.mark.parametrize("shape", [(0, 5, 7), (6, 0, 7), (6, 5, 0)])
def test_empty_products(schedule, shape):
    m, k, n = shape
    p = 65521
    beta = 0 if schedule in (capi.WS_READONLY_INPLACE, capi.WS_OVR, capi.WS_OVL,
                             capi.WS_IPMM_ACC) else 7
    A, B, C = inputs.uniform(43, m, k, n, p, with_c=True)
    st, C2, _, _ = call(schedule, A, B, C, 3, beta, p, 2)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 3, beta, p))


@pytest.mark.parametrize("schedule,shape,levels,beta,blocks", [
    (capi.WS_BLOCKED, (512, 2048, 512), 1, 1, 2), (capi.WS_BLOCKED_ACC, (1024, 1024, 1024), 2, 1, 2),
    (capi.WS_OVERWRITE, (512, 4096, 256), 1, 0, 0), (capi.WS_OVERWRITE, (256, 2048, 512), 1, 1, 0),
    (capi.WS_IPMM_ACC, (512, 1024, 512), 1, 0, 0), (capi.WS_OVL, (1024, 1024, 1024), 2, 0, 0),
    (capi.WS_TWO_TEMP, (1024, 1024, 1024), 3, 1, 0), (capi.WS_HL_THREE_TEMP, (512, 4096, 512), 2, 1, 0)])
@pytest.mark.parametrize("p", [8388593, 16777213])
def test_extreme_entries_under_schedules(schedule, shape, levels, beta, blocks, p):
    """Every entry of A, B, C is p - 1 (the largest residue): since
    (p-1)^2 = 1 mod p the product is k everywhere, so C = alpha*k + beta*(p-1)
    mod p in closed form, whatever the schedule makes of the operands."""
    m, k, n = shape
    A = np.full((m, k), p - 1, dtype=np.int64)
    B = np.full((k, n), p - 1, dtype=np.int64)
    C = np.full((m, n), p - 1, dtype=np.int64)
    alpha = p - 3
    st, C2, _, _ = call(schedule, A, B, C, alpha, beta, p, levels, blocks=blocks)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    want = (alpha * k + beta * (p - 1)) % p
    assert np.all(C2 == want)


def test_attached_workspace_exact_size_and_no_hidden_allocation():
    t = __import__("torch")
    p = 65521
    n = 512
    A, B, C = inputs.uniform(5, n, n, n, p, with_c=True)
    need = capi.wsmul_workspace_bytes(n, n, n, capi.WS_F64, capi.WS_TWO_TEMP, 2, 1)
    assert need == 8 * 2 * (256 * 256 + 128 * 128)
    ws = t.empty(need // 8, dtype=t.float64, device="cuda:0")
    st, C2, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 2, 3, p, 2, workspace=ws, workspace_bytes=need)
    assert st == capi.WS_OK
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 2, 3, p))
    assert capi.wsmul_get_stats().internal_alloc_bytes == 0
    free0 = t.cuda.mem_get_info()[0]
    st, C3, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 2, 3, p, 2, workspace=ws, workspace_bytes=need)
    assert t.cuda.mem_get_info()[0] == free0
    assert np.array_equal(C3, C2)
    st, _, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 2, 3, p, 2, workspace=ws,
                       workspace_bytes=need - 8)
    assert st == capi.WS_ENOMEM


def test_range_check_flag():
    p = 65521
    A, B, C = inputs.uniform(6, 32, 32, 32, p, with_c=True)
    A[3, 4] = p
    st, C2, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 1, 1, p, 1, flags=capi.WS_FLAG_CHECK)
    assert st == capi.WS_ERANGE
    assert np.array_equal(C2, C)           # nothing written
    A[3, 4] = 0
    st, C2, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 1, 1, p, 1, flags=capi.WS_FLAG_CHECK)
    assert st == capi.WS_OK
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 1, 1, p))


def test_trace_counts_launches():
    p = 65521
    capi.wsmul_reset_stats()
    A, B, C = inputs.uniform(8, 256, 256, 256, p, with_c=True)
    st, _, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 1, 1, p, 2, flags=capi.WS_FLAG_TRACE)
    assert st == capi.WS_OK
    tr = capi.wsmul_get_trace()
    s = capi.wsmul_get_stats()
    assert tr.gemm_launches == s.gemm_launches == 49
    assert tr.add_launches == s.add_launches
    assert tr.gemm_ms > 0 and tr.add_ms > 0
