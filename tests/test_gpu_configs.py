"""GPU parity at the full sizes of the named workloads, element by element.

Every entry of every product is compared with the oracle's full product
(oracle O1), in the launch configuration the benchmark times (caller
workspace of the reported size on torch's current stream; the 2000-product
batch as one graph replay).  A mismatch reports the first differing
(row, column).  The largest product (16384^3) is checked in bands of rows so
that each test does a bounded share of the oracle's work.

Workloads: 4096^3 C <- A*B + C mod 65521 under Table 9 and Table 6 at three
levels, classical, and Section 7.2's blocks; 8192 x 4096 x 8192 mod 8388593
under Algorithm 2 and Table 1; Algorithm 1 on 4096 x 8192 x 4096,
8192 x 8192 x 4096 and 8192 x 16384 x 8192; 16384^3 mod 1048573 on the 8-bit
digit base (classical and Table 1 at one level), on the binary64 base (Table 1
at two levels) and as the autotuner chooses; the 2000-product batch.
"""
import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

pytestmark = pytest.mark.gpu

_cache = {}


def _torch():
    import torch
    return torch


def assert_same(got, want, what):
    """Full comparison; on a mismatch name the first differing entry."""
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, c = (int(x) for x in bad[0])
        raise AssertionError("%s: %d entries differ; first at (row %d, col %d): got %d, want %d"
                             % (what, len(bad), r, c, int(got[r, c]), int(want[r, c])))


def _cached(key, make):
    """One workload's inputs and oracle product at a time (host memory)."""
    if key not in _cache:
        _cache.clear()
        _cache[key] = make()
    return _cache[key]


def run_product(A, B, C, alpha, beta, p, schedule, levels, *, base=capi.WS_BASE_F64_MFMA,
                blocks=0, keep_inputs=True, expect_ws=None):
    """One product on cuda:0 with a caller workspace of exactly the reported
    size; returns C as int64.  Read-only schedules are checked to leave A and
    B bitwise unchanged (on the device)."""
    t = _torch()
    m, k = A.shape
    n = B.shape[1]
    dA = t.from_numpy(A.astype(np.float64)).to("cuda:0")
    dB = t.from_numpy(B.astype(np.float64)).to("cuda:0")
    dC = (t.from_numpy(C.astype(np.float64)).to("cuda:0") if C is not None
          else t.full((m, n), -1.0, dtype=t.float64, device="cuda:0"))
    stream = t.cuda.current_stream()
    args = capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, schedule, levels, base=base,
                          stream=stream, blocks=blocks)
    need = capi.wsmul_plan_info(args).workspace_bytes
    if expect_ws is not None:
        assert need == expect_ws, (need, expect_ws)
    ws = t.empty(max(need // 8, 1), dtype=t.float64, device="cuda:0")
    args = capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, schedule, levels, base=base,
                          stream=stream, blocks=blocks, workspace=ws, workspace_bytes=need)
    if keep_inputs:
        A0, B0 = dA.clone(), dB.clone()
    st = capi.wsmul_mod_p_ex(args)
    t.cuda.synchronize()
    assert st == capi.WS_OK, capi.wsmul_last_error()
    if keep_inputs:
        assert t.equal(dA, A0) and t.equal(dB, B0), "a read-only schedule changed its inputs"
        del A0, B0
    out = dC.cpu().numpy().astype(np.int64)
    del dA, dB, dC, ws
    return out


# ------------------------------------------------ 4096^3, C <- A*B + C mod 65521
def _c2():
    def make():
        w = inputs.WORKLOADS["acc_4096_p65521_l3"]
        A, B, C = inputs.uniform(w["seed"], w["m"], w["k"], w["n"], w["p"], with_c=True)
        return A, B, C, w["p"], ref.matmul_mod_p(A, B, C, 1, 1, w["p"])
    return _cached(("c2",), make)


@pytest.mark.parametrize("schedule,levels,ws", [
    (capi.WS_TWO_TEMP, 3, 88_080_384), (capi.WS_OVERWRITE, 3, 88_080_384),
    (capi.WS_CLASSICAL, 0, 0), (capi.WS_TWO_TEMP, 1, 67_108_864)])
def test_acc_4096_full(schedule, levels, ws):
    A, B, C, p, want = _c2()
    print("4096^3 accumulate, schedule", schedule, "levels", levels, flush=True)
    got = run_product(A, B, C, 1, 1, p, schedule, levels, expect_ws=ws,
                      keep_inputs=schedule != capi.WS_OVERWRITE)
    assert_same(got, want, "4096^3 schedule %d, %d levels" % (schedule, levels))


@pytest.mark.parametrize("schedule,levels,t,ws", [
    (capi.WS_BLOCKED, 3, 2, 33_030_144), (capi.WS_BLOCKED_ACC, 3, 2, 22_020_096),
    (capi.WS_BLOCKED_ACC, 2, 2, 20_971_520), (capi.WS_BLOCKED, 2, 3, 3 * (684**2 + 342**2) * 8)])
def test_acc_4096_blocked_full(schedule, levels, t, ws):
    """Section 7.2's blocks on the same product (ragged parts for t = 3)."""
    A, B, C, p, want = _c2()
    print("4096^3 blocked", schedule, levels, t, flush=True)
    got = run_product(A, B, C, 1, 1, p, schedule, levels, blocks=t, expect_ws=ws)
    assert_same(got, want, "4096^3 blocked schedule %d, t = %d" % (schedule, t))
    assert capi.wsmul_get_stats().internal_alloc_bytes == 0


# ------------------------------------------ 8192 x 4096 x 8192, C = A*B mod 8388593
def _c3():
    def make():
        w = inputs.WORKLOADS["ipmm_8192x4096x8192_p8388593"]
        A, B, _ = inputs.uniform(w["seed"], w["m"], w["k"], w["n"], w["p"])
        return A, B, w["p"], ref.matmul_mod_p(A, B, None, 1, 0, w["p"])
    return _cached(("c3",), make)


@pytest.mark.parametrize("schedule,levels,ws", [
    (capi.WS_READONLY_INPLACE, 1, 0), (capi.WS_READONLY_INPLACE, 2, 0),
    (capi.WS_TWO_TEMP, 1, 201_326_592), (capi.WS_TWO_TEMP, 2, 251_658_240),
    (capi.WS_CLASSICAL, 0, 0)])
def test_8192x4096x8192_full(schedule, levels, ws):
    A, B, p, want = _c3()
    print("8192x4096x8192 schedule", schedule, "levels", levels, flush=True)
    got = run_product(A, B, None, 1, 0, p, schedule, levels, expect_ws=ws)
    assert_same(got, want, "8192x4096x8192 schedule %d, %d levels" % (schedule, levels))


# ----------------------------------------------- Algorithm 1 at the paper's shapes
def _alg1(shape):
    def make():
        m, k, n = shape
        A, B, _ = inputs.uniform(41 if shape != (8192, 16384, 8192) else 6, m, k, n, 8388593)
        return A, B, ref.matmul_mod_p(A, B, None, 1, 0, 8388593)
    return _cached(("alg1", shape), make)


@pytest.mark.parametrize("shape,levels", [((4096, 8192, 4096), 2), ((8192, 8192, 4096), 2),
                                          ((8192, 16384, 8192), 1), ((8192, 16384, 8192), 2)])
def test_algorithm1_full(shape, levels):
    """Algorithm 1 (no workspace; A, and B when m = n, overwritten) on shapes
    the paper times, the largest in the configuration the benchmark runs."""
    A, B, want = _alg1(shape)
    print("Algorithm 1", shape, "levels", levels, flush=True)
    got = run_product(A, B, None, 1, 0, 8388593, capi.WS_OVERWRITE, levels, expect_ws=0,
                      keep_inputs=False)
    assert_same(got, want, "Algorithm 1 %s, %d levels" % (shape, levels))
    s = capi.wsmul_get_stats()
    assert s.workspace_bytes == 0 and s.internal_alloc_bytes == 0


# ------------------------------------------------- 16384^3, C = A*B mod 1048573
C4_RUNS = [
    # label, schedule, levels, base
    ("classical, int8 digits", capi.WS_CLASSICAL, 0, capi.WS_BASE_I8_LIMBS),
    ("Table 1, 1 level, int8 digits", capi.WS_TWO_TEMP, 1, capi.WS_BASE_I8_LIMBS),
    ("Table 1, 2 levels, binary64", capi.WS_TWO_TEMP, 2, capi.WS_BASE_F64_MFMA),
    ("autotuned", capi.WS_AUTO, -1, capi.WS_BASE_AUTO),
]
C4_BANDS = 8


def _c4():
    def make():
        w = inputs.WORKLOADS["t1_16384_p1048573"]
        A, B, _ = inputs.uniform(w["seed"], w["m"], w["k"], w["n"], w["p"])
        outs = []
        for label, sched, lev, base in C4_RUNS:
            print("16384^3:", label, flush=True)
            outs.append(run_product(A, B, None, 1, 0, w["p"], sched, lev, base=base))
        return A, B, w["p"], outs
    return _cached(("c4",), make)


@pytest.mark.parametrize("band", range(C4_BANDS))
def test_16384_full(band):
    """Every entry of the 16384^3 product under four plans, one band of rows
    of the oracle's product per test."""
    A, B, p, outs = _c4()
    rows = A.shape[0] // C4_BANDS
    r0, r1 = band * rows, (band + 1) * rows
    want = ref.matmul_mod_p(A[r0:r1], B, None, 1, 0, p)
    for (label, _, _, _), got in zip(C4_RUNS, outs):
        assert_same(got[r0:r1], want, "16384^3 %s, rows %d..%d" % (label, r0, r1 - 1))


# ------------------------------------------------------ the 2000-product batch
def test_batch_workload_2000_full():
    """All 2000 products of the batch workload (sizes log-uniform in
    [64, 2048], three moduli, autotuned) in one graph replay, every entry of
    every product against the oracle."""
    t = _torch()
    _cache.clear()
    probs = inputs.batch_problems()
    assert len(probs) == 2000
    args, dev = [], []
    for pr in probs:
        A, B = inputs.batch_inputs(pr)
        m, k, n, p = pr["m"], pr["k"], pr["n"], pr["p"]
        dA = t.from_numpy(A).cuda()
        dB = t.from_numpy(B).cuda()
        dC = t.full((m, n), -1.0, dtype=t.float64, device="cuda:0")
        dev.append((dA, dB, dC))
        args.append(capi.make_args(m, k, n, p, dA, dB, dC, 1, 0, capi.WS_AUTO, -1,
                                   base=capi.WS_BASE_F64_MFMA, stream=t.cuda.current_stream()))
    st, handle = capi.wsmul_graph_capture(args)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    try:
        assert capi.wsmul_graph_launch(handle, t.cuda.current_stream()) == capi.WS_OK
        assert capi.wsmul_graph_check(handle, t.cuda.current_stream()) == capi.WS_OK
        t.cuda.synchronize()
    finally:
        capi.wsmul_graph_destroy(handle)
    for pr, (dA, dB, dC) in zip(probs, dev):
        A, B = inputs.batch_inputs(pr)
        want = ref.matmul_mod_p(A, B, None, 1, 0, pr["p"])
        got = dC.cpu().numpy().astype(np.int64)
        assert_same(got, want, "batch product %d (%d x %d x %d mod %d)"
                    % (pr["index"], pr["m"], pr["k"], pr["n"], pr["p"]))
