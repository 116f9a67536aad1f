"""GPU parity of the batched persistent launch and its hipGraph replay.

Each product of a batch is checked in full against the oracle (the
2000-product workload in test_gpu_configs.py)."""
import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _mk_batch(specs, seed):
    """specs: (m, k, n, p, schedule, levels, beta).  Returns host and device data."""
    t = _torch()
    host, dev, args = [], [], []
    rng = np.random.default_rng(seed)
    for i, spec in enumerate(specs):
        m, k, n, p, sched, lev, beta = spec[:7]
        A, B, C = inputs.uniform(seed * 1000 + i, m, k, n, p, with_c=True)
        dA = t.from_numpy(A.astype(np.float64)).cuda()
        dB = t.from_numpy(B.astype(np.float64)).cuda()
        dC = t.from_numpy(C.astype(np.float64)).cuda()
        alpha = int(rng.integers(1, p))
        host.append((A, B, C, alpha, beta, p))
        dev.append((dA, dB, dC))
        args.append(capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, sched, lev,
                                   base=capi.WS_BASE_F64_MFMA,
                                   stream=t.cuda.current_stream(),
                                   blocks=spec[7] if len(spec) > 7 else 0))
    return host, dev, args


SPECS = [
    (64, 64, 64, 65521, capi.WS_CLASSICAL, 0, 0), (100, 37, 213, 8388593, capi.WS_CLASSICAL, 0, 5),
    (128, 128, 128, 1048573, capi.WS_TWO_TEMP, 1, 0), (256, 256, 256, 65521, capi.WS_TWO_TEMP, 2, 3),
    (200, 300, 150, 8388593, capi.WS_TWO_TEMP, 2, 0), (256, 256, 256, 65521, capi.WS_OVERWRITE, 2, 0),
    (256, 128, 256, 8388593, capi.WS_READONLY_INPLACE, 2, 0), (96, 96, 96, 65521, capi.WS_HL_THREE_TEMP, 1, 7),
    (333, 444, 555, 1048573, capi.WS_AUTO, -1, 0), (1024, 512, 768, 8388593, capi.WS_AUTO, -1, 9),
    (1, 1, 1, 65521, capi.WS_CLASSICAL, 0, 1), (65, 2047, 17, 8388593, capi.WS_CLASSICAL, 0, 0),
]


def test_batched_mixed():
    t = _torch()
    host, dev, args = _mk_batch(SPECS, 3)
    st = capi.wsmul_batched(args, capi.WS_FLAG_SYNC)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    t.cuda.synchronize()
    for (A, B, C, alpha, beta, p), (dA, dB, dC) in zip(host, dev):
        got = dC.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, ref.matmul_mod_p(A, B, C, alpha, beta, p))


SPECS_MORE = [
    # the blocked accumulation of Section 7.2 (last field: t), Tables 4 and 8,
    # Algorithm 1 and Algorithm 2 with Table 9, side by side in one batch
    (256, 256, 256, 65521, capi.WS_BLOCKED, 2, 3, 2), (384, 384, 384, 8388593, capi.WS_BLOCKED, 1, 5, 3),
    (256, 256, 256, 65521, capi.WS_BLOCKED_ACC, 2, 3, 2), (256, 128, 512, 65521, capi.WS_ACR, 2, 11),
    (256, 512, 128, 8388593, capi.WS_OVERWRITE, 2, 0), (128, 384, 128, 65521, capi.WS_OVERWRITE, 2, 0),
    (256, 256, 256, 65521, capi.WS_OVL, 2, 0), (256, 512, 256, 8388593, capi.WS_IPMM_ACC, 2, 0),
]


def test_batched_more_schedules():
    t = _torch()
    host, dev, args = _mk_batch(SPECS_MORE, 4)
    st = capi.wsmul_batched(args, capi.WS_FLAG_SYNC)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    t.cuda.synchronize()
    for (A, B, C, alpha, beta, p), (dA, dB, dC) in zip(host, dev):
        got = dC.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, ref.matmul_mod_p(A, B, C, alpha, beta, p))


def test_graph_replays_with_eager_work_between():
    t = _torch()
    specs = [s for s in SPECS if s[4] != capi.WS_OVERWRITE]
    host, dev, args = _mk_batch(specs, 4)
    st, handle = capi.wsmul_graph_capture(args)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    try:
        for rep in range(3):
            # eager work between replays: fresh inputs and C, plus unrelated kernels
            newhost = []
            for i, ((A, B, C, alpha, beta, p), (dA, dB, dC)) in enumerate(zip(host, dev)):
                A2, B2, C2 = inputs.uniform(500 + 10 * rep + i, A.shape[0], A.shape[1], B.shape[1],
                                            p, with_c=True)
                dA.copy_(t.from_numpy(A2.astype(np.float64)))
                dB.copy_(t.from_numpy(B2.astype(np.float64)))
                dC.copy_(t.from_numpy(C2.astype(np.float64)))
                newhost.append((A2, B2, C2, alpha, beta, p))
            scratch = t.ones(1 << 20, device="cuda:0").sum()
            t.cuda.synchronize()
            assert capi.wsmul_graph_launch(handle, t.cuda.current_stream()) == capi.WS_OK
            assert capi.wsmul_graph_check(handle, t.cuda.current_stream()) == capi.WS_OK
            t.cuda.synchronize()
            assert float(scratch) == float(1 << 20)
            for (A, B, C, alpha, beta, p), (dA, dB, dC) in zip(newhost, dev):
                got = dC.cpu().numpy().astype(np.int64)
                assert np.array_equal(got, ref.matmul_mod_p(A, B, C, alpha, beta, p)), rep
    finally:
        capi.wsmul_graph_destroy(handle)


@pytest.mark.parametrize("shape,p,beta", [((300, 200, 100), 65521, 0), ((1024, 1024, 1024), 1048573, 0),
                                          ((512, 512, 512), 8388593, 3)])
def test_autotuned_calls(shape, p, beta):
    from .gpu_util import call
    m, k, n = shape
    A, B, C = inputs.uniform(21, m, k, n, p, with_c=True)
    st, C2, _, _ = call(capi.WS_AUTO, A, B, C, 5, beta, p, -1, base=capi.WS_BASE_AUTO)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 5, beta, p))


def test_batch_with_base_left_to_the_library():
    """Products whose base is left at WS_BASE_AUTO (the zero default) run on
    the binary64 base inside a batch, even at sizes where the autotuner would
    pick the 8-bit digit base for a single call."""
    t = _torch()
    specs = [(2048, 2048, 2048, 65521, capi.WS_AUTO, -1, 0), (1024, 1024, 1024, 1048573, capi.WS_AUTO, -1, 4),
             (300, 500, 200, 8388593, capi.WS_TWO_TEMP, 1, 0)]
    host, dev, args = _mk_batch(specs, 6)
    for a in args:
        a.base = capi.WS_BASE_AUTO
    st = capi.wsmul_batched(args, capi.WS_FLAG_SYNC)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    t.cuda.synchronize()
    for (A, B, C, alpha, beta, p), (dA, dB, dC) in zip(host, dev):
        got = dC.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, ref.matmul_mod_p(A, B, C, alpha, beta, p))

