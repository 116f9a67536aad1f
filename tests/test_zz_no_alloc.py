"""The no-allocation entry point (wsmul_mod_p_noalloc) against wsmul_mod_p_ex.

Two calls in a row on one GPU, the second on a smaller product, each compared
bit for bit with the allocating entry point on the same inputs (and with the
oracle); no device memory is allocated during the calls; products too large
for the static scratch and attached workspaces are refused before any
launch."""
import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(x):
    t = _torch()
    return t.from_numpy(np.ascontiguousarray(x).astype(np.float64)).to("cuda:0")


def _run(entry, A, B, C, alpha, beta, p, schedule, levels, base):
    t = _torch()
    m, k = A.shape
    n = B.shape[1]
    dA, dB, dC = _dev(A), _dev(B), _dev(C)
    t.cuda.synchronize()
    args = capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, schedule, levels, base=base,
                          stream=t.cuda.current_stream())
    free0 = t.cuda.mem_get_info()[0]
    st = entry(args)
    t.cuda.synchronize()
    free1 = t.cuda.mem_get_info()[0]
    assert st == capi.WS_OK, capi.wsmul_last_error()
    host = lambda x: x.cpu().numpy().astype(np.int64)
    return host(dC), host(dA), host(dB), free0 - free1, capi.wsmul_get_stats()


CASES = [
    # (schedule, levels, base, beta, first shape, second (smaller) shape, p)
    (capi.WS_TWO_TEMP, 2, capi.WS_BASE_F64_MFMA, 7, (512, 512, 512), (256, 256, 256), 65521),
    (capi.WS_TWO_TEMP, 1, capi.WS_BASE_I8_LIMBS, 0, (1024, 1024, 1024), (300, 260, 190), 1048573),
    (capi.WS_OVERWRITE, 2, capi.WS_BASE_F64_MFMA, 3, (256, 256, 256), (128, 128, 128), 8388593),
    (capi.WS_READONLY_INPLACE, 2, capi.WS_BASE_F64_MFMA, 0, (512, 256, 512), (256, 128, 256), 8388593),
]


def _first_use():
    """The first call on a device looks the array up, which makes the runtime
    map it there; measure allocations only after that."""
    A, B, C = inputs.uniform(1, 8, 8, 8, 65521, with_c=True)
    _run(capi.wsmul_mod_p_noalloc, A, B, C, 1, 0, 65521, capi.WS_CLASSICAL, 0,
         capi.WS_BASE_F64_MFMA)


@pytest.mark.parametrize("schedule,levels,base,beta,first,second,p", CASES)
def test_noalloc_equals_allocating_call(schedule, levels, base, beta, first, second, p):
    _first_use()
    for i, (m, k, n) in enumerate((first, second)):
        print("no-alloc", schedule, levels, base, (m, k, n), flush=True)
        A, B, C = inputs.uniform(700 + 10 * i + schedule, m, k, n, p, with_c=True)
        want, wantA, wantB, _, s_ex = _run(capi.wsmul_mod_p_ex, A, B, C, 5, beta, p,
                                           schedule, levels, base)
        got, gotA, gotB, grew, s = _run(capi.wsmul_mod_p_noalloc, A, B, C, 5, beta, p,
                                        schedule, levels, base)
        assert np.array_equal(got, want), (m, k, n)
        assert np.array_equal(gotA, wantA) and np.array_equal(gotB, wantB)
        assert np.array_equal(got, ref.matmul_mod_p(A, B, C, 5, beta, p))
        assert s.internal_alloc_bytes == 0 and s.workspace_bytes == s_ex.workspace_bytes
        assert grew == 0, "device memory was allocated during the call"


def test_noalloc_refuses_what_does_not_fit():
    t = _torch()
    p = 65521
    m = k = n = 6000              # Table 1: two 3000 x 3000 temporaries, 144 MB
    A, B, _ = inputs.uniform(9, m, k, n, p)
    dA, dB = _dev(A), _dev(B)
    dC = t.full((m, n), 3.0, dtype=t.float64, device="cuda:0")
    args = capi.make_args(m, k, n, p, dA, dB, dC, 1, 0, capi.WS_TWO_TEMP, 1,
                          stream=t.cuda.current_stream())
    assert capi.wsmul_mod_p_noalloc(args) == capi.WS_ENOMEM
    assert "static scratch" in capi.wsmul_last_error()
    t.cuda.synchronize()
    assert bool((dC == 3.0).all())
    ws = t.empty(16, dtype=t.float64, device="cuda:0")
    small = capi.make_args(64, 64, 64, p, dA, dB, dC, 1, 0, capi.WS_TWO_TEMP, 1,
                           stream=t.cuda.current_stream(), workspace=ws, workspace_bytes=128)
    assert capi.wsmul_mod_p_noalloc(small) == capi.WS_EINVAL
