"""Helpers for GPU tests: move seeded inputs to cuda:0 and call the C-ABI."""
import numpy as np

from paper_0707_2347_amd import capi


def torch():
    import torch as t
    return t


def to_dev(x, dtype):
    t = torch()
    tdt = t.float64 if dtype == capi.WS_F64 else t.int64
    return t.from_numpy(np.ascontiguousarray(x).astype(np.float64 if dtype == capi.WS_F64
                                                       else np.int64)).to("cuda:0").to(tdt)


def to_host(x):
    return x.cpu().numpy().astype(np.int64)


def call(schedule, A, B, C, alpha, beta, p, levels, *, dtype=capi.WS_F64, base=capi.WS_BASE_F64_MFMA,
         flags=0, workspace=None, workspace_bytes=0, blocks=0):
    """Run one product on cuda:0; return (status, C, A, B) as int64 numpy arrays."""
    t = torch()
    m, k = A.shape
    n = B.shape[1]
    dA, dB = to_dev(A, dtype), to_dev(B, dtype)
    dC = to_dev(C if C is not None else np.zeros((m, n), np.int64), dtype)
    stream = t.cuda.current_stream()
    args = capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, schedule, levels, dtype=dtype,
                          base=base, stream=stream, flags=flags, workspace=workspace,
                          workspace_bytes=workspace_bytes, blocks=blocks)
    st = capi.wsmul_mod_p_ex(args)
    t.cuda.synchronize()
    return st, to_host(dC), to_host(dA), to_host(dB)
