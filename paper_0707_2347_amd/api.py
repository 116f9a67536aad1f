"""Torch-facing call of the C-ABI: C <- (alpha*A*B + beta*C) mod p on cuda
tensors.

Argument marshalling only.  It checks devices, storage types and row-major
strides, passes the leading dimensions and the current stream, and raises
``capi.WsError`` on a non-zero status; every step of the computation runs in
libwsmul.so, which must be built (there is no other implementation).
"""
from . import capi

_SCHEDULES = dict(capi.SCHEDULES)
_BASES = {"auto": capi.WS_BASE_AUTO, "f64": capi.WS_BASE_F64_MFMA, "int8": capi.WS_BASE_I8_LIMBS}


def _ld(t, name):
    """Leading dimension of a row-major 2-D view (unit column stride)."""
    if t.dim() != 2:
        raise ValueError("%s must be a matrix" % name)
    if t.shape[0] > 0 and t.shape[1] > 0 and t.stride(1) != 1:
        raise ValueError("%s must have unit column stride (row-major)" % name)
    return max(t.stride(0), t.shape[1]) if t.shape[0] > 1 else t.shape[1]


def mod_p_matmul(A, B, C=None, *, p, alpha=1, beta=0, schedule="auto", levels=-1, base="auto",
                 blocks=0, workspace=None, stream=None, check=False):
    """C <- (alpha*A*B + beta*C) mod p, in place in ``C`` (allocated when None).

    A (m x k), B (k x n) and C (m x n) are cuda tensors of one storage type,
    float64 holding integers or int64, with entries in [0, p).  ``schedule``
    is a name of ``capi.SCHEDULES`` ("auto", "two_temp", "overwrite",
    "readonly_inplace", "hl_three_temp", "ovr", "accr", "blocked",
    "blocked_acc", "ovl", "acr", "ipmm_acc") or a ws_schedule value;
    ``levels`` -1 and ``base`` "auto" leave the choice to the autotuner;
    ``blocks`` is t of the blocked schedules.  ``workspace`` is an optional
    cuda tensor lent as the schedule's temporaries.  Overwriting schedules
    leave A and/or B in their documented state.  Returns C."""
    import torch
    if C is None:
        C = torch.zeros((A.shape[0], B.shape[1]), dtype=A.dtype, device=A.device)
        beta = 0
    for t, name in ((A, "A"), (B, "B"), (C, "C")):
        if not t.is_cuda:
            raise ValueError("%s must be a cuda tensor" % name)
        if t.dtype not in (torch.float64, torch.int64):
            raise ValueError("%s must hold float64 or int64" % name)
    if not (A.dtype == B.dtype == C.dtype):
        raise ValueError("A, B and C must share one storage type")
    if A.shape[1] != B.shape[0] or C.shape != (A.shape[0], B.shape[1]):
        raise ValueError("shapes do not form a product: %s x %s -> %s"
                         % (tuple(A.shape), tuple(B.shape), tuple(C.shape)))
    sched = _SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    kind = _BASES[base] if isinstance(base, str) else int(base)
    m, k = A.shape
    n = B.shape[1]
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    flags = capi.WS_FLAG_CHECK if check else 0
    args = capi.make_args(m, k, n, int(p), A, B, C, int(alpha), int(beta), sched, int(levels),
                          dtype=capi.WS_F64 if A.dtype == torch.float64 else capi.WS_I64,
                          base=kind, lda=_ld(A, "A"), ldb=_ld(B, "B"), ldc=_ld(C, "C"),
                          workspace=workspace,
                          workspace_bytes=0 if workspace is None
                          else workspace.numel() * workspace.element_size(),
                          stream=stream, flags=flags, blocks=int(blocks))
    with torch.cuda.device(A.device):
        capi.check(capi.wsmul_mod_p_ex(args))
    return C
