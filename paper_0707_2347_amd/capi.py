"""ctypes binding of libwsmul.so (the C-ABI of include/wsmul.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Matrix arguments may be torch tensors on the GPU (their data_ptr()
is passed) or integer device addresses.  The functions keep the C names and
return the C status codes; :func:`check` turns a non-zero status into an
exception carrying wsmul_last_error().
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwsmul.so")

# ws_status
WS_OK, WS_EINVAL, WS_ESHAPE, WS_EMODULUS, WS_ERANGE, WS_ESCHEDULE, WS_ENOMEM, WS_EHIP = range(8)
# ws_schedule
(WS_CLASSICAL, WS_TWO_TEMP, WS_OVERWRITE, WS_READONLY_INPLACE, WS_HL_THREE_TEMP, WS_AUTO,
 WS_OVR, WS_ACCR, WS_BLOCKED, WS_BLOCKED_ACC, WS_OVL, WS_ACR, WS_IPMM_ACC) = range(13)
WS_F64, WS_I64 = 0, 1
WS_BASE_AUTO, WS_BASE_F64_MFMA, WS_BASE_I8_LIMBS = 0, 1, 2
WS_FLAG_CHECK, WS_FLAG_NOFUSE, WS_FLAG_TRACE, WS_FLAG_SYNC = 1, 2, 4, 8
(WS_TILE_BIG128, WS_TILE_LDS128, WS_TILE_DMA64, WS_TILE_LDS64, WS_TILE_DMA32,
 WS_TILE_SK32, WS_TILE_DMA16) = range(7)
WS_TILE_KINDS = 7
WS_MAX_IN, WS_MAX_OUT = 8, 6
WSMUL_NOALLOC_SCRATCH_BYTES = 128 << 20
WS_ROWS = 13
WS_ROW_ADD, WS_ROW_MUL, WS_ROW_ACC = 0, 1, 2
WS_COEF_ONE, WS_COEF_MINUS_ONE, WS_COEF_BETA, WS_COEF_MINUS_BETA = 1, 2, 3, 4
WS_ROW_MAX_TEMPS, WS_ROW_MAX_ROWS = 4, 64
WS_BUF_A, WS_BUF_B, WS_BUF_C, WS_BUF_W = 0, 1, 2, 3
WS_OP_ADD, WS_OP_GEMM = 0, 1
WS_FORM_RESIDUES, WS_FORM_DIGITS_A, WS_FORM_DIGITS_B = 0, 1, 2

SCHEDULES = {"classical": WS_CLASSICAL, "two_temp": WS_TWO_TEMP, "overwrite": WS_OVERWRITE,
             "readonly_inplace": WS_READONLY_INPLACE, "hl_three_temp": WS_HL_THREE_TEMP,
             "auto": WS_AUTO, "ovr": WS_OVR, "accr": WS_ACCR, "blocked": WS_BLOCKED,
             "blocked_acc": WS_BLOCKED_ACC, "ovl": WS_OVL, "acr": WS_ACR,
             "ipmm_acc": WS_IPMM_ACC}

_i64, _i32, _u32, _u64, _vp, _dbl = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double)


class ws_args(ctypes.Structure):
    _fields_ = [("m", _i64), ("k", _i64), ("n", _i64), ("p", _i64),
                ("lda", _i64), ("ldb", _i64), ("ldc", _i64),
                ("alpha", _i64), ("beta", _i64),
                ("A", _vp), ("B", _vp), ("C", _vp),
                ("dtype", _i32), ("schedule", _i32), ("levels", _i32), ("base", _i32),
                ("workspace", _vp), ("workspace_bytes", _u64),
                ("stream", _vp), ("flags", _u32), ("blocks", _u32)]


class ws_stats(ctypes.Structure):
    _fields_ = [("workspace_bytes", _u64), ("peak_temp_bytes", _u64),
                ("internal_alloc_bytes", _u64), ("add_launches", _u64),
                ("gemm_launches", _u64), ("element_additions", _u64),
                ("base_flops", _u64), ("rows", _u64), ("levels", _u64),
                ("schedule", _i64), ("base", _i64), ("scratch_bytes", _u64),
                ("batch_phases", _u64), ("live_alloc_bytes", _u64)]


class ws_row(ctypes.Structure):
    _fields_ = [("op", _i32), ("dst", _i32), ("x", _i32), ("y", _i32),
                ("cx", _i32), ("cy", _i32), ("cs", _i32), ("sign", _i32)]


class ws_trace(ctypes.Structure):
    _fields_ = [("add_launches", _u64), ("gemm_launches", _u64),
                ("add_ms", _dbl), ("gemm_ms", _dbl), ("add_bytes", _dbl), ("gemm_flops", _dbl),
                ("split_launches", _u64), ("split_ms", _dbl), ("split_bytes", _dbl),
                ("digit_adds", _u64), ("unsplit_operands", _u64)]


class ws_view(ctypes.Structure):
    _fields_ = [("buf", _i32), ("form", _i32), ("off", _i64), ("rows", _i64),
                ("cols", _i64), ("ld", _i64)]


class ws_op_desc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("nin", _i32), ("nout", _i32), ("depth", _i32),
                ("alpha", _i64), ("a", ws_view), ("b", ws_view),
                ("in_", ws_view * WS_MAX_IN), ("out", ws_view * WS_MAX_OUT),
                ("coef", (_i64 * WS_MAX_IN) * WS_MAX_OUT)]


_lib = None


def lib():
    """Load libwsmul.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libwsmul.so is not built: run __graft_entry__.build() "
                               "(no other implementation exists)")
        # The torch wheel ships its own HIP runtime.  Load it before the
        # library so that both bind to that one runtime (the one that owns the
        # tensors and streams passed in); opened first, the library would bring
        # the system runtime in beside it and find no device for its launches.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "wsmul_mod_p": (ctypes.c_int, [_i64, _i64, _i64, _i64, _vp, _vp, _vp, _i64, _i64,
                                           ctypes.c_int, ctypes.c_int]),
            "wsmul_mod_p_i64": (ctypes.c_int, [_i64, _i64, _i64, _i64, _vp, _vp, _vp, _i64,
                                               _i64, ctypes.c_int, ctypes.c_int]),
            "wsmul_mod_p_ex": (ctypes.c_int, [ctypes.POINTER(ws_args)]),
            "wsmul_mod_p_noalloc": (ctypes.c_int, [ctypes.POINTER(ws_args)]),
            "wsmul_mod_p_rows": (ctypes.c_int, [ctypes.POINTER(ws_args), ctypes.POINTER(ws_row),
                                                ctypes.c_int, ctypes.c_int]),
            "wsmul_register_rows": (ctypes.c_int, [ctypes.POINTER(ws_row), ctypes.c_int,
                                                   ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
            "wsmul_workspace_bytes": (ctypes.c_size_t, [_i64, _i64, _i64, ctypes.c_int,
                                                        ctypes.c_int, ctypes.c_int,
                                                        ctypes.c_int]),
            "wsmul_set_workspace": (ctypes.c_int, [_vp, ctypes.c_size_t]),
            "wsmul_set_stream": (ctypes.c_int, [_vp]),
            "wsmul_get_stats": (ctypes.c_int, [ctypes.POINTER(ws_stats)]),
            "wsmul_get_trace": (ctypes.c_int, [ctypes.POINTER(ws_trace)]),
            "wsmul_reset_stats": (ctypes.c_int, []),
            "wsmul_last_error": (ctypes.c_char_p, []),
            "wsmul_schedule_name": (ctypes.c_char_p, [ctypes.c_int]),
            "wsmul_version": (ctypes.c_char_p, []),
            "wsmul_plan_info": (ctypes.c_int, [ctypes.POINTER(ws_args),
                                               ctypes.POINTER(ws_stats)]),
            "wsmul_plan_export": (ctypes.c_int, [ctypes.POINTER(ws_args),
                                                 ctypes.POINTER(ws_op_desc), _i64,
                                                 ctypes.POINTER(_i64)]),
            "wsmul_batched": (ctypes.c_int, [ctypes.POINTER(ws_args), ctypes.c_int, _u32]),
            "wsmul_graph_capture": (ctypes.c_int, [ctypes.POINTER(ws_args), ctypes.c_int,
                                                   ctypes.POINTER(_vp)]),
            "wsmul_graph_launch": (ctypes.c_int, [_vp, _vp]),
            "wsmul_graph_check": (ctypes.c_int, [_vp, _vp]),
            "wsmul_graph_destroy": (ctypes.c_int, [_vp]),
            "wsmul_autotune": (ctypes.c_int, [_i64, _i64, _i64, _i64, ctypes.c_int,
                                              ctypes.c_size_t, ctypes.POINTER(ws_args)]),
            "wsmul_tune_tiles": (ctypes.c_int, [_i64, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(_dbl)]),
            "wsmul_set_tile": (ctypes.c_int, [_i64, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int]),
            "wsmul_tune_plan": (ctypes.c_int, [ctypes.POINTER(ws_args), ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


class WsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("wsmul status %d: %s" % (status, message))
        self.status = status


def check(status):
    if status != WS_OK:
        raise WsError(status, lib().wsmul_last_error().decode())
    return status


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


# ------------------------------------------------------------ entry points
def wsmul_mod_p(m, k, n, p, A, B, C, alpha, beta, schedule, levels):
    return lib().wsmul_mod_p(m, k, n, p, _ptr(A), _ptr(B), _ptr(C), alpha, beta,
                             schedule, levels)


def wsmul_mod_p_i64(m, k, n, p, A, B, C, alpha, beta, schedule, levels):
    return lib().wsmul_mod_p_i64(m, k, n, p, _ptr(A), _ptr(B), _ptr(C), alpha, beta,
                                 schedule, levels)


def make_args(m, k, n, p, A=None, B=None, C=None, alpha=1, beta=0, schedule=WS_TWO_TEMP,
              levels=1, dtype=WS_F64, base=WS_BASE_F64_MFMA, lda=0, ldb=0, ldc=0,
              workspace=None, workspace_bytes=0, stream=None, flags=0, blocks=0):
    a = ws_args()
    a.m, a.k, a.n, a.p = m, k, n, p
    a.lda, a.ldb, a.ldc = lda, ldb, ldc
    a.alpha, a.beta = alpha, beta
    a.A, a.B, a.C = _ptr(A), _ptr(B), _ptr(C)
    a.dtype, a.schedule, a.levels, a.base = dtype, schedule, levels, base
    a.workspace, a.workspace_bytes = _ptr(workspace), workspace_bytes
    a.stream = _stream(stream)
    a.flags = flags
    a.blocks = blocks
    return a


def wsmul_mod_p_ex(args):
    return lib().wsmul_mod_p_ex(ctypes.byref(args))


def make_rows(rows):
    """A ctypes array of ws_row from (op, dst, x, y, cx, cy, cs, sign) tuples."""
    arr = (ws_row * len(rows))()
    for r, t in zip(arr, rows):
        r.op, r.dst, r.x, r.y, r.cx, r.cy, r.cs, r.sign = t
    return arr


def wsmul_mod_p_rows(args, rows, ntemps):
    arr = rows if isinstance(rows, ctypes.Array) else make_rows(rows)
    return lib().wsmul_mod_p_rows(ctypes.byref(args), arr, len(arr), ntemps)


def wsmul_register_rows(rows, ntemps):
    """Return (status, id) of a registered row schedule."""
    arr = rows if isinstance(rows, ctypes.Array) else make_rows(rows)
    out = ctypes.c_int(0)
    st = lib().wsmul_register_rows(arr, len(arr), ntemps, ctypes.byref(out))
    return st, out.value


def wsmul_mod_p_noalloc(args):
    return lib().wsmul_mod_p_noalloc(ctypes.byref(args))


def wsmul_workspace_bytes(m, k, n, dtype, schedule, levels, beta_nonzero):
    return lib().wsmul_workspace_bytes(m, k, n, dtype, schedule, levels, int(beta_nonzero))


def wsmul_set_workspace(ptr, nbytes):
    return lib().wsmul_set_workspace(_ptr(ptr), nbytes)


def wsmul_set_stream(stream):
    return lib().wsmul_set_stream(_stream(stream))


def wsmul_get_stats():
    s = ws_stats()
    check(lib().wsmul_get_stats(ctypes.byref(s)))
    return s


def wsmul_get_trace():
    t = ws_trace()
    check(lib().wsmul_get_trace(ctypes.byref(t)))
    return t


def wsmul_reset_stats():
    return lib().wsmul_reset_stats()


def wsmul_last_error():
    return lib().wsmul_last_error().decode()


def wsmul_schedule_name(table):
    return lib().wsmul_schedule_name(table).decode()


def wsmul_plan_info(args):
    s = ws_stats()
    check(lib().wsmul_plan_info(ctypes.byref(args), ctypes.byref(s)))
    return s


def wsmul_plan_export(args):
    cnt = _i64(0)
    check(lib().wsmul_plan_export(ctypes.byref(args), None, 0, ctypes.byref(cnt)))
    ops = (ws_op_desc * max(cnt.value, 1))()
    check(lib().wsmul_plan_export(ctypes.byref(args), ops, cnt.value, ctypes.byref(cnt)))
    return list(ops)[:cnt.value]


def wsmul_batched(args_list, flags=0):
    arr = (ws_args * max(len(args_list), 1))(*args_list)
    return lib().wsmul_batched(arr, len(args_list), flags)


def wsmul_graph_capture(args_list):
    arr = (ws_args * max(len(args_list), 1))(*args_list)
    h = _vp()
    st = lib().wsmul_graph_capture(arr, len(args_list), ctypes.byref(h))
    return st, h.value


def wsmul_graph_launch(handle, stream=None):
    return lib().wsmul_graph_launch(handle, _stream(stream))


def wsmul_graph_check(handle, stream=None):
    return lib().wsmul_graph_check(handle, _stream(stream))


def wsmul_graph_destroy(handle):
    return lib().wsmul_graph_destroy(handle)


def wsmul_autotune(m, k, n, p, dtype=WS_F64, mem_budget=(1 << 64) - 1, schedule=WS_AUTO,
                   levels=-1, base=WS_BASE_AUTO, beta=0, blocks=0):
    """Return (status, schedule, levels, base, blocks) chosen for one product."""
    c = ws_args()
    c.schedule, c.levels, c.base, c.beta, c.blocks = schedule, levels, base, beta, blocks
    st = lib().wsmul_autotune(m, k, n, p, dtype, mem_budget, ctypes.byref(c))
    return st, c.schedule, c.levels, c.base, c.blocks


def wsmul_tune_tiles(m, k, n, p, dtype=WS_F64, reps=5):
    """Return (status, kind kept, per-kind microseconds) for one product shape."""
    best = ctypes.c_int(-1)
    times = (_dbl * WS_TILE_KINDS)()
    st = lib().wsmul_tune_tiles(m, k, n, p, dtype, reps, ctypes.byref(best), times)
    return st, best.value, list(times)


def wsmul_set_tile(m, k, n, p, dtype, kind):
    return lib().wsmul_set_tile(m, k, n, p, dtype, kind)


def wsmul_tune_plan(args, reps=5):
    return lib().wsmul_tune_plan(ctypes.byref(args), reps)
