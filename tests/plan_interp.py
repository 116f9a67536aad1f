"""Run an exported plan (wsmul_plan_export) with numpy on flat host buffers.

A stand-in for the device: it executes the operation list exactly as the
header documents it (elementwise groups and base products with epilogues),
so planner, fusion, peeling and workspace placement can be checked on the
CPU against the oracle.  It computes nothing on its own account -- it is not
an oracle.
"""
import numpy as np

from paper_0707_2347_amd import capi


def _view(buf, v):
    if v.rows == 0 or v.cols == 0:
        return np.zeros((v.rows, v.cols), dtype=np.int64)
    need = v.off + (v.rows - 1) * v.ld + v.cols
    assert 0 <= v.off and need <= buf.size, "view outside its buffer"
    return np.lib.stride_tricks.as_strided(buf[v.off:], shape=(v.rows, v.cols),
                                           strides=(v.ld * 8, 8))


def _modprod(X, Y, p):
    s = np.zeros((X.shape[0], Y.shape[1]), dtype=np.int64)
    step = max(1, (2**62) // max((p - 1) ** 2, 1))
    for l0 in range(0, X.shape[1], step):
        s = (s + X[:, l0:l0 + step] @ Y[l0:l0 + step, :]) % p
    return s


POISON = -(1 << 40)    # stands for bytes that hold digit planes: never a residue


def _span(v):
    return v.off, v.off + (v.rows - 1) * v.ld + v.cols


def _meets(v, w):
    if v.buf != w.buf or 0 in (v.rows, v.cols, w.rows, w.cols):
        return False
    a0, a1 = _span(v)
    b0, b1 = _span(w)
    return a0 < b1 and b0 < a1


def _key(v):
    return (v.buf, v.off, v.rows, v.cols, v.ld)


def _check_planes_view(v, form):
    """The layout conditions the device needs for a view held as digit planes."""
    assert v.buf == capi.WS_BUF_W and v.ld == v.cols and v.off % 2 == 0, "planes view not dense"
    if form == capi.WS_FORM_DIGITS_A:
        assert v.rows % 128 == 0 and v.cols % 64 == 0, "A-role planes need whole tiles"
    else:
        assert form == capi.WS_FORM_DIGITS_B, "unknown form"
        assert v.cols % 128 == 0 and v.rows % 64 == 0, "B-role planes need whole tiles"


def run(ops, bufs, p):
    """bufs: [A, B, C, W] flat int64 arrays, modified in place.

    Views whose form is a digit-plane form (the digit base's execution list)
    are kept aside, keyed by view and form, while their block is overwritten
    with a value that is no residue: a read of such a block as residues, a
    read of planes nobody wrote, or a group that reads a view in one form and
    writes it in another (on the device its workgroups would overwrite bytes
    others still read) fails.  Views of A and B with a form read the inputs
    as they were at the start (planes of the whole input)."""
    planes = {}
    # Views of A or B with a form read planes of the whole input, split at
    # the start of the call: the plan must never write that input.
    originals = [bufs[0].copy(), bufs[1].copy()]
    views = [v for op in ops for v in ([op.a, op.b] if op.kind == capi.WS_OP_GEMM else []) +
             [op.in_[i] for i in range(op.nin)]]
    for b in (capi.WS_BUF_A, capi.WS_BUF_B):
        if any(v.form and v.buf == b for v in views):
            assert not any(op.out[o].buf == b for op in ops for o in range(op.nout)), \
                "an input read as planes is written"

    def read(v):
        if v.form and v.buf in (capi.WS_BUF_A, capi.WS_BUF_B):
            r0, c0 = divmod(v.off, v.ld)
            if v.form == capi.WS_FORM_DIGITS_A:
                assert v.buf == capi.WS_BUF_A and r0 % 128 == 0 and v.rows % 128 == 0 and \
                    c0 % 64 == 0 and v.cols % 64 == 0, "A planes need whole tiles"
            else:
                assert v.buf == capi.WS_BUF_B and c0 % 128 == 0 and v.cols % 128 == 0 and \
                    r0 % 64 == 0 and v.rows % 64 == 0, "B planes need whole tiles"
            return _view(originals[v.buf], v).copy()
        if v.form:
            _check_planes_view(v, v.form)
            assert (_key(v), v.form) in planes, "digit planes read before they were written"
            return planes[(_key(v), v.form)].copy()
        x = _view(bufs[v.buf], v).copy()
        assert not np.any(x == POISON), "residues read from a block that holds digit planes"
        return x

    def write(v, x):
        for k in [k for k in planes if _meets(v, _Viewish(k[0]))]:
            del planes[k]
        if v.form:
            _check_planes_view(v, v.form)
            planes[(_key(v), v.form)] = x
            _view(bufs[v.buf], v)[...] = POISON
        else:
            _view(bufs[v.buf], v)[...] = x

    for op in ops:
        nin, nout = op.nin, op.nout
        ins = [None] * nin
        if op.kind == capi.WS_OP_GEMM:
            a = read(op.a)
            b = read(op.b)
            ins[0] = (op.alpha % p) * _modprod(a, b, p) % p
            first = 1
        else:
            first = 0
            for i in range(nin):
                for o in range(nout):
                    if _key(op.in_[i]) == _key(op.out[o]):
                        assert op.in_[i].form == op.out[o].form, "view rewritten in another form"
        for i in range(first, nin):
            ins[i] = read(op.in_[i])
        outs = []
        for o in range(nout):
            acc = np.zeros_like(ins[0] if ins[0] is not None else ins[first])
            for i in range(nin):
                acc = (acc + int(op.coef[o][i]) * ins[i]) % p
            outs.append(acc)
        for o in range(nout):
            write(op.out[o], outs[o])


class _Viewish:
    """A view rebuilt from a planes key (for the overlap test)."""

    def __init__(self, key):
        self.buf, self.off, self.rows, self.cols, self.ld = key
