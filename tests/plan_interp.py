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


def run(ops, bufs, p):
    """bufs: [A, B, C, W] flat int64 arrays, modified in place."""
    for op in ops:
        nin, nout = op.nin, op.nout
        ins = [None] * nin
        if op.kind == capi.WS_OP_GEMM:
            a = _view(bufs[op.a.buf], op.a)
            b = _view(bufs[op.b.buf], op.b)
            ins[0] = (op.alpha % p) * _modprod(a, b, p) % p
            first = 1
        else:
            first = 0
        for i in range(first, nin):
            ins[i] = _view(bufs[op.in_[i].buf], op.in_[i]).copy()
        outs = []
        for o in range(nout):
            acc = np.zeros_like(ins[0] if ins[0] is not None else ins[first])
            for i in range(nin):
                acc = (acc + int(op.coef[o][i]) * ins[i]) % p
            outs.append(acc)
        for o in range(nout):
            _view(bufs[op.out[o].buf], op.out[o])[...] = outs[o]
