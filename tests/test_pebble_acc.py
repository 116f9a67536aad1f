"""The schedule search of Section 4 for the accumulating product
C <- alpha*A*B + beta*C with read-only inputs (tests/pebble_acc.py).

* The two computation graphs (Table 9's and Table 2's) compute alpha*A*B +
  beta*C: evaluated on formal symbols, their four results are that identity
  (so the graphs themselves are pinned, independently of any schedule).
* On Table 9's graph the search finds no schedule with 0 or 1 temporaries
  and finds one with 2, the count of Table 9; on Table 2's graph it needs 3,
  the count of Table 2.  With 2 temporaries Table 9's graph needs 10
  pre-additions (two formed twice, as Table 9 does), with 3 it needs 8.
* The stored schedules (tests/golden/acc_search.json, written by
  tests/golden/make_acc_search.py) are what the search finds; replayed on
  physical blocks of formal symbols with every read checked they leave
  exactly alpha*A*B + beta*C in C and A, B untouched, and on residues they
  equal the oracle's product.  The Table 9 graph's schedule places its
  values differently from Table 9 itself.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import inputs

from . import pebble_acc as pa
from .test_oracle_symbolic import Sym

sys.setrecursionlimit(10000)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "acc_search.json")
P = 65521


def _sym_blocks():
    a = [Sym.atom(("a", i // 2, i % 2)) for i in range(4)]
    b = [Sym.atom(("b", i // 2, i % 2)) for i in range(4)]
    c = [Sym.atom(("c", i // 2, i % 2)) for i in range(4)]
    return a, b, c


def _want(a, b, c, alpha, beta):
    prod = [a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
            a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]]
    return [x * alpha + y * beta for x, y in zip(prod, c)]


@pytest.mark.parametrize("graph", ["table9", "table2"])
def test_graph_computes_the_accumulating_product(graph):
    """Evaluate the graph node by node on formal symbols (alpha = 3, beta = 5
    over Z/p): the four results are alpha*A*B + beta*C."""
    g = pa.GRAPHS[graph]
    a, b, c = _sym_blocks()
    env = dict(zip(("A11", "A12", "A21", "A22"), a))
    env.update(zip(("B11", "B12", "B21", "B22"), b))
    env.update(zip(pa.C_IN, c))
    left = set(g)
    while left:
        for v in list(left):
            if all(u in env for u in pa.parents(g, v)):
                env[v] = pa.value_of(g, v, env, 3, 5, lambda x, y: x * y)
                left.discard(v)
    got = [env[v] for v, _ in sorted(pa.FINAL.items(), key=lambda kv: kv[1])]
    assert all(x == y for x, y in zip(got, _want(a, b, c, 3, 5)))


@pytest.mark.parametrize("graph,fewer", [("table9", [0, 1]), ("table2", [0, 1, 2])])
def test_no_schedule_with_fewer_temporaries(graph, fewer):
    for t in fewer:
        moves, _ = pa.search(graph, t)
        assert moves is None, (graph, t)


def test_table9_graph_fits_two_temporaries():
    moves, _ = pa.search("table9", 2)
    assert moves is not None
    rows = pa.to_rows("table9", moves, 2)
    a, b, c = _sym_blocks()
    got = pa.run_rows("table9", rows, a, b, c, 3, 5, None, lambda x, y: x * y)
    assert all(x == y for x, y in zip(got, _want(a, b, c, 3, 5)))


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("graph", ["table9", "table2"])
def test_stored_schedule_is_exact(graph):
    d = _golden()[graph]
    rows = [(v, kind, block, tuple(bl)) for v, kind, block, bl in d["rows"]]
    # the stored rows are the physical placement of the stored moves
    assert rows == pa.to_rows(graph, [tuple(m) for m in d["moves"]], d["temps"])
    a, b, c = _sym_blocks()
    got = pa.run_rows(graph, rows, a, b, c, 7, 11, None, lambda x, y: x * y)
    assert all(x == y for x, y in zip(got, _want(a, b, c, 7, 11)))
    # no row writes A or B, and the library's records name the same blocks
    assert all(block not in pa.A_IN for _, _, block, _ in rows)
    assert len(d["library_rows"]) == len(rows)
    assert [tuple(r) for r in d["library_rows"]] == pa.library_rows(graph, rows)


@pytest.mark.parametrize("graph", ["table9", "table2"])
@pytest.mark.parametrize("p", [P, 8388593])
def test_stored_schedule_on_residues(graph, p):
    d = _golden()[graph]
    rows = [(v, kind, block, tuple(bl)) for v, kind, block, bl in d["rows"]]
    n = 32
    A, B, C = inputs.uniform(5, n, n, n, p, with_c=True)
    q = lambda M: [M[:16, :16], M[:16, 16:], M[16:, :16], M[16:, 16:]]
    alpha, beta = 3, p - 2
    got = pa.run_rows(graph, rows, q(A), q(B), q(C), alpha, beta, p,
                      lambda x, y: ref.matmul_mod_p(x, y, None, 1, 0, p))
    want = ref.matmul_mod_p(A, B, C, alpha, beta, p)
    assert all(np.array_equal(x, y) for x, y in zip(got, q(want)))


def test_stored_counts_and_difference_from_table9():
    d = _golden()
    assert d["table9"]["temps"] == 2 and d["table9"]["pre_additions"] == 10
    assert set(d["table9"]["no_schedule_with_temps"]) == {"0", "1"}
    assert set(d["table9"]["no_schedule_with_pre_additions"]) == {"8", "9"}
    assert d["table2"]["temps"] == 3 and d["table2"]["pre_additions"] == 8
    # Table 9 keeps S blocks in X and T blocks in Y and never writes a
    # pre-addition into C; the found schedule does not follow that placement.
    placements = {(v, block) for v, kind, block, _ in d["table9"]["rows"] if kind == "pre"}
    table9 = {("S1", "X"), ("T1", "Y"), ("S2", "X"), ("T2", "Y"), ("S4", "X"),
              ("S3", "X"), ("T3", "Y"), ("T4", "Y")}
    assert placements != table9


# ------------------------------------------------- the planner runs the rows
def _interp_rows(graph, n, levels, p, alpha, beta, seed, fuse=True):
    from paper_0707_2347_amd import capi
    from . import plan_interp
    d = _golden()[graph]
    st, sid = capi.wsmul_register_rows([tuple(r) for r in d["library_rows"]], d["temps"])
    assert st == capi.WS_OK, capi.wsmul_last_error()
    A, B, C = inputs.uniform(seed, n, n, n, p, with_c=True)
    args = capi.make_args(n, n, n, p, alpha=alpha, beta=beta, schedule=capi.WS_ROWS,
                          levels=levels, blocks=sid, flags=0 if fuse else capi.WS_FLAG_NOFUSE)
    info = capi.wsmul_plan_info(args)
    ops = capi.wsmul_plan_export(args)
    rng = np.random.default_rng(seed)
    W = rng.integers(0, p, size=max(info.workspace_bytes // 8, 1))     # garbage temporaries
    bufs = [A.copy().ravel(), B.copy().ravel(), C.copy().ravel(), W]
    plan_interp.run(ops, bufs, p)
    return (A, B, C), bufs, info


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("graph,temps", [("table9", 2), ("table2", 3)])
@pytest.mark.parametrize("n,levels", [(16, 1), (32, 2), (64, 3)])
def test_planner_runs_the_stored_rows(graph, temps, n, levels, fuse):
    """The library's data-driven emitter expands the stored rows at every
    level (plain products as Table 1, accumulating ones into the same rows):
    the plan, run by the numpy stand-in on garbage temporaries, equals the
    oracle, leaves A and B untouched, and its workspace is `temps` blocks of
    a quarter of C per level."""
    p = 8388593 if levels % 2 else 65521
    (A, B, C), bufs, info = _interp_rows(graph, n, levels, p, 6, p - 3, n + levels, fuse=fuse)
    assert np.array_equal(bufs[2].reshape(n, n), ref.matmul_mod_p(A, B, C, 6, p - 3, p))
    assert np.array_equal(bufs[0].reshape(n, n), A) and np.array_equal(bufs[1].reshape(n, n), B)
    assert info.workspace_bytes == 8 * temps * sum((n >> i) ** 2 for i in range(1, levels + 1))


def test_row_schedule_argument_errors():
    from paper_0707_2347_amd import capi
    d = _golden()["table9"]
    rows = [tuple(r) for r in d["library_rows"]]
    bad_dst = [(0, 5, 0, 1, 1, 1, 0, 0)] + rows[1:]                 # writes A12
    self_mul = [(1, 12, 12, 13, 0, 0, 0, 1)] + rows[1:]             # product on its operand
    for r, t in [(bad_dst, 2), (self_mul, 2), (rows, 5), ([(0, 16, 0, 1, 1, 1, 0, 0)], 2)]:
        st, _ = capi.wsmul_register_rows(r, t)
        assert st == capi.WS_EINVAL
    st, sid = capi.wsmul_register_rows(rows, 2)
    assert st == capi.WS_OK
    st2, sid2 = capi.wsmul_register_rows(rows, 2)
    assert sid2 == sid                                             # equal rows, equal id
    def info_status(m, k, n, levels, blocks):
        import ctypes
        args = capi.make_args(m, k, n, 65521, schedule=capi.WS_ROWS, levels=levels, blocks=blocks)
        return capi.lib().wsmul_plan_info(ctypes.byref(args), ctypes.byref(capi.ws_stats()))
    assert info_status(48, 48, 40, 1, sid) == capi.WS_ESHAPE        # not square
    assert info_status(48, 48, 48, 5, sid) == capi.WS_ESHAPE        # 48 not divisible by 32
    assert info_status(48, 48, 48, 1, 4095) == capi.WS_ESCHEDULE    # no such schedule
    assert info_status(48, 48, 48, 1, sid) == capi.WS_OK
