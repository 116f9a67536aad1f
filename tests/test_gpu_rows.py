"""GPU parity of schedules found by the search of Section 4 (not tables of
the paper): the stored row lists (tests/golden/acc_search.json) run by the
library's data-driven emitter at one to four levels, on both bases and both
storage types, element by element against the oracle; A and B stay intact
and the workspace is the schedule's count."""
import json
import os

import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

from .gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "acc_search.json")


def _rows(graph):
    with open(GOLDEN) as f:
        d = json.load(f)[graph]
    return [tuple(r) for r in d["library_rows"]], d["temps"]


@pytest.mark.parametrize("graph", ["table9", "table2"])
@pytest.mark.parametrize("n,levels,p,beta", [(256, 1, 65521, 7), (256, 3, 8388593, 0),
                                             (512, 2, 1048573, 5), (1024, 3, 8388593, 9),
                                             (1024, 4, 65521, 1)])
@pytest.mark.parametrize("dtype,base", [(capi.WS_F64, capi.WS_BASE_F64_MFMA),
                                        (capi.WS_I64, capi.WS_BASE_F64_MFMA),
                                        (capi.WS_F64, capi.WS_BASE_I8_LIMBS)])
def test_search_found_schedule(graph, n, levels, p, beta, dtype, base):
    t = __import__("torch")
    rows, temps = _rows(graph)
    print("rows", graph, n, levels, p, beta, dtype, base, flush=True)
    A, B, C = inputs.uniform(n + levels + beta, n, n, n, p, with_c=True)
    dA, dB, dC = to_dev(A, dtype), to_dev(B, dtype), to_dev(C, dtype)
    args = capi.make_args(n, n, n, p, dA, dB, dC, 5, beta, capi.WS_ROWS, levels, dtype=dtype,
                          base=base, stream=t.cuda.current_stream())
    st = capi.wsmul_mod_p_rows(args, rows, temps)
    t.cuda.synchronize()
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(to_host(dC), ref.matmul_mod_p(A, B, C, 5, beta, p))
    assert np.array_equal(to_host(dA), A) and np.array_equal(to_host(dB), B)
    s = capi.wsmul_get_stats()
    assert s.workspace_bytes == 8 * temps * sum((n >> i) ** 2 for i in range(1, levels + 1))


def test_search_found_schedules_in_a_batch():
    """Both found schedules as products of one batch (ws_args.blocks = id)."""
    t = __import__("torch")
    host, dev, args = [], [], []
    for i, graph in enumerate(["table9", "table2", "table9"]):
        rows, temps = _rows(graph)
        st, sid = capi.wsmul_register_rows(rows, temps)
        assert st == capi.WS_OK
        n, p = 256 * (i + 1), 8388593
        A, B, C = inputs.uniform(90 + i, n, n, n, p, with_c=True)
        d = [to_dev(x, capi.WS_F64) for x in (A, B, C)]
        host.append((A, B, C, p))
        dev.append(d)
        args.append(capi.make_args(n, n, n, p, *d, 3, 4, capi.WS_ROWS, 2, blocks=sid,
                                   stream=t.cuda.current_stream()))
    st = capi.wsmul_batched(args, capi.WS_FLAG_SYNC)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    for (A, B, C, p), d in zip(host, dev):
        assert np.array_equal(to_host(d[2]), ref.matmul_mod_p(A, B, C, 3, 4, p))
