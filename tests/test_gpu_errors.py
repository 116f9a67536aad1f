"""GPU tests of the error paths: argument errors write nothing, and a failure
injected from the host in the middle of a plan (WSMUL_FAULT_AT) returns
WS_EHIP, releases the memory the call allocated, and leaves the library
ready for the next call.  No kernel faults: the injected failure stops the
launch loop on the host."""
import os

import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

from .gpu_util import call

pytestmark = pytest.mark.gpu


@pytest.fixture
def fault_at():
    def set_(i):
        os.environ["WSMUL_FAULT_AT"] = str(i)
    yield set_
    os.environ.pop("WSMUL_FAULT_AT", None)


@pytest.mark.parametrize("base", [capi.WS_BASE_F64_MFMA, capi.WS_BASE_I8_LIMBS])
@pytest.mark.parametrize("op", [0, 3, 9])
def test_injected_failure_releases_memory(fault_at, base, op):
    """Table 1 at two levels with the library's own workspace (and, on the
    digit base, its digit scratch): the call fails before operation `op`,
    every byte it allocated is released, and the same call then succeeds."""
    p = 1048573
    m = k = n = 512
    A, B, _ = inputs.uniform(61 + op, m, k, n, p)
    C = np.full((m, n), 5, dtype=np.int64)
    fault_at(op)
    st, C2, A2, B2 = call(capi.WS_TWO_TEMP, A, B, C, 1, 0, p, 2, base=base)
    assert st == capi.WS_EHIP
    assert "WSMUL_FAULT_AT" in capi.wsmul_last_error()
    s = capi.wsmul_get_stats()
    assert s.live_alloc_bytes == 0
    assert np.array_equal(A2, A) and np.array_equal(B2, B)     # read-only schedule
    if op == 0:
        assert np.array_equal(C2, C)                           # nothing was launched
    os.environ.pop("WSMUL_FAULT_AT")
    st, C3, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 1, 0, p, 2, base=base)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C3, ref.matmul_mod_p(A, B, None, 1, 0, p))
    s = capi.wsmul_get_stats()
    assert s.live_alloc_bytes == 0 and s.internal_alloc_bytes > 0


def test_injected_failure_in_an_accumulating_overwrite_plan(fault_at):
    """Table 6 (overwrites A and B) fails half way; the next call on fresh
    inputs is exact."""
    p = 65521
    n = 256
    A, B, C = inputs.uniform(71, n, n, n, p, with_c=True)
    fault_at(20)
    st, _, _, _ = call(capi.WS_OVERWRITE, A, B, C, 3, 4, p, 2)
    assert st == capi.WS_EHIP
    assert capi.wsmul_get_stats().live_alloc_bytes == 0
    os.environ.pop("WSMUL_FAULT_AT")
    st, C2, _, _ = call(capi.WS_OVERWRITE, A, B, C, 3, 4, p, 2)
    assert st == capi.WS_OK
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 3, 4, p))


@pytest.mark.parametrize("case,status", [
    (dict(p=1), capi.WS_EMODULUS), (dict(levels=3, shape=(100, 100, 100), schedule=capi.WS_OVERWRITE),
                                    capi.WS_ESHAPE),
    (dict(schedule=capi.WS_READONLY_INPLACE, beta=3), capi.WS_ESCHEDULE),
    (dict(base=7), capi.WS_EINVAL)])
def test_argument_errors_write_nothing(case, status):
    p = case.get("p", 65521)
    m, k, n = case.get("shape", (64, 64, 64))
    A, B, C = inputs.uniform(81, m, k, n, max(p, 2), with_c=True)
    st, C2, A2, B2 = call(case.get("schedule", capi.WS_TWO_TEMP), A, B, C, 1, case.get("beta", 1),
                          p, case.get("levels", 1), base=case.get("base", capi.WS_BASE_F64_MFMA))
    assert st == status, capi.wsmul_last_error()
    assert np.array_equal(C2, C) and np.array_equal(A2, A) and np.array_equal(B2, B)
