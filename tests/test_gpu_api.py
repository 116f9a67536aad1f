"""The torch-facing call: strided views, storage types, schedules by name,
errors raised from the library's status codes."""
import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import api, capi, inputs

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    import torch
    return torch.from_numpy(x.astype(np.float64 if dtype == "f64" else np.int64)).cuda()


@pytest.mark.parametrize("dtype", ["f64", "i64"])
@pytest.mark.parametrize("schedule,levels,beta", [("auto", -1, 5), ("two_temp", 2, 0),
                                                  ("blocked", 1, 3), ("hl_three_temp", 1, 7)])
def test_views_and_schedules(dtype, schedule, levels, beta):
    import torch
    p = 1048573
    A, B, C = inputs.uniform(61, 300, 260, 200, p, with_c=True)
    big = _dev(np.zeros((320, 300), np.int64), dtype)
    dA = big[10:310, 20:280]                 # a strided view, lda = 300
    dA.copy_(_dev(A, dtype))
    dB, dC = _dev(B, dtype), _dev(C, dtype)
    out = api.mod_p_matmul(dA, dB, dC, p=p, alpha=9, beta=beta, schedule=schedule,
                           levels=levels, blocks=2)
    torch.cuda.synchronize()
    assert out is dC
    assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref.matmul_mod_p(A, B, C, 9, beta, p))
    assert np.array_equal(dA.cpu().numpy().astype(np.int64), A)


def test_allocates_c_and_raises_on_bad_input():
    import torch
    p = 65521
    A, B, _ = inputs.uniform(62, 64, 64, 64, p)
    dA, dB = _dev(A, "f64"), _dev(B, "f64")
    C = api.mod_p_matmul(dA, dB, p=p, schedule="readonly_inplace", levels=2)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.int64), ref.matmul_mod_p(A, B, None, 1, 0, p))
    with pytest.raises(capi.WsError) as e:
        api.mod_p_matmul(dA, dB, C, p=p, beta=1, schedule="readonly_inplace", levels=1)
    assert e.value.status == capi.WS_ESCHEDULE
    dA[0, 0] = p
    with pytest.raises(capi.WsError) as e:
        api.mod_p_matmul(dA, dB, C, p=p, schedule="two_temp", levels=1, check=True)
    assert e.value.status == capi.WS_ERANGE
    with pytest.raises(ValueError):
        api.mod_p_matmul(dA, dB.t(), C, p=p)  # column-major view
