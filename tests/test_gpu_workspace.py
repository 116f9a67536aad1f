"""Device-measured temporaries: the workspace a schedule reports is exactly
the memory its launches touch.  The workspace and a guard band behind it are
filled with a sentinel that is not a residue; after the product every
workspace entry holds a residue (all of it was used) and the guard band still
holds the sentinel (nothing beyond it was written)."""
import numpy as np
import pytest

from oracle import ref
from oracle.schedules import replay_shape
from paper_0707_2347_amd import capi, inputs

from .gpu_util import call

pytestmark = pytest.mark.gpu

GUARD = 4096
SENTINEL = -7.0

CASES = [
    # selector, shape, levels, beta, blocks, oracle schedule (for the count)
    (capi.WS_TWO_TEMP, (256, 256, 256), 3, 0, 0, "t1"),
    (capi.WS_TWO_TEMP, (256, 128, 384), 2, 0, 0, "t1"),
    (capi.WS_TWO_TEMP, (256, 256, 256), 3, 5, 0, "acc"),
    (capi.WS_HL_THREE_TEMP, (256, 384, 128), 2, 5, 0, "hl"),
    (capi.WS_OVERWRITE, (256, 256, 256), 2, 5, 0, "aclr"),
    (capi.WS_OVR, (256, 256, 256), 3, 0, 0, "ovr"),
    (capi.WS_OVL, (256, 256, 256), 3, 0, 0, "ovl"),
    (capi.WS_ACCR, (256, 256, 256), 2, 5, 0, "accr"),
    (capi.WS_ACR, (256, 128, 512), 2, 5, 0, "acr"),
    (capi.WS_BLOCKED, (384, 384, 384), 2, 5, 3, "blocked"),
    (capi.WS_BLOCKED_ACC, (256, 256, 256), 2, 5, 2, "blocked_acc"),
]


@pytest.mark.parametrize("schedule,shape,levels,beta,blocks,name", CASES)
def test_workspace_touched_is_the_reported_count(schedule, shape, levels, beta, blocks, name):
    torch = __import__("torch")
    m, k, n = shape
    p = 65521
    need = capi.wsmul_plan_info(capi.make_args(m, k, n, p, beta=beta, schedule=schedule,
                                               levels=levels, blocks=blocks)).workspace_bytes
    count = replay_shape(name, m, k, n, p, levels, beta_nonzero=bool(beta), blocks=blocks or 2)
    assert need == 8 * count.peak > 0
    ws = torch.full((need // 8 + GUARD,), SENTINEL, dtype=torch.float64, device="cuda:0")
    A, B, C = inputs.uniform(81, m, k, n, p, with_c=True)
    st, C2, _, _ = call(schedule, A, B, C, 4, beta, p, levels, workspace=ws,
                        workspace_bytes=need, blocks=blocks)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 4, beta, p))
    w = ws.cpu().numpy()
    used, guard = w[:need // 8], w[need // 8:]
    assert np.all(guard == SENTINEL), "written beyond the reported workspace"
    assert np.all((used >= 0) & (used < p)), "part of the reported workspace was never used"
    assert capi.wsmul_get_stats().internal_alloc_bytes == 0
