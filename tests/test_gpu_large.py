"""Addition groups over blocks of 2^31 entries or more.  The elementwise
kernel indexes fewer than 2^31 items per launch, so the library runs such a
group as slices of whole rows.  C = A*B mod p with m = n near 92682 and k = 64
under Table 1 at one level: the post-additions work on C's quadrants of about
46341 x 46341 = 2^31 entries (odd and even row lengths, so both the 8-byte
and the 16-byte access paths), C itself is 69 GB.  Unfused, the
post-additions are addition groups over the quadrants; fused, they are the
epilogues of the quadrant products.  Entries sampled at random, and every
entry of the rows on both sides of each slice boundary, are compared with the
oracle."""
import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

pytestmark = pytest.mark.gpu

LIMIT = (1 << 31) - 1   # elements per slice, as the library cuts them


@pytest.mark.parametrize("m", [92682, 92684])
def test_quadrants_of_two_to_the_31_entries(m):
    """Both plans of one shape, on one allocation."""
    torch = __import__("torch")
    n, k, p = m, 64, 1048573
    h = m // 2
    assert h * h > LIMIT
    need = capi.wsmul_workspace_bytes(m, k, n, capi.WS_F64, capi.WS_TWO_TEMP, 1, 0)
    free, _ = torch.cuda.mem_get_info()
    if free < 8 * m * n + need + (8 << 30):
        pytest.skip("needs %.0f GB of free device memory" % ((8 * m * n + need) / 1e9))
    A, B, _ = inputs.uniform(91, m, k, n, p)
    dA = torch.from_numpy(A.astype(np.float64)).to("cuda:0")
    dB = torch.from_numpy(B.astype(np.float64)).to("cuda:0")
    dC = torch.empty((m, n), dtype=torch.float64, device="cuda:0")
    per = LIMIT // h
    edge = [0, per - 1, per, h - 1]
    rng = np.random.default_rng(7)
    rows = np.concatenate([rng.integers(0, m, 4096),
                           np.repeat([r + q for r in edge for q in (0, h)], 4)])
    cols = np.concatenate([rng.integers(0, n, 4096),
                           np.tile([0, h - 1, h, n - 1], 2 * len(edge))])
    want = ref.matmul_entries(A, B, None, 1, 0, p, rows, cols)
    ri, ci = torch.from_numpy(rows).to("cuda:0"), torch.from_numpy(cols).to("cuda:0")
    # Whole rows on both sides of every slice boundary, in both row halves.
    full_rows = np.array(sorted({r + q for r in edge + [per - 2, per + 1] for q in (0, h)
                                 if 0 <= r + q < m}), dtype=np.int64)
    want_rows = ref.matmul_mod_p(A[full_rows], B, None, 1, 0, p)
    fr = torch.from_numpy(full_rows).to("cuda:0")
    try:
        for flags in (capi.WS_FLAG_NOFUSE, 0):
            print("m = n =", m, "flags", flags, flush=True)
            dC.fill_(-1.0)
            args = capi.make_args(m, k, n, p, dA, dB, dC, 1, 0, capi.WS_TWO_TEMP, 1,
                                  stream=torch.cuda.current_stream(), flags=flags)
            st = capi.wsmul_mod_p_ex(args)
            torch.cuda.synchronize()
            assert st == capi.WS_OK, capi.wsmul_last_error()
            got = dC[ri, ci].cpu().numpy().astype(np.int64)
            assert np.array_equal(got, want), flags
            got_rows = dC[fr].cpu().numpy().astype(np.int64)
            assert np.array_equal(got_rows, want_rows), flags
    finally:
        del dC, dA, dB
        torch.cuda.empty_cache()
