"""Tile choice of the binary64 base products: every kernel kind, pinned on
the same products, gives the oracle's result bit for bit (plain and folded
sums, centred and uncentred operands, ragged shapes, both storage types, and
inside a schedule); measured tuning keeps the fastest admissible kind."""
import numpy as np
import pytest

from oracle import ref
from paper_0707_2347_amd import capi, inputs

from .gpu_util import call

pytestmark = pytest.mark.gpu


def _admissible(kind, m, k, n):
    """Kinds that can take a dense m x k by k x n product (torch buffers are
    16-byte aligned; lda = k, ldb = n)."""
    even = k % 2 == 0 and n % 2 == 0
    if kind == capi.WS_TILE_BIG128:
        return m % 128 == 0 and n % 128 == 0 and k % 16 == 0 and k > 0 and even
    if kind == capi.WS_TILE_DMA64:
        return m % 64 == 0 and n % 64 == 0 and k % 8 == 0 and k > 0 and even
    if kind == capi.WS_TILE_DMA32:
        return m % 32 == 0 and n % 32 == 0 and k % 16 == 0 and k > 0 and even
    if kind == capi.WS_TILE_DMA16:
        return m % 16 == 0 and n % 16 == 0 and k % 16 == 0 and k > 0 and even
    return True


@pytest.mark.parametrize("shape,p,dtype", [((512, 512, 512), 65521, capi.WS_F64),
                                           ((384, 640, 256), 8388593, capi.WS_F64),
                                           ((256, 1024, 256), 16777213, capi.WS_I64),
                                           ((200, 300, 100), 16777213, capi.WS_F64),
                                           ((128, 4096, 64), 8388593, capi.WS_F64),
                                           # inner dimensions that are not whole 64-deep
                                           # chunks: the split kernels deal uneven
                                           # numbers of sub-chunks to their waves
                                           ((256, 48, 256), 65521, capi.WS_F64),
                                           ((192, 336, 128), 8388593, capi.WS_F64),
                                           ((128, 24, 64), 1048573, capi.WS_I64),
                                           ((64, 16, 32), 16777213, capi.WS_F64),
                                           ((320, 1040, 96), 8388593, capi.WS_F64)])
def test_every_kind_is_exact(shape, p, dtype):
    m, k, n = shape
    A, B, C = inputs.uniform(71, m, k, n, p, with_c=True)
    want = ref.matmul_mod_p(A, B, C, 6, 5, p)
    kinds = [t for t in range(capi.WS_TILE_KINDS) if _admissible(t, m, k, n)]
    assert capi.WS_TILE_SK32 in kinds
    try:
        for kind in kinds:
            print("tile kind", kind, shape, p, dtype, flush=True)
            assert capi.wsmul_set_tile(m, k, n, p, dtype, kind) == capi.WS_OK
            st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, C, 6, 5, p, 0, dtype=dtype)
            assert st == capi.WS_OK, capi.wsmul_last_error()
            assert np.array_equal(C2, want), kind
    finally:
        capi.wsmul_set_tile(m, k, n, p, dtype, -1)


def test_every_leaf_kind_inside_table9():
    """Table 9 at 512^3 with two levels: its 128^3 leaves on each kind."""
    p, n = 1048573, 512
    A, B, C = inputs.uniform(72, n, n, n, p, with_c=True)
    want = ref.matmul_mod_p(A, B, C, 3, 7, p)
    try:
        for kind in range(capi.WS_TILE_KINDS):
            capi.wsmul_set_tile(128, 128, 128, p, capi.WS_F64, kind)
            st, C2, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 3, 7, p, 2)
            assert st == capi.WS_OK, capi.wsmul_last_error()
            assert np.array_equal(C2, want), kind
    finally:
        capi.wsmul_set_tile(128, 128, 128, p, capi.WS_F64, -1)


def test_tuning_keeps_the_fastest_admissible_kind():
    m = k = n = 512
    p = 65521
    try:
        st, best, times = capi.wsmul_tune_tiles(m, k, n, p, capi.WS_F64, 5)
        assert st == capi.WS_OK, capi.wsmul_last_error()
        timed = [t for t in range(capi.WS_TILE_KINDS) if times[t] >= 0]
        assert timed == [t for t in range(capi.WS_TILE_KINDS) if _admissible(t, m, k, n)]
        assert best in timed and times[best] == min(times[t] for t in timed)
        A, B, C = inputs.uniform(73, m, k, n, p, with_c=True)
        st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, C, 1, 1, p, 0)
        assert st == capi.WS_OK and np.array_equal(C2, ref.matmul_mod_p(A, B, C, 1, 1, p))
    finally:
        capi.wsmul_set_tile(m, k, n, p, capi.WS_F64, -1)


def test_tuning_a_plan():
    p, n = 65521, 256
    A, B, C = inputs.uniform(74, n, n, n, p, with_c=True)
    args = capi.make_args(n, n, n, p, beta=1, schedule=capi.WS_TWO_TEMP, levels=2)
    shapes = {(o.a.rows, o.a.cols, o.b.cols) for o in capi.wsmul_plan_export(args)
              if o.kind == capi.WS_OP_GEMM}
    try:
        args.A = args.B = args.C = 16          # pointers are not used by tuning
        assert capi.wsmul_tune_plan(args, 3) == capi.WS_OK, capi.wsmul_last_error()
        st, C2, _, _ = call(capi.WS_TWO_TEMP, A, B, C, 1, 1, p, 2)
        assert st == capi.WS_OK and np.array_equal(C2, ref.matmul_mod_p(A, B, C, 1, 1, p))
    finally:
        for m, k, nn in shapes:
            capi.wsmul_set_tile(m, k, nn, p, capi.WS_F64, -1)


def test_tile_argument_errors():
    assert capi.wsmul_tune_tiles(0, 5, 5, 65521)[0] == capi.WS_EINVAL
    assert capi.wsmul_tune_tiles(5, 5, 5, 1)[0] == capi.WS_EMODULUS
    assert capi.wsmul_set_tile(5, 5, 5, 65521, capi.WS_F64, capi.WS_TILE_KINDS) == capi.WS_EINVAL


@pytest.mark.parametrize("shape,p", [((1536, 64, 1536), 65521),        # 32 x 32 direct by rounds
                                     ((2304, 64, 2304), 8388593),      # 64 x 64 direct by rounds
                                     ((3072, 48, 3072), 65521),        # 64 x 64 direct by rounds
                                     ((3000, 40, 3000), 1048573),      # 64 x 64 register-staged
                                     ((4000, 32, 4000), 65521),        # 128 x 128 register-staged
                                     ((768, 96, 768), 16777213)])      # 32 x 32 direct
def test_default_rule_shapes_are_exact(shape, p):
    """Products that the round-count rules send to each kind, on the default
    choice, against the oracle."""
    m, k, n = shape
    A, B, C = inputs.uniform(75, m, k, n, p, with_c=True)
    print("default rule", shape, p, flush=True)
    st, C2, _, _ = call(capi.WS_CLASSICAL, A, B, C, 2, 3, p, 0)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert np.array_equal(C2, ref.matmul_mod_p(A, B, C, 2, 3, p))
