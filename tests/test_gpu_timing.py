"""Kernel timing through the ABI: HIP events around each launch, on the
stream it runs on; the per-launch list agrees with the summed figure."""

import numpy as np
import pytest

from tests.gpu_util import device_of, parent_host, stream_handle, to_mh, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_1705_04807_amd as m
    return m


def test_kernel_times(mh):
    torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        p, T, N = 65521, 64, 512
        A, B, C = (parent_host(s, p, N) for s in (91, 92, 93))
        Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X in (A, B, C))
        mh.check(mh.mh_ctx_set_timing(ctx, 1))
        for _ in range(3):
            mh.check(mh.mh_matmul_modp(ctx, Cd.data_ptr(), N, 0, 0, Ad.data_ptr(), N, 0, 0,
                                       Bd.data_ptr(), N, 0, 0, N, N, N, p, T,
                                       mh.MH_MODE_LIMB_I8, stream_handle()))
        each = mh.mh_ctx_kernel_times(ctx, mh.MH_K_GEMM_LIMB)
        total, n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_GEMM_LIMB)
        assert n == 3 and len(each) == 3 and all(t > 0 for t in each)
        assert sum(each) == pytest.approx(total, rel=1e-6)
        assert mh.mh_ctx_kernel_times(ctx, mh.MH_K_GEMM_LIMB, cap=1) == each[:1]
        assert len(mh.mh_ctx_kernel_times(ctx, mh.MH_K_PACK)) == 3  # one record per call
        mh.mh_ctx_kernel_time(ctx, mh.MH_K_GEMM_LIMB, reset=True)
        assert mh.mh_ctx_kernel_times(ctx, mh.MH_K_GEMM_LIMB) == []
        assert mh.lib.mh_ctx_kernel_times(ctx, mh.MH_K_COUNT, None, 0, None) == mh.MH_E_INVALID
        assert mh.lib.mh_ctx_kernel_times(ctx, 0, None, -1, None) == mh.MH_E_INVALID
    finally:
        mh.mh_ctx_destroy(ctx)
