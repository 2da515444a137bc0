"""The sustained-rate probes: argument checks, and rates that are positive
and no higher than the published peaks (5.0 POP/s dense int8 on MI355X; the
plain form's multiply-accumulate pair at most 256 CUs x 4 SIMDs x 16 lanes x
2.4 GHz / 2 = 19.66 T/s), with a margin for clock measurement."""

import ctypes as ct

import pytest

from tests.gpu_util import say, stream_handle, torch_cuda

pytestmark = pytest.mark.gpu


def test_probe_mfma_i8():
    import paper_1705_04807_amd as mh
    torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        out = ct.c_double()
        for bad in (0, 1, 3, (1 << 24) + 2):
            assert mh.lib.mh_probe_mfma_i8(ctx, bad, ct.byref(out), stream_handle()) == \
                mh.MH_E_INVALID
        assert mh.lib.mh_probe_mfma_i8(ctx, 1000, None, stream_handle()) == mh.MH_E_INVALID
        say("probe mfma")
        pops = mh.mh_probe_mfma_i8(ctx, 20000, stream_handle())
        say("sustained int8 MFMA %.3f POP/s" % (pops / 1e15))
        assert 0.5e15 < pops < 5.2e15
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)


def test_probe_valu_mac():
    import paper_1705_04807_amd as mh
    torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        out = ct.c_double()
        for bad in (0, -1, (1 << 24) + 1):
            assert mh.lib.mh_probe_valu_mac(ctx, bad, ct.byref(out), stream_handle()) == \
                mh.MH_E_INVALID
        assert mh.lib.mh_probe_valu_mac(ctx, 100, None, stream_handle()) == mh.MH_E_INVALID
        say("probe valu mac")
        macs = mh.mh_probe_valu_mac(ctx, 2048, stream_handle())
        say("sustained 96-bit multiply-accumulate %.2f T/s" % (macs / 1e12))
        assert 1e12 < macs < 20.5e12
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)
