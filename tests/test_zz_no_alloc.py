"""mh_matmul_modp_noalloc against mh_matmul_modp, through the C ABI.

The entry point that allocates nothing keeps its operand panels in the
library's fixed 128 MiB device array.  Two calls in a row on one context,
the second with a smaller input:

1. a product whose panels (about 400 MiB of limbs) exceed the array, so it
   runs as chunked sub-products inside it: 6000 x 8000 x 7000 at p = 2^31 - 1
   on non-aligned blocks of 8192^2 parents;
2. a small non-aligned product at p = 65521 in 4096^2 parents, in the limb,
   plain and FP64 forms, additive and subtractive.

Each result must equal, on every word of the C parent, the result of
mh_matmul_modp on the same inputs (and, for the small product, the
oracle's).  The context's own workspace must stay unallocated, and timing
(on) must record no launches for these calls.
"""

import numpy as np
import pytest

import oracle
from seeded_inputs import residues_torch
from tests.gpu_util import (device_of, host_of, parent_host, say, stream_handle, to_cart,
                            to_mh, torch_cuda)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_1705_04807_amd as m
    return m


def _both(mh, ctx, C, A, B, N, off, m, k, n, p, T, mode):
    """C parent after the no-allocation call and after mh_matmul_modp, from the same C."""
    rc, cc, ra, ca, rb, cb = off
    C2 = C.clone()
    mh.check(mh.mh_matmul_modp_noalloc(ctx, C.data_ptr(), N, rc, cc, A.data_ptr(), N, ra, ca,
                                       B.data_ptr(), N, rb, cb, m, k, n, p, T, mode,
                                       stream_handle()), "noalloc")
    mh.check(mh.mh_matmul_modp(ctx, C2.data_ptr(), N, rc, cc, A.data_ptr(), N, ra, ca,
                               B.data_ptr(), N, rb, cb, m, k, n, p, T, mode, stream_handle()),
             "matmul")
    return C, C2


def test_noalloc_matches_matmul_two_calls(mh):
    torch = torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        mh.check(mh.mh_ctx_set_timing(ctx, True))
        # ---- call 1: panels larger than the scratch array (chunked)
        N, T, p = 8192, 64, 2**31 - 1
        off, m, k, n = (64, 33, 1000, 150, 117, 1048), 6000, 8000, 7000
        say("noalloc 1:", N, off, m, k, n, p)
        parents = []
        for s in (8001, 8002, 8003):
            X = residues_torch(s, p, N, N, device="cuda")
            parents.append(to_mh(mh, ctx, X, N, T))
            del X
        A, B, C = parents
        A0, B0 = A.clone(), B.clone()
        Cn = C.clone()
        rc, cc, ra, ca, rb, cb = off
        mh.check(mh.mh_matmul_modp_noalloc(ctx, Cn.data_ptr(), N, rc, cc, A.data_ptr(), N, ra,
                                           ca, B.data_ptr(), N, rb, cb, m, k, n, p, T,
                                           mh.MH_MODE_LIMB_I8, stream_handle()), "noalloc 1")
        torch.cuda.synchronize()
        s, limit, held = mh.mh_ctx_workspace_info(ctx)
        mh.check(s)
        assert held == 0, "the no-allocation call left a context workspace of %d bytes" % held
        _, launches = mh.mh_ctx_kernel_time(ctx, mh.MH_K_GEMM_LIMB, reset=True)
        assert launches == 0
        mh.check(mh.mh_matmul_modp(ctx, C.data_ptr(), N, rc, cc, A.data_ptr(), N, ra, ca,
                                   B.data_ptr(), N, rb, cb, m, k, n, p, T, mh.MH_MODE_LIMB_I8,
                                   stream_handle()), "matmul 1")
        torch.cuda.synchronize()
        bad = int((Cn != C).sum().item())
        say("noalloc 1: %d words differ" % bad)
        assert bad == 0
        assert torch.equal(A, A0) and torch.equal(B, B0)
        del parents, A, B, C, Cn, A0, B0
        torch.cuda.empty_cache()

        # ---- call 2: a smaller product, every form, both signs
        N, T, p = 4096, 64, 65521
        off, m, k, n = (100, 7, 33, 2000, 517, 64), 1000, 1500, 900
        rc, cc, ra, ca, rb, cb = off
        Ah, Bh, Ch = (parent_host(s, p, N) for s in (8011, 8012, 8013))
        A, B = to_mh(mh, ctx, device_of(Ah), N, T), to_mh(mh, ctx, device_of(Bh), N, T)
        for mode in (mh.MH_MODE_LIMB_I8, mh.MH_MODE_PLAIN_U32, mh.MH_MODE_FP64,
                     mh.MH_MODE_LIMB_I8 | mh.MH_SUBTRACT):
            say("noalloc 2: mode", mode)
            C = to_mh(mh, ctx, device_of(Ch), N, T)
            Cn, Cm = _both(mh, ctx, C, A, B, N, off, m, k, n, p, T, mode)
            got = host_of(to_cart(mh, ctx, Cn, N, T))
            assert np.array_equal(got, host_of(to_cart(mh, ctx, Cm, N, T))), mode
            want = Ch.copy()
            oracle.matmul_modp_view(want, Ah, Bh, p, rc, cc, ra, ca, rb, cb, m, k, n,
                                    subtract=bool(mode & mh.MH_SUBTRACT))
            assert np.array_equal(got, want), mode
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)
        torch.cuda.empty_cache()


def test_noalloc_rejects_what_matmul_rejects(mh):
    """Argument errors are the same as mh_matmul_modp's, before any device work."""
    torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        args = (ctx, 256, 256, 0, 0, 256, 256, 0, 0, 256, 256, 0, 0, 64, 64, 64)
        assert mh.mh_matmul_modp_noalloc(*args, 2**31 + 1, 64, 2, 0) == 4  # MH_E_MODULUS
        assert mh.mh_matmul_modp_noalloc(*args, 65521, 48, 2, 0) == 6      # MH_E_UNSUPPORTED
        bad = (ctx, 256, 100, 0, 0, 256, 100, 0, 0, 256, 100, 0, 0, 64, 64, 64)
        assert mh.mh_matmul_modp_noalloc(*bad, 65521, 64, 2, 0) == 2       # MH_E_SHAPE
    finally:
        mh.mh_ctx_destroy(ctx)
