"""The int32 accumulator bound of the limb form, driven to its limit on the GPU.

With every residue equal to H_L = 127 (256^L - 1) / 255, the largest value L
balanced base-256 digits hold, all digits are 127, and the shift with L digit
pairs grows by L * 127^2 per depth: over a full k-block (the longest the
bound allows) it reaches 98.3 % of 2^31 at L = 3 and 4, so a k-block 2 %
longer would overflow.  The product crosses a k-block boundary (k = kblock +
64), so the reduction between k-blocks runs with the accumulators at that
peak.  Constant operands make the
expected value closed-form, (c + k a b) mod p, at any size, so the parents
(constant, hence the same in any layout) are filled on the device.  Bar:
bit-exact on the 128 x 128 output block, every other word unchanged.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import say, stream_handle, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_1705_04807_amd as m
    return m


@pytest.mark.parametrize("mode", ["limb", "limb_lds", "plain"])
@pytest.mark.parametrize("L,p,N", [(4, 2**31 - 1, 32768), (3, (1 << 24) - 3, 65536)])
def test_full_kblock_all_digits_127(mh, monkeypatch, mode, L, p, N):
    torch = torch_cuda()
    if mode == "limb_lds":  # the LDS-staged configuration instead of the small-output one
        monkeypatch.setenv("MH_LIMB_CFG", "11")
    T, m, n = 64, 128, 128
    H = 127 * (256**L - 1) // 255
    digits, ok = oracle.limb_digits(H, p, L)
    assert ok and digits == [127] * L
    s, info = mh.mh_plan_describe(N, 0, 0, N, 0, 0, N, 0, 0, m, N, n, p, T, mh.MH_MODE_LIMB_I8)
    mh.check(s)
    assert info.limbs == L
    k = (info.kblock // 64 + 1) * 64  # one full k-block and one more 64-deep step
    assert k <= N
    peak = L * 127 * 127 * info.kblock  # the L-pair shift after the first k-block
    assert 0.98 * 2**31 < peak < 2**31
    c = p - 1
    ctx = mh.mh_ctx_create(0)
    try:
        A = torch.full((N * N,), H, dtype=torch.int32, device="cuda")
        C = torch.full((N * N,), c, dtype=torch.int32, device="cuda")
        form = mh.MH_MODE_PLAIN_U32 if mode == "plain" else mh.MH_MODE_LIMB_I8
        say("kblock bound", L, p, N, "k", k, "kblock", info.kblock, mode)
        # B = A (the same constant parent, read only)
        mh.check(mh.mh_matmul_modp(ctx, C.data_ptr(), N, 0, 0, A.data_ptr(), N, 0, 0,
                                   A.data_ptr(), N, 0, 0, m, k, n, p, T, form,
                                   stream_handle()))
        want = (c + k * H * H) % p
        # the 128 x 128 block at (0, 0) is tiles 0..3 in Z order: words 0 .. m n - 1
        head = C[:m * n].cpu().numpy().view(np.uint32)
        assert np.all(head == want), (int(head.min()), int(head.max()), want)
        assert int((C[m * n:] != c).sum().item()) == 0
        assert int((A != H).sum().item()) == 0
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)
        del A, C
        torch.cuda.empty_cache()
