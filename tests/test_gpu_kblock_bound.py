"""The int32 accumulator bound of the limb form, driven to its limit on the GPU.

The bound (|d_t d_u| <= 2^14, at most L digit pairs per shift, so
|T_s| <= kblock L 2^14 < 2^31) is reached as closely as centred residues
allow:

* every residue H_L = 127 (256^L - 1) / 255, the largest value L balanced
  base-256 digits hold: all digits 127, and the shift with L digit pairs
  grows by L 127^2 per depth, 98.3 % of 2^31 over a full k-block at L = 3
  and 4;
* residues whose digits mix -128 and 127 so that the products of a shift
  are all -128 * 127 or (-128)^2: for p = 65521, x = 32880 is centred to
  -32641 = 127 - 128 * 256, digits (127, -128), and |T_1| = 2 * 127 * 128
  per depth, 99.1 % of 2^31 over a k-block; for p = 2^31 - 1,
  x = 2138996608 is centred to -8487039 with digits (-128, -128, 127, 127),
  and |T_3| = 4 * 127 * 128 per depth, 99.0 % of 2^31.

The product crosses a k-block boundary (k = kblock + 64), so the reduction
between k-blocks runs with the accumulators at that peak.  Constant operands
make the expected value closed-form, (c + k x^2) mod p, at any size, so the
parents (constant, hence the same in any layout) are filled on the device.
Bar: bit-exact on the 128 x 128 output block, every other word unchanged.
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


def _shift_peak(digits):
    """Largest |sum_{t+u=s} d_t d_u| over the shifts s of a constant operand."""
    L = len(digits)
    return max(abs(sum(digits[t] * digits[s - t] for t in range(L) if 0 <= s - t < L))
               for s in range(2 * L - 1))


@pytest.mark.parametrize("mode", ["limb", "limb_lds", "plain"])
@pytest.mark.parametrize("L,p,N,x,digits,frac", [
    (4, 2**31 - 1, 32768, None, [127] * 4, 0.982),
    (3, (1 << 24) - 3, 65536, None, [127] * 3, 0.983),
    (2, 65521, 65536, 32880, [127, -128], 0.991),
    (4, 2**31 - 1, 32768, 2138996608, [-128, -128, 127, 127], 0.990),
])
def test_full_kblock_extreme_digits(mh, monkeypatch, mode, L, p, N, x, digits, frac):
    torch = torch_cuda()
    if mode == "limb_lds":  # the LDS-staged configuration instead of the small-output one
        monkeypatch.setenv("MH_LIMB_CFG", "11")
    T, m, n = 64, 128, 128
    H = 127 * (256**L - 1) // 255 if x is None else x
    got_digits, ok = oracle.limb_digits(H, p, L)
    assert ok and got_digits == digits
    s, info = mh.mh_plan_describe(N, 0, 0, N, 0, 0, N, 0, 0, m, N, n, p, T, mh.MH_MODE_LIMB_I8)
    mh.check(s)
    assert info.limbs == L
    k = (info.kblock // 64 + 1) * 64  # one full k-block and one more 64-deep step
    assert k <= N
    peak = _shift_peak(digits) * info.kblock  # the largest shift after the first k-block
    assert frac * 2**31 < peak < 2**31
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
