"""Every limb GEMM configuration against the oracle, for every limb count.

The tuner may pick any configuration that fits, so each one is checked on a
ragged product whose k spans several pipeline stages and ends inside one,
once with the reduction interval the bound allows and once with 128-deep
k-blocks (MH_LIMB_KBLOCK), so that the epilogue also runs between k-blocks
with stages still in flight.  Bar: bit-exact.
"""

import numpy as np
import pytest

from tests.gpu_util import (device_of, expected_view, host_of, parent_host, say,
                            stream_handle, to_cart, to_mh, torch_cuda)

pytestmark = pytest.mark.gpu

PRIMES = {1: 251, 2: 65521, 3: (1 << 24) - 3, 4: 2**31 - 1}
N, T = 1024, 64
NCFG = 16  # entries of the configuration table
OFF = dict(rc=17, cc=40, ra=3, ca=100, rb=60, cb=7, m=300, k=700, n=333)


@pytest.fixture(scope="module")
def mh():
    import paper_1705_04807_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mh):
    torch_cuda()
    c = mh.mh_ctx_create(0)
    yield c
    mh.mh_ctx_destroy(c)


@pytest.fixture(scope="module")
def operands(mh, ctx):
    out = {}
    for L, p in PRIMES.items():
        A, B, C = (parent_host(7000 + 10 * L + s, p, N) for s in range(3))
        Ad, Bd = to_mh(mh, ctx, device_of(A), N, T), to_mh(mh, ctx, device_of(B), N, T)
        want = expected_view(C, A, B, p, OFF["rc"], OFF["cc"], OFF["ra"], OFF["ca"], OFF["rb"],
                             OFF["cb"], OFF["m"], OFF["k"], OFF["n"])
        out[L] = (C, Ad, Bd, want)
    return out


@pytest.mark.parametrize("kblock", [None, 128])
@pytest.mark.parametrize("cfg", range(NCFG))
@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_configuration(mh, ctx, operands, monkeypatch, L, cfg, kblock):
    p = PRIMES[L]
    monkeypatch.setenv("MH_LIMB_CFG", str(cfg))
    if kblock:
        monkeypatch.setenv("MH_LIMB_KBLOCK", str(kblock))
    else:
        monkeypatch.delenv("MH_LIMB_KBLOCK", raising=False)
    s, info = mh.mh_plan_describe(N, OFF["rc"], OFF["cc"], N, OFF["ra"], OFF["ca"], N,
                                  OFF["rb"], OFF["cb"], OFF["m"], OFF["k"], OFF["n"], p, T,
                                  mh.MH_MODE_LIMB_I8)
    mh.check(s)
    if info.kernel_cfg != cfg:
        pytest.skip("configuration %d does not fit %d limbs" % (cfg, L))
    assert info.kblock == (kblock or info.kblock)
    C, Ad, Bd, want = operands[L]
    Cd = to_mh(mh, ctx, device_of(C), N, T)
    say("limb cfg", cfg, "L", L, "kblock", kblock)
    mh.check(mh.mh_matmul_modp(ctx, Cd.data_ptr(), N, OFF["rc"], OFF["cc"], Ad.data_ptr(), N,
                               OFF["ra"], OFF["ca"], Bd.data_ptr(), N, OFF["rb"], OFF["cb"],
                               OFF["m"], OFF["k"], OFF["n"], p, T, mh.MH_MODE_LIMB_I8,
                               stream_handle()))
    got = host_of(to_cart(mh, ctx, Cd, N, T))
    assert np.array_equal(got, want)
    assert mh.mh_ctx_last_device_error(ctx) == 0
