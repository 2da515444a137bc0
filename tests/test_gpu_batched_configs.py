"""Every limb GEMM configuration in the batched persistent kernel.

The batch is large enough (several hundred to a few thousand output blocks)
that every persistent workgroup pops several tasks, so each configuration's
LDS stage buffers are reused across output blocks of different products;
half the runs also force 128-deep k-blocks, so epilogues run between
k-blocks with stages in flight.  One batch per limb count, checked against
the oracle on every C parent.  Bar: bit-exact.
"""

import numpy as np
import pytest

from tests.gpu_util import (device_of, expected_view, host_of, parent_host, say,
                            stream_handle, to_cart, to_mh, torch_cuda)
from tests.test_gpu_limb_configs import NCFG

pytestmark = pytest.mark.gpu

PRIMES = {2: 65521, 4: 2**31 - 1}
N, T, NPAR, COUNT = 2048, 64, 4, 32


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


def draw(g):
    """COUNT products with wide outputs (400..700 square-ish) and short k,
    output blocks disjoint within each of NPAR C parents."""
    calls, used = [], [[] for _ in range(NPAR)]
    while len(calls) < COUNT:
        m, n = int(g.integers(400, 701)), int(g.integers(400, 701))
        k = int(g.integers(33, 200))
        ci = len(calls) % NPAR
        rc, cc = int(g.integers(0, N - m + 1)), int(g.integers(0, N - n + 1))
        if any(not (rc + m <= r or r + mm <= rc or cc + n <= c or c + nn <= cc)
               for r, c, mm, nn in used[ci]):
            continue
        used[ci].append((rc, cc, m, n))
        calls.append(dict(ci=ci, rc=rc, cc=cc, m=m, k=k, n=n,
                          ra=int(g.integers(0, N - m + 1)), ca=int(g.integers(0, N - k + 1)),
                          rb=int(g.integers(0, N - k + 1)), cb=int(g.integers(0, N - n + 1))))
    return calls


@pytest.fixture(scope="module")
def batches(mh, ctx):
    out = {}
    for L, p in PRIMES.items():
        g = np.random.default_rng(6100 + L)
        A, B = parent_host(6200 + L, p, N), parent_host(6300 + L, p, N)
        Cs = [parent_host(6400 + 10 * L + i, p, N) for i in range(NPAR)]
        calls = draw(g)
        want = [C.copy() for C in Cs]
        for c in calls:
            want[c["ci"]] = expected_view(want[c["ci"]], A, B, p, c["rc"], c["cc"], c["ra"],
                                          c["ca"], c["rb"], c["cb"], c["m"], c["k"], c["n"])
        Ad, Bd = to_mh(mh, ctx, device_of(A), N, T), to_mh(mh, ctx, device_of(B), N, T)
        out[L] = (calls, Cs, want, Ad, Bd)
    return out


@pytest.mark.parametrize("kblock", [None, 128])
@pytest.mark.parametrize("cfg", range(NCFG))
@pytest.mark.parametrize("L", sorted(PRIMES))
def test_batched_configuration(mh, ctx, batches, monkeypatch, L, cfg, kblock):
    p = PRIMES[L]
    monkeypatch.setenv("MH_LIMB_CFG", str(cfg))
    if kblock:
        monkeypatch.setenv("MH_LIMB_KBLOCK", str(kblock))
    else:
        monkeypatch.delenv("MH_LIMB_KBLOCK", raising=False)
    s, info = mh.mh_plan_describe(N, 0, 0, N, 0, 0, N, 0, 0, 512, 512, 512, p, T,
                                  mh.MH_MODE_LIMB_I8)
    mh.check(s)
    if info.kernel_cfg != cfg:
        pytest.skip("configuration %d does not fit %d limbs" % (cfg, L))
    calls, Cs, want, Ad, Bd = batches[L]
    Cds = [to_mh(mh, ctx, device_of(C), N, T) for C in Cs]
    descs = mh.make_descs([dict(C=Cds[c["ci"]].data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(),
                                NC=N, NA=N, NB=N, rc=c["rc"], cc=c["cc"], ra=c["ra"],
                                ca=c["ca"], rb=c["rb"], cb=c["cb"], m=c["m"], k=c["k"],
                                n=c["n"]) for c in calls])
    say("batched cfg", cfg, "L", L, "kblock", kblock)
    mh.check(mh.mh_matmul_modp_batched(ctx, descs, len(calls), p, T, mh.MH_MODE_LIMB_I8,
                                       stream_handle()), "batched")
    for ci, Cd in enumerate(Cds):
        assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), want[ci]), ci
    assert mh.mh_ctx_last_device_error(ctx) == 0


@pytest.mark.parametrize("kblock", [None, 128])
@pytest.mark.parametrize("cfg", [11, 12, 13])
def test_batched_configuration_a_parent(mh, ctx, batches, monkeypatch, cfg, kblock):
    """The configurations with the form that reads A from a panel of the
    whole parent (forced with MH_BATCH_APARENT=1), at two limbs."""
    L, p = 2, PRIMES[2]
    monkeypatch.setenv("MH_LIMB_CFG", str(cfg))
    monkeypatch.setenv("MH_BATCH_APARENT", "1")
    if kblock:
        monkeypatch.setenv("MH_LIMB_KBLOCK", str(kblock))
    else:
        monkeypatch.delenv("MH_LIMB_KBLOCK", raising=False)
    calls, Cs, want, Ad, Bd = batches[L]
    Cds = [to_mh(mh, ctx, device_of(C), N, T) for C in Cs]
    descs = mh.make_descs([dict(C=Cds[c["ci"]].data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(),
                                NC=N, NA=N, NB=N, rc=c["rc"], cc=c["cc"], ra=c["ra"],
                                ca=c["ca"], rb=c["rb"], cb=c["cb"], m=c["m"], k=c["k"],
                                n=c["n"]) for c in calls])
    say("batched a-parent cfg", cfg, "kblock", kblock)
    mh.check(mh.mh_matmul_modp_batched(ctx, descs, len(calls), p, T, mh.MH_MODE_LIMB_I8,
                                       stream_handle()), "batched")
    s, last_cfg, _, forms = mh.mh_ctx_last_batch_config(ctx)
    assert last_cfg == cfg and forms & mh.MH_BATCH_FORM_A_PARENT
    for ci, Cd in enumerate(Cds):
        assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), want[ci]), ci
    assert mh.mh_ctx_last_device_error(ctx) == 0
