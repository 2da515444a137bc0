"""The autotuner: tuning runs never touch the caller's output, choices are
cached and persisted, and tuned products stay bit-exact."""

import os

import numpy as np
import pytest

from tests.gpu_util import (device_of, expected_view, host_of, parent_host, say,
                            stream_handle, to_cart, to_mh, torch_cuda)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_1705_04807_amd as m
    return m


def _product(mh, ctx, p, T, N, P, seeds):
    A, B, C = (parent_host(s, p, N) for s in seeds)
    Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X in (A, B, C))
    mh.check(mh.mh_matmul_modp(ctx, Cd.data_ptr(), N, P[0], P[1], Ad.data_ptr(), N, P[2], P[3],
                               Bd.data_ptr(), N, P[4], P[5], P[6], P[7], P[8], p, T,
                               mh.MH_MODE_LIMB_I8, stream_handle()))
    got = host_of(to_cart(mh, ctx, Cd, N, T))
    want = expected_view(C, A, B, p, *P)
    return got, want


def test_tune_single_then_cache(mh, tmp_path):
    torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        p, T, N = 65521, 64, 1024
        P = (64, 33, 100, 150, 51, 204, 700, 650, 720)
        assert mh.mh_ctx_tune_lookup(ctx, p, T, 700, 650, 720) == -1
        mh.check(mh.mh_ctx_set_autotune(ctx, 2))
        say("tune single")
        got, want = _product(mh, ctx, p, T, N, P, (61, 62, 63))
        assert np.array_equal(got, want)  # tuning wrote only its scratch output
        cfg = mh.mh_ctx_tune_lookup(ctx, p, T, 700, 650, 720)
        assert cfg >= 0
        got, want = _product(mh, ctx, p, T, N, P, (64, 65, 66))  # cached choice
        assert np.array_equal(got, want)
        path = str(tmp_path / "tune.json")
        mh.check(mh.mh_ctx_tune_cache_save(ctx, path))
        assert '"mh-tune-1"' in open(path).read()
    finally:
        mh.mh_ctx_destroy(ctx)
    ctx2 = mh.mh_ctx_create(0)
    try:
        s, n = mh.mh_ctx_tune_cache_load(ctx2, path)
        assert s == 0 and n >= 1
        assert mh.mh_ctx_tune_lookup(ctx2, p, T, 700, 650, 720) == cfg
        assert mh.mh_ctx_tune_cache_load(ctx2, str(tmp_path / "missing.json"))[0] == \
            mh.MH_E_INVALID
        assert mh.mh_ctx_set_autotune(ctx2, 3) == mh.MH_E_INVALID
    finally:
        mh.mh_ctx_destroy(ctx2)


def test_tune_batched(mh):
    torch_cuda()
    ctx = mh.mh_ctx_create(0)
    try:
        mh.check(mh.mh_ctx_set_autotune(ctx, 2))
        p, T, N = 2**31 - 1, 32, 1024
        A, B, C = (parent_host(s, p, N) for s in (71, 72, 73))
        Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X in (A, B, C))
        calls = [dict(rc=0, cc=0, ra=5, ca=7, rb=9, cb=11, m=300, k=257, n=190),
                 dict(rc=400, cc=500, ra=50, ca=70, rb=90, cb=110, m=200, k=333, n=350),
                 dict(rc=700, cc=0, ra=500, ca=700, rb=300, cb=10, m=250, k=90, n=400)]
        descs = mh.make_descs([dict(c, C=Cd.data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(),
                                    NC=N, NA=N, NB=N) for c in calls])
        say("tune batched")
        for rep in range(2):
            mh.check(mh.mh_matmul_modp_batched(ctx, descs, 3, p, T, mh.MH_MODE_LIMB_I8,
                                               stream_handle()))
            for c in calls:
                C = expected_view(C, A, B, p, c["rc"], c["cc"], c["ra"], c["ca"], c["rb"],
                                  c["cb"], c["m"], c["k"], c["n"])
            assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), C), rep
    finally:
        mh.mh_ctx_destroy(ctx)


def test_cached_configuration_that_does_not_fit_is_ignored(mh, tmp_path):
    # A cache entry naming configuration 3 (128 x 128 blocks, built for at
    # most two limbs) for a four-limb bucket: the product falls back to the
    # built-in choice and stays exact.
    torch_cuda()
    p, T, N = 2**31 - 1, 64, 1024
    P = (3, 70, 10, 20, 30, 40, 500, 600, 450)
    ctx = mh.mh_ctx_create(0)
    try:
        tag_path = str(tmp_path / "probe.json")
        mh.check(mh.mh_ctx_tune_cache_save(ctx, tag_path))
        device_line = [l for l in open(tag_path) if '"device"' in l][0]
        key = "single L=4 T=64 m=9 k=10 n=9"
        path = str(tmp_path / "bad.json")
        with open(path, "w") as f:
            f.write(device_line)
            f.write(' "entries": [\n  {"key": "%s", "cfg": 3, "ms": 1.0}\n ]}\n' % key)
        s, n = mh.mh_ctx_tune_cache_load(ctx, path)
        assert s == mh.MH_OK and n == 1
        assert mh.mh_ctx_tune_lookup(ctx, p, T, 500, 600, 450) == 3
        mh.check(mh.mh_ctx_set_autotune(ctx, 1))  # use the cache, never tune
        got, want = _product(mh, ctx, p, T, N, P, (81, 82, 83))
        assert np.array_equal(got, want)
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)
