"""A seeded sweep over the whole product interface: random tile edge,
modulus, parent sizes, block placements, arithmetic form and the subtract
flag, every case against the oracle on whole parents.  Bar: bit-exact."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import device_of, host_of, parent_host, say, stream_handle, to_cart, to_mh, torch_cuda

pytestmark = pytest.mark.gpu

PRIMES = [2, 3, 251, 257, 40961, 65521, 65537, (1 << 24) - 3, 67108859, 2**31 - 1]


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


@pytest.mark.parametrize("seed", range(48))
def test_random_case(mh, ctx, seed):
    g = np.random.default_rng(90_000 + seed)
    T = int(g.choice([16, 32, 64, 128]))
    p = int(g.choice(PRIMES))
    forms = [mh.MH_MODE_PLAIN_U32, mh.MH_MODE_LIMB_I8, mh.MH_MODE_AUTO,
             mh.MH_MODE_PLAIN_ELEMENTWISE]
    if p < (1 << 26):
        forms.append(mh.MH_MODE_FP64)
    mode = int(g.choice(forms)) | (mh.MH_SUBTRACT if g.integers(0, 2) else 0)
    NA, NB, NC = (T << int(g.integers(0, 4 if T <= 32 else 3)) for _ in range(3))
    m = int(g.integers(1, min(NC, NA) + 1))
    k = int(g.integers(1, min(NA, NB) + 1))
    n = int(g.integers(1, min(NC, NB) + 1))
    rc, cc = int(g.integers(0, NC - m + 1)), int(g.integers(0, NC - n + 1))
    ra, ca = int(g.integers(0, NA - m + 1)), int(g.integers(0, NA - k + 1))
    rb, cb = int(g.integers(0, NB - k + 1)), int(g.integers(0, NB - n + 1))
    say("sweep", seed, dict(T=T, p=p, mode=mode, N=(NA, NB, NC), mkn=(m, k, n)))
    A, B, C = (parent_host(91_000 + 3 * seed + i, p, N) for i, N in enumerate((NA, NB, NC)))
    Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X, N in ((A, NA), (B, NB), (C, NC)))
    mh.check(mh.mh_matmul_modp(ctx, Cd.data_ptr(), NC, rc, cc, Ad.data_ptr(), NA, ra, ca,
                               Bd.data_ptr(), NB, rb, cb, m, k, n, p, T, mode,
                               stream_handle()))
    want = C.copy()
    oracle.matmul_modp_view(want, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n,
                            subtract=bool(mode & mh.MH_SUBTRACT))
    assert np.array_equal(host_of(to_cart(mh, ctx, Cd, NC, T)), want)
    assert np.array_equal(host_of(to_cart(mh, ctx, Ad, NA, T)), A)
    assert mh.mh_ctx_last_device_error(ctx) == 0
