"""GPU parity of the FP64-MFMA form (primes below 2^26) against the oracle.

Bar: bit-exact.  The largest prime below 2^26 forces a reduction mod p every
two MFMA steps (depth 8), so long products there exercise the deferred
reduction at its tightest bound; p = 65521 never reduces before the end.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import (device_of, expected_view, host_of, parent_host, say,
                            stream_handle, to_cart, to_mh, torch_cuda)
from tests.test_gpu_parity import _rand_product, run_product

pytestmark = pytest.mark.gpu

P26 = 67108859  # largest prime below 2^26
FP64 = 3


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


@pytest.mark.parametrize("p", [2, 3, 251, 65521, (1 << 24) - 3, P26])
@pytest.mark.parametrize("T", [16, 64, 128])
def test_aligned_square(mh, ctx, p, T):
    P = dict(NC=256, NA=256, NB=256, rc=0, cc=0, ra=0, ca=0, rb=0, cb=0, m=256, k=256, n=256)
    run_product(mh, ctx, P, p, T, mh.MH_MODE_FP64, seeds=(61, 62, 63))


@pytest.mark.parametrize("seed", range(10))
def test_random_nonaligned(mh, ctx, seed):
    g = np.random.default_rng(1500 + seed)
    T = int(g.choice([16, 32, 64, 128]))
    p = int(g.choice([3, 65521, 40961, (1 << 24) - 3, P26]))
    P = _rand_product(g, T, 3 if T <= 32 else 2)
    run_product(mh, ctx, P, p, T, mh.MH_MODE_FP64, seeds=(1600 + seed, 1700 + seed, 1800 + seed))


@pytest.mark.parametrize("kind", ["H", "H1", "pm1"])
def test_extreme_values_tightest_bound(mh, ctx, kind):
    # every centred value at its largest magnitude, k = 2048: 256 reductions
    # at depth 8, each right at the 2^53 bound
    p = P26
    H = (p - 1) // 2
    val = {"H": H, "H1": H + 1, "pm1": p - 1}[kind]
    N, T = 2048, 64
    A = np.full((N, N), val, np.uint32)
    B = np.full((N, N), val, np.uint32)
    C = np.full((N, N), p - 1, np.uint32)
    P = dict(NC=N, NA=N, NB=N, rc=0, cc=0, ra=0, ca=0, rb=0, cb=0, m=256, k=N, n=384)
    run_product(mh, ctx, P, p, T, mh.MH_MODE_FP64, C_host=C, A_host=A, B_host=B)


def test_subtract_and_batched(mh, ctx):
    p, T, N = P26, 64, 1024
    A, B, C = (parent_host(s, p, N) for s in (71, 72, 73))
    Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X in (A, B, C))
    say("fp64 subtract")
    rc, cc, ra, ca, rb, cb, m, k, n = 5, 600, 130, 7, 300, 301, 400, 555, 333
    mh.check(mh.mh_matmul_modp(ctx, Cd.data_ptr(), N, rc, cc, Ad.data_ptr(), N, ra, ca,
                               Bd.data_ptr(), N, rb, cb, m, k, n, p, T,
                               mh.MH_MODE_FP64 | mh.MH_SUBTRACT, stream_handle()))
    want = C.copy()
    oracle.matmul_modp_view(want, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n, subtract=True)
    assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), want)
    say("fp64 batched")
    calls = [dict(rc=500, cc=0, ra=0, ca=0, rb=0, cb=0, m=300, k=400, n=200),
             dict(rc=0, cc=0, ra=1, ca=2, rb=3, cb=4, m=64, k=1000, n=65),
             dict(rc=900, cc=900, ra=17, ca=900, rb=5, cb=3, m=100, k=100, n=100)]
    descs = mh.make_descs([dict(C=Cd.data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(), NC=N, NA=N,
                                NB=N, **c) for c in calls])
    mh.check(mh.mh_matmul_modp_batched(ctx, descs, len(calls), p, T, mh.MH_MODE_FP64,
                                       stream_handle()))
    for c in calls:
        want = expected_view(want, A, B, p, c["rc"], c["cc"], c["ra"], c["ca"], c["rb"],
                             c["cb"], c["m"], c["k"], c["n"])
    assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), want)
    assert mh.mh_ctx_last_device_error(ctx) == 0


def test_modulus_limit(mh, ctx):
    torch = torch_cuda()
    X = torch.zeros(256 * 256, dtype=torch.int32, device="cuda")
    Y = torch.zeros(256 * 256, dtype=torch.int32, device="cuda")
    for p, ok in [(P26, True), ((1 << 26) + 15, False), (2**31 - 1, False)]:
        st = mh.mh_matmul_modp(ctx, X.data_ptr(), 256, 0, 0, Y.data_ptr(), 256, 0, 0,
                               Y.data_ptr(), 256, 0, 0, 8, 8, 8, p, 32, mh.MH_MODE_FP64, 0)
        assert st == (mh.MH_OK if ok else mh.MH_E_MODULUS), p
    torch.cuda.synchronize()
