"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

* 4096^3, p = 65521: every output of the limb and FP64 forms against the full
  oracle product.
* 8192^3, p = 2^31 - 1, one GPU's 2048 x 4096 x 8192 share of it (the 4 x 2
  split of C), and the non-aligned 6000 x 3000 x 5000 product inside 8192^2
  parents: every word of the C parent against the oracle's full product
  (the definition on the Cartesian parents, so words outside the block must
  be unchanged); the limb and plain forms (and the FP64 form where
  p < 2^26) agree on every word; sampled outputs recomputed one by one and
  Freivalds' check (two random vectors) as second, independent checks.
"""

import numpy as np
import pytest

import oracle
from seeded_inputs import residues_np, residues_torch
from tests.gpu_util import host_of, say, stream_handle, to_cart, to_mh, torch_cuda

pytestmark = pytest.mark.gpu
P31 = 2**31 - 1


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


def make_parents(mh, ctx, N, T, p, seeds):
    torch = torch_cuda()
    cart, mhp = [], []
    for s in seeds:
        X = residues_torch(s, p, N, N, device="cuda")
        torch.cuda.synchronize()
        cart.append(X)
        mhp.append(to_mh(mh, ctx, X, N, T))
    torch.cuda.synchronize()
    return cart, mhp


def run(mh, ctx, Cm, Am, Bm, N, off, m, k, n, p, T, mode):
    rc, cc, ra, ca, rb, cb = off
    mh.check(mh.mh_matmul_modp(ctx, Cm.data_ptr(), N, rc, cc, Am.data_ptr(), N, ra, ca,
                               Bm.data_ptr(), N, rb, cb, m, k, n, p, T, mode, stream_handle()))


def test_4096_cube_p65521_full_oracle(mh, ctx):
    N, T, p = 4096, 64, 65521
    say("fullsize 4096^3")
    cart, (Am, Bm, Cm) = make_parents(mh, ctx, N, T, p, (2001, 2002, 2003))
    A, B, C0 = (host_of(X) for X in cart)
    Cf = Cm.clone()
    run(mh, ctx, Cm, Am, Bm, N, (0,) * 6, N, N, N, p, T, mh.MH_MODE_LIMB_I8)
    say("fullsize 4096^3 fp64")
    run(mh, ctx, Cf, Am, Bm, N, (0,) * 6, N, N, N, p, T, mh.MH_MODE_FP64)
    got = host_of(to_cart(mh, ctx, Cm, N, T))
    want = C0.copy()
    oracle.matmul_modp(want, A, B, p)
    assert np.array_equal(got, want)
    assert np.array_equal(host_of(to_cart(mh, ctx, Cf, N, T)), want)


def _check_block(mh, ctx, N, T, p, off, m, k, n, seeds, samples=384):
    rc, cc, ra, ca, rb, cb = off
    torch = torch_cuda()
    cart, (Am, Bm, Cm) = make_parents(mh, ctx, N, T, p, seeds)
    Cm2 = Cm.clone()
    Cm3 = Cm.clone() if p <= 0x3FFFFFF else None
    say("fullsize limb", N, off, m, k, n, p)
    run(mh, ctx, Cm, Am, Bm, N, off, m, k, n, p, T, mh.MH_MODE_LIMB_I8)
    say("fullsize plain", N, off, m, k, n, p)
    run(mh, ctx, Cm2, Am, Bm, N, off, m, k, n, p, T, mh.MH_MODE_PLAIN_U32)
    if Cm3 is not None:
        say("fullsize fp64", N, off, m, k, n, p)
        run(mh, ctx, Cm3, Am, Bm, N, off, m, k, n, p, T, mh.MH_MODE_FP64)
    torch.cuda.synchronize()
    # independent kernels agree on every word of the parent
    assert torch.equal(Cm, Cm2)
    if Cm3 is not None:
        assert torch.equal(Cm, Cm3)
    got = host_of(to_cart(mh, ctx, Cm, N, T))
    A, B, C0 = (host_of(X) for X in cart)
    # the whole parent against the oracle's full product, word by word
    say("fullsize oracle", N, off, m, k, n, p)
    want = C0.copy()
    oracle.matmul_modp_view(want, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n)
    bad = int(np.count_nonzero(got != want))
    assert bad == 0, "%d words differ from the oracle" % bad
    del want
    Ab = np.ascontiguousarray(A[ra:ra + m, ca:ca + k])
    Bb = np.ascontiguousarray(B[rb:rb + k, cb:cb + n])
    Cb0 = np.ascontiguousarray(C0[rc:rc + m, cc:cc + n])
    Cb = np.ascontiguousarray(got[rc:rc + m, cc:cc + n])
    # sampled outputs, including the block's corners and edges, one by one
    g = np.random.default_rng(7)
    rows = np.concatenate([[0, 0, m - 1, m - 1], g.integers(0, m, samples)])
    cols = np.concatenate([[0, n - 1, 0, n - 1], g.integers(0, n, samples)])
    want = oracle.matmul_modp_entries(rows, cols, Cb0, Ab, Bb, p)
    assert np.array_equal(Cb[rows, cols], want)
    # the whole block, probabilistically (each vector misses an error w.p. <= 1/p)
    for s in (11, 12):
        x = residues_np(s, p, 1, n)[0]
        assert oracle.freivalds(Cb, Cb0, Ab, Bb, p, x)


def test_8192_cube_p31(mh, ctx):
    _check_block(mh, ctx, 8192, 64, P31, (0,) * 6, 8192, 8192, 8192, (4001, 4002, 4003))


def test_8192_cube_shard_p31(mh, ctx):
    _check_block(mh, ctx, 8192, 64, P31, (2048, 4096, 2048, 0, 0, 4096), 2048, 8192, 4096,
                 (4001, 4002, 4003))


def test_nonaligned_blocks_8192_parents(mh, ctx):
    _check_block(mh, ctx, 8192, 64, 65521, (64, 33, 1000, 1500, 517, 2048), 6000, 3000, 5000,
                 (3001, 3002, 3003))
