"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: bit-exact (integer arithmetic; the stated error is zero).  Whole
parents are compared, so words outside the C block must be unchanged, and
the A and B parents are checked unchanged too.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import (device_of, expected_view, host_of, parent_host, say,
                            stream_handle, to_cart, to_mh, torch_cuda)

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


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("T", [16, 32, 64, 128])
@pytest.mark.parametrize("q", [0, 2, 3])
@pytest.mark.parametrize("pad", [0, 3, 4])
def test_layout_raw_and_roundtrip(mh, ctx, T, q, pad):
    torch = torch_cuda()
    N = T << q
    say("layout", T, N, pad)
    X = parent_host(11 + q + T, P31, N)
    ld = N + pad
    Xp = np.zeros((N, ld), np.uint32)
    Xp[:, :N] = X
    src = device_of(Xp)
    dst = torch.empty(N * N, dtype=torch.int32, device="cuda")
    mh.check(mh.mh_layout_from_cartesian(ctx, dst.data_ptr(), src.data_ptr(), ld, N, T,
                                         stream_handle()))
    raw = host_of(dst)
    assert np.array_equal(raw, oracle.mh_from_cartesian(X, T))
    back = torch.zeros((N, ld), dtype=torch.int32, device="cuda")
    mh.check(mh.mh_layout_to_cartesian(ctx, back.data_ptr(), ld, dst.data_ptr(), N, T,
                                       stream_handle()))
    got = host_of(back)
    assert np.array_equal(got[:, :N], X)
    assert not got[:, N:].any()  # padding columns untouched


def test_layout_errors(mh, ctx):
    torch = torch_cuda()
    a = torch.zeros(64 * 64, dtype=torch.int32, device="cuda")
    assert mh.mh_layout_from_cartesian(ctx, a.data_ptr(), a.data_ptr(), 64, 64, 16, 0) == \
        mh.MH_E_ALIAS
    b = torch.zeros(64 * 64, dtype=torch.int32, device="cuda")
    assert mh.mh_layout_from_cartesian(ctx, b.data_ptr(), a.data_ptr(), 63, 64, 16, 0) == \
        mh.MH_E_INVALID
    assert mh.mh_layout_from_cartesian(ctx, b.data_ptr(), a.data_ptr(), 64, 48, 16, 0) == \
        mh.MH_E_SHAPE
    assert mh.mh_layout_from_cartesian(ctx, b.data_ptr(), a.data_ptr(), 64, 64, 8, 0) == \
        mh.MH_E_UNSUPPORTED


# ----------------------------------------------------------------- product

def run_product(mh, ctx, P, p, T, mode, seeds=(1, 2, 3), C_host=None, A_host=None,
                B_host=None):
    """Run one product through the library and compare whole parents with the oracle."""
    NC, NA, NB = P["NC"], P["NA"], P["NB"]
    A = A_host if A_host is not None else parent_host(seeds[0], p, NA)
    B = B_host if B_host is not None else parent_host(seeds[1], p, NB)
    C = C_host if C_host is not None else parent_host(seeds[2], p, NC)
    say("product", P, "p", p, "T", T, "mode", mode)
    Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X, N in ((A, NA), (B, NB), (C, NC)))
    st = mh.mh_matmul_modp(ctx, Cd.data_ptr(), NC, P["rc"], P["cc"], Ad.data_ptr(), NA,
                           P["ra"], P["ca"], Bd.data_ptr(), NB, P["rb"], P["cb"], P["m"],
                           P["k"], P["n"], p, T, mode, stream_handle())
    mh.check(st, "mh_matmul_modp")
    got = host_of(to_cart(mh, ctx, Cd, NC, T))
    want = expected_view(C, A, B, p, P["rc"], P["cc"], P["ra"], P["ca"], P["rb"], P["cb"],
                         P["m"], P["k"], P["n"])
    bad = np.argwhere(got != want)
    assert bad.size == 0, "first mismatches %s got %s want %s" % (
        bad[:5].tolist(), got[tuple(bad[:5].T)], want[tuple(bad[:5].T)])
    assert np.array_equal(host_of(to_cart(mh, ctx, Ad, NA, T)), A)
    assert np.array_equal(host_of(to_cart(mh, ctx, Bd, NB, T)), B)
    assert mh.mh_ctx_last_device_error(ctx) == 0


MODES = pytest.mark.parametrize("mode", [1, 2, 4])  # plain, limb, elementwise comparator


@MODES
def test_small_aligned_256(mh, ctx, mode):
    # A, B 256 x 256, C zero-initialised, p = 65521, T' = 32, offsets 0
    P = dict(NC=256, NA=256, NB=256, rc=0, cc=0, ra=0, ca=0, rb=0, cb=0, m=256, k=256, n=256)
    run_product(mh, ctx, P, 65521, 32, mode, seeds=(1001, 1002, 1003),
                C_host=np.zeros((256, 256), np.uint32))


@MODES
@pytest.mark.parametrize("p", [2, 251, 65521, (1 << 24) - 3, P31])
def test_aligned_square_all_primes(mh, ctx, mode, p):
    P = dict(NC=256, NA=256, NB=256, rc=0, cc=0, ra=0, ca=0, rb=0, cb=0, m=256, k=256, n=256)
    run_product(mh, ctx, P, p, 64, mode, seeds=(21, 22, 23))


def _rand_product(g, T, qmax):
    NC, NA, NB = (T * 2 ** int(g.integers(1, qmax + 1)) for _ in range(3))
    m = int(g.integers(1, min(NC, NA) + 1))
    k = int(g.integers(1, min(NA, NB) + 1))
    n = int(g.integers(1, min(NC, NB) + 1))
    return dict(NC=NC, NA=NA, NB=NB, m=m, k=k, n=n,
                rc=int(g.integers(0, NC - m + 1)), cc=int(g.integers(0, NC - n + 1)),
                ra=int(g.integers(0, NA - m + 1)), ca=int(g.integers(0, NA - k + 1)),
                rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1)))


@MODES
@pytest.mark.parametrize("seed", range(10))
def test_random_nonaligned(mh, ctx, mode, seed):
    g = np.random.default_rng(500 + seed)
    T = int(g.choice([16, 32, 64, 128]))
    p = int(g.choice([3, 65521, 40961, (1 << 24) - 3, P31]))
    P = _rand_product(g, T, 3 if T <= 32 else 2)
    run_product(mh, ctx, P, p, T, mode, seeds=(600 + seed, 700 + seed, 800 + seed))


@MODES
def test_nonaligned_like_tu_step(mh, ctx, mode):
    # scattered blocks on all three operands, ragged against every grid
    P = dict(NC=512, NA=512, NB=512, rc=64, cc=33, ra=100, ca=150, rb=51, cb=204,
             m=300, k=250, n=275)
    run_product(mh, ctx, P, 65521, 64, mode, seeds=(31, 32, 33))


@MODES
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (1, 300, 1), (300, 1, 300), (0, 5, 5),
                                   (5, 0, 5), (5, 5, 0), (33, 65, 97)])
def test_degenerate_sizes(mh, ctx, mode, m, k, n):
    P = dict(NC=512, NA=512, NB=512, rc=511 - m if m else 0, cc=17, ra=3, ca=512 - k,
             rb=512 - k, cb=512 - n, m=m, k=k, n=n)
    run_product(mh, ctx, P, P31, 32, mode, seeds=(41, 42, 43))


@MODES
def test_same_parent_disjoint_blocks(mh, ctx, mode):
    # The Schur update of a TU step: one matrix, C block written from A and B blocks
    torch = torch_cuda()
    N, T, p = 512, 32, 65521
    X = parent_host(51, p, N)
    Xd = to_mh(mh, ctx, device_of(X), N, T)
    rc, cc, ra, ca, rb, cb, m, k, n = 300, 290, 0, 5, 40, 250, 200, 220, 210
    st = mh.mh_matmul_modp(ctx, Xd.data_ptr(), N, rc, cc, Xd.data_ptr(), N, ra, ca,
                           Xd.data_ptr(), N, rb, cb, m, k, n, p, T, mode, stream_handle())
    mh.check(st)
    got = host_of(to_cart(mh, ctx, Xd, N, T))
    want = X.copy()
    prod = np.zeros((m, n), np.uint32)
    oracle.matmul_modp(prod, np.ascontiguousarray(X[ra:ra + m, ca:ca + k]),
                       np.ascontiguousarray(X[rb:rb + k, cb:cb + n]), p)
    want[rc:rc + m, cc:cc + n] = ((want[rc:rc + m, cc:cc + n].astype(np.uint64) + prod) % p)
    assert np.array_equal(got, want)


def test_alias_rejected(mh, ctx):
    torch = torch_cuda()
    X = torch.zeros(256 * 256, dtype=torch.int32, device="cuda")
    Y = torch.zeros(256 * 256, dtype=torch.int32, device="cuda")
    d = X.data_ptr()
    # C block overlaps the A block in the same parent
    assert mh.mh_matmul_modp(ctx, d, 256, 0, 0, d, 256, 10, 10, Y.data_ptr(), 256, 0, 0,
                             20, 20, 20, 65521, 32, 1, 0) == mh.MH_E_ALIAS
    # overlapping storage of another shape
    assert mh.mh_matmul_modp(ctx, d, 256, 0, 0, d + 4 * 64, 128, 100, 0, Y.data_ptr(), 256,
                             0, 0, 4, 4, 4, 65521, 32, 1, 0) == mh.MH_E_ALIAS
    assert mh.mh_matmul_modp(ctx, d, 256, 0, 0, Y.data_ptr(), 256, 0, 0, Y.data_ptr(), 256,
                             0, 0, 4, 4, 4, 1, 32, 1, 0) == mh.MH_E_MODULUS
    assert mh.mh_matmul_modp(ctx, d, 256, 250, 0, Y.data_ptr(), 256, 0, 0, Y.data_ptr(), 256,
                             0, 0, 8, 4, 4, 65521, 32, 1, 0) == mh.MH_E_BOUNDS
    # A parent not 16-byte aligned
    Z = torch.zeros(256 * 256 + 4, dtype=torch.int32, device="cuda")
    assert mh.mh_matmul_modp(ctx, d, 256, 0, 0, Z.data_ptr() + 4, 256, 0, 0, Y.data_ptr(), 256,
                             0, 0, 4, 4, 4, 65521, 32, 2, 0) == mh.MH_E_INVALID


@MODES
@pytest.mark.parametrize("p", [65521, P31])
@pytest.mark.parametrize("kind", ["pm1", "H", "H1", "lowdigits"])
def test_adversarial_values(mh, ctx, mode, p, kind):
    # residues at the edges of the limb representation: p-1 everywhere, the
    # largest centred value H_L, the most negative one (H_L + 1), and values
    # whose low digits are all -128
    L = 2 if p < 65536 else 4
    H = 127 * (256**L - 1) // 255
    val = {"pm1": p - 1, "H": H, "H1": H + 1,
           "lowdigits": (0x80 * (1 + 256 + 65536)) % p}[kind]
    N, T = 1024, 64
    A = np.full((N, N), val, np.uint32)
    B = np.full((N, N), val, np.uint32)
    C = np.full((N, N), p - 1, np.uint32)
    P = dict(NC=N, NA=N, NB=N, rc=0, cc=0, ra=0, ca=0, rb=0, cb=0, m=N, k=N, n=N)
    run_product(mh, ctx, P, p, T, mode, C_host=C, A_host=A, B_host=B)


@MODES
@pytest.mark.parametrize("p", [2, 65521, P31])
def test_subtractive_update(mh, ctx, mode, p):
    # C := C - A.B mod p, the Schur complement step, on scattered blocks
    N, T = 512, 64
    A, B, C = (parent_host(s, p, N) for s in (81, 82, 83))
    Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X in (A, B, C))
    rc, cc, ra, ca, rb, cb, m, k, n = 30, 70, 100, 3, 200, 41, 300, 257, 333
    mh.check(mh.mh_matmul_modp(ctx, Cd.data_ptr(), N, rc, cc, Ad.data_ptr(), N, ra, ca,
                               Bd.data_ptr(), N, rb, cb, m, k, n, p, T,
                               mode | mh.MH_SUBTRACT, stream_handle()))
    want = C.copy()
    oracle.matmul_modp_view(want, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n, subtract=True)
    assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), want)
    assert mh.mh_matmul_modp(ctx, Cd.data_ptr(), N, 0, 0, Ad.data_ptr(), N, 0, 0, Bd.data_ptr(),
                             N, 0, 0, 4, 4, 4, p, T, mode | 0x200, 0) == mh.MH_E_UNSUPPORTED


@MODES
def test_subtractive_schur_same_parent(mh, ctx, mode):
    # One matrix: X[rc.., cc..] -= X[ra.., ca..] X[rb.., cb..], blocks disjoint
    N, T, p = 512, 32, P31
    X = parent_host(91, p, N)
    Xd = to_mh(mh, ctx, device_of(X), N, T)
    rc, cc, ra, ca, rb, cb, m, k, n = 257, 260, 1, 2, 33, 260, 250, 190, 240
    mh.check(mh.mh_matmul_modp(ctx, Xd.data_ptr(), N, rc, cc, Xd.data_ptr(), N, ra, ca,
                               Xd.data_ptr(), N, rb, cb, m, k, n, p, T,
                               mode | mh.MH_SUBTRACT, stream_handle()))
    want = X.copy()
    prod = np.zeros((m, n), np.uint32)
    oracle.matmul_modp(prod, np.ascontiguousarray(X[ra:ra + m, ca:ca + k]),
                       np.ascontiguousarray(X[rb:rb + k, cb:cb + n]), p)
    blk = want[rc:rc + m, cc:cc + n].astype(np.int64) - prod.astype(np.int64)
    want[rc:rc + m, cc:cc + n] = (blk % p).astype(np.uint32)
    assert np.array_equal(host_of(to_cart(mh, ctx, Xd, N, T)), want)


# ------------------------------------------------------- padded parents

@pytest.mark.parametrize("rows,cols,T,ldpad", [(1000, 700, 32, 0), (333, 517, 16, 3),
                                               (64, 64, 64, 0), (129, 1, 128, 5)])
def test_padded_layout_roundtrip(mh, ctx, rows, cols, T, ldpad):
    torch = torch_cuda()
    s, N = mh.mh_parent_size(rows, cols, T)
    mh.check(s)
    say("padded layout", rows, cols, T, N)
    X = parent_host(301 + T, P31, max(rows, cols))[:rows, :cols]
    ld = cols + ldpad
    Xp = np.full((rows, ld), 0xDEADBEEF, np.uint32)
    Xp[:, :cols] = X
    src = device_of(Xp)
    dst = torch.full((N * N,), -1, dtype=torch.int32, device="cuda")
    mh.check(mh.mh_layout_from_cartesian_padded(ctx, dst.data_ptr(), N, src.data_ptr(), ld,
                                                rows, cols, T, stream_handle()))
    full = np.zeros((N, N), np.uint32)
    full[:rows, :cols] = X
    assert np.array_equal(host_of(dst), oracle.mh_from_cartesian(full, T))
    back = device_of(np.full((rows, ld), 7, np.uint32))
    mh.check(mh.mh_layout_to_cartesian_padded(ctx, back.data_ptr(), ld, rows, cols,
                                              dst.data_ptr(), N, T, stream_handle()))
    got = host_of(back)
    assert np.array_equal(got[:, :cols], X)
    assert (got[:, cols:] == 7).all()  # row padding of the destination untouched
    assert mh.mh_layout_from_cartesian_padded(ctx, dst.data_ptr(), N, src.data_ptr(), ld,
                                              N + 1, cols, T, 0) == mh.MH_E_INVALID


@MODES
def test_schur_update_on_padded_matrix(mh, ctx, mode):
    # The caller side of a TU step on a 1000 x 1000 matrix (not a power of two):
    # pad into a 1024 x 1024 parent, X22 -= X21 X12 mod p, read the matrix back.
    torch = torch_cuda()
    p, T, n0, h = 65521, 32, 1000, 437
    s, N = mh.mh_parent_size(n0, n0, T)
    X = parent_host(401, p, n0)
    src = device_of(X)
    Xm = torch.empty(N * N, dtype=torch.int32, device="cuda")
    mh.check(mh.mh_layout_from_cartesian_padded(ctx, Xm.data_ptr(), N, src.data_ptr(), n0, n0,
                                                n0, T, stream_handle()))
    r = n0 - h
    mh.check(mh.mh_matmul_modp(ctx, Xm.data_ptr(), N, h, h, Xm.data_ptr(), N, h, 0,
                               Xm.data_ptr(), N, 0, h, r, h, r, p, T, mode | mh.MH_SUBTRACT,
                               stream_handle()))
    out = device_of(np.zeros((n0, n0), np.uint32))
    mh.check(mh.mh_layout_to_cartesian_padded(ctx, out.data_ptr(), n0, n0, n0, Xm.data_ptr(), N,
                                              T, stream_handle()))
    want = X.copy()
    oracle.matmul_modp_view(want, X, X, p, h, h, h, 0, 0, h, r, h, r, subtract=True)
    assert np.array_equal(host_of(out), want)
