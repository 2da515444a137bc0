"""GPU parity of the batched persistent path (queue + graph replay) against the
oracle.  Bar: bit-exact over every parent."""

import numpy as np
import pytest

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


def draw_batch(g, count, NA, NB, NC, nC, smax):
    """count products with disjoint C blocks spread over nC parents."""
    calls, used = [], [[] for _ in range(nC)]
    while len(calls) < count:
        m, k, n = (int(g.integers(1, smax + 1)) for _ in range(3))
        ci = len(calls) % nC
        for _ in range(200):
            rc, cc = int(g.integers(0, NC - m + 1)), int(g.integers(0, NC - n + 1))
            if all(rc + m <= r or r + mm <= rc or cc + n <= c or c + nn <= cc
                   for r, c, mm, nn in used[ci]):
                break
        else:
            continue
        used[ci].append((rc, cc, m, n))
        calls.append(dict(ci=ci, rc=rc, cc=cc, m=m, k=k, n=n,
                          ra=int(g.integers(0, NA - m + 1)), ca=int(g.integers(0, NA - k + 1)),
                          rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1))))
    return calls


def run_batch(mh, ctx, calls, A, B, Cs, Ad, Bd, Cds, NA, NB, NC, p, T, mode):
    descs = mh.make_descs([dict(C=Cds[c["ci"]].data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(),
                                NC=NC, NA=NA, NB=NB, rc=c["rc"], cc=c["cc"], ra=c["ra"],
                                ca=c["ca"], rb=c["rb"], cb=c["cb"], m=c["m"], k=c["k"],
                                n=c["n"]) for c in calls])
    mh.check(mh.mh_matmul_modp_batched(ctx, descs, len(calls), p, T, mode, stream_handle()),
             "batched")
    for c in calls:
        Cs[c["ci"]] = expected_view(Cs[c["ci"]], A, B, p, c["rc"], c["cc"], c["ra"], c["ca"],
                                    c["rb"], c["cb"], c["m"], c["k"], c["n"])
    for ci, Cd in enumerate(Cds):
        got = host_of(to_cart(mh, ctx, Cd, NC, T))
        assert np.array_equal(got, Cs[ci]), "C parent %d differs" % ci
    assert mh.mh_ctx_last_device_error(ctx) == 0


@pytest.mark.parametrize("mode", [2, 1])
@pytest.mark.parametrize("p,T", [(65521, 64), (P31, 32), (251, 16), ((1 << 24) - 3, 128)])
def test_batched_random(mh, ctx, mode, p, T):
    g = np.random.default_rng(900 + T + mode)
    NA = NB = NC = 1024
    nC = 3
    A, B = parent_host(901, p, NA), parent_host(902, p, NB)
    Cs = [parent_host(910 + i, p, NC) for i in range(nC)]
    Ad, Bd = to_mh(mh, ctx, device_of(A), NA, T), to_mh(mh, ctx, device_of(B), NB, T)
    Cds = [to_mh(mh, ctx, device_of(C), NC, T) for C in Cs]
    calls = draw_batch(g, 24, NA, NB, NC, nC, 300)
    say("batched", p, T, mode, len(calls))
    run_batch(mh, ctx, calls, A, B, Cs, Ad, Bd, Cds, NA, NB, NC, p, T, mode)


@pytest.mark.parametrize("apar", ["0", "1"])
@pytest.mark.parametrize("p,T", [(65521, 32), (65521, 128), (251, 64), (251, 32), (65521, 16)])
def test_batched_early_c_forms(mh, ctx, monkeypatch, apar, p, T):
    """The persistent GEMM forms that load C two stages ahead of the epilogue
    (one and two limbs, 32 <= T) and that read A from a panel of the whole
    parent (MH_BATCH_APARENT=1; A blocks at every row and column phase,
    including blocks at the parent's edges and panels starting above the
    parent's first row): tile sizes other than 64, and thin products whose
    output blocks leave whole waves of a workgroup outside them (those waves
    load words they discard and store nothing)."""
    monkeypatch.setenv("MH_BATCH_APARENT", apar)
    g = np.random.default_rng(950 + T + p % 97)
    NA = NB = NC = 1024
    nC = 3
    A, B = parent_host(951, p, NA), parent_host(952, p, NB)
    Cs = [parent_host(960 + i, p, NC) for i in range(nC)]
    Ad, Bd = to_mh(mh, ctx, device_of(A), NA, T), to_mh(mh, ctx, device_of(B), NB, T)
    Cds = [to_mh(mh, ctx, device_of(C), NC, T) for C in Cs]
    calls = [c for c in draw_batch(g, 24, NA, NB, NC, nC, 300) if c["ci"] < 2]
    for i in range(6):  # thin blocks in parent 2, rows disjoint
        m, k, n = 1 + 7 * i, 33 + 50 * i, 100 + 37 * i
        calls.append(dict(ci=2, rc=5 + 150 * i, cc=17 + 3 * i, m=m, k=k, n=n,
                          ra=int(g.integers(0, NA - m + 1)), ca=int(g.integers(0, NA - k + 1)),
                          rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1))))
    # A blocks at the parent's corners (first row and column, last row and
    # column) with C offsets whose row phase exceeds A's first row
    # (the last two also end on C's last row, the last one on its last column)
    for i, (ra, ca, m, k) in enumerate([(0, 0, 70, 90), (NA - 45, NA - 77, 45, 77),
                                        (3, NA - 200, 90, 200), (NA - 90, 1, 90, 31)]):
        n = 50 + 20 * i
        rc = 930 + i % 2 if i < 2 else NC - m
        cc = 400 + 150 * i if i < 3 else NC - n
        calls.append(dict(ci=2, rc=rc, cc=cc, m=m, k=k, n=n, ra=ra, ca=ca,
                          rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1))))
    say("batched early C", p, T, len(calls))
    run_batch(mh, ctx, calls, A, B, Cs, Ad, Bd, Cds, NA, NB, NC, p, T, 2)


def test_batched_a_parent_two_parents(mh, ctx, monkeypatch):
    """The A-parent form with two A parents of different sizes in one batch
    (each packed once, each product reading its own parent's panel)."""
    monkeypatch.setenv("MH_BATCH_APARENT", "1")
    monkeypatch.setenv("MH_LIMB_CFG", "11")  # (small products would get configuration 6)
    p, T = 65521, 64
    NA1, NA2, NB, NC = 1024, 512, 1024, 1024
    A1, A2 = parent_host(971, p, NA1), parent_host(972, p, NA2)
    B = parent_host(973, p, NB)
    Cs = [parent_host(974 + i, p, NC) for i in range(2)]
    A1d, A2d = to_mh(mh, ctx, device_of(A1), NA1, T), to_mh(mh, ctx, device_of(A2), NA2, T)
    Bd = to_mh(mh, ctx, device_of(B), NB, T)
    Cds = [to_mh(mh, ctx, device_of(C), NC, T) for C in Cs]
    g = np.random.default_rng(970)
    calls, descs = [], []
    for i in range(16):  # a 4 x 4 grid of disjoint output cells in each C parent
        ci, cell = i % 2, i // 2
        two = i % 3 == 0
        NA = NA2 if two else NA1
        m, k, n = int(g.integers(20, 250)), int(g.integers(20, 400)), int(g.integers(20, 250))
        c = dict(ci=ci, rc=(cell % 4) * 256 + int(g.integers(0, 256 - m + 1)),
                 cc=(cell // 4) * 256 + int(g.integers(0, 256 - n + 1)), m=m, k=k, n=n,
                 ra=int(g.integers(0, NA - m + 1)), ca=int(g.integers(0, NA - k + 1)),
                 rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1)), two=two)
        calls.append(c)
        descs.append(dict(C=Cds[ci].data_ptr(), A=(A2d if two else A1d).data_ptr(),
                          B=Bd.data_ptr(), NC=NC, NA=NA, NB=NB, rc=c["rc"], cc=c["cc"],
                          ra=c["ra"], ca=c["ca"], rb=c["rb"], cb=c["cb"], m=m, k=k, n=n))
    say("batched a-parent, two parents")
    mh.check(mh.mh_matmul_modp_batched(ctx, mh.make_descs(descs), len(descs), p, T,
                                       mh.MH_MODE_LIMB_I8, stream_handle()), "batched")
    s, _, _, forms = mh.mh_ctx_last_batch_config(ctx)
    assert forms & mh.MH_BATCH_FORM_A_PARENT
    for c in calls:
        Cs[c["ci"]] = expected_view(Cs[c["ci"]], A2 if c["two"] else A1, B, p, c["rc"], c["cc"],
                                    c["ra"], c["ca"], c["rb"], c["cb"], c["m"], c["k"], c["n"])
    for ci, Cd in enumerate(Cds):
        assert np.array_equal(host_of(to_cart(mh, ctx, Cd, NC, T)), Cs[ci]), ci
    assert mh.mh_ctx_last_device_error(ctx) == 0


def test_batched_graph_replay_new_queue(mh, ctx):
    # one captured graph, three batches with different contents and sizes
    p, T = 65521, 64
    NA = NB = NC = 1024
    A, B = parent_host(921, p, NA), parent_host(922, p, NB)
    Cs = [parent_host(930 + i, p, NC) for i in range(2)]
    Ad, Bd = to_mh(mh, ctx, device_of(A), NA, T), to_mh(mh, ctx, device_of(B), NB, T)
    Cds = [to_mh(mh, ctx, device_of(C), NC, T) for C in Cs]
    g = np.random.default_rng(77)
    for rep, (count, smax) in enumerate([(10, 400), (30, 150), (10, 400)]):
        say("replay", rep)
        calls = draw_batch(g, count, NA, NB, NC, 2, smax)
        run_batch(mh, ctx, calls, A, B, Cs, Ad, Bd, Cds, NA, NB, NC, p, T, 2)


def test_batched_tu_level_shapes(mh, ctx):
    # sizes 64 u + r with u in 1..4, r in 1..63, offsets anywhere in 2048 parents
    p, T = 65521, 64
    NA = NB = NC = 2048
    g = np.random.default_rng(5000)
    A, B = parent_host(5001, p, NA), parent_host(5002, p, NB)
    Cs = [parent_host(5100 + i, p, NC) for i in range(4)]
    Ad, Bd = to_mh(mh, ctx, device_of(A), NA, T), to_mh(mh, ctx, device_of(B), NB, T)
    Cds = [to_mh(mh, ctx, device_of(C), NC, T) for C in Cs]
    calls = []
    used = [[] for _ in range(4)]
    while len(calls) < 32:
        m, k, n = (64 * int(g.integers(1, 5)) + int(g.integers(1, 64)) for _ in range(3))
        ci = len(calls) % 4
        rc, cc = int(g.integers(0, NC - m + 1)), int(g.integers(0, NC - n + 1))
        if any(not (rc + m <= r or r + mm <= rc or cc + n <= c or c + nn <= cc)
               for r, c, mm, nn in used[ci]):
            continue
        used[ci].append((rc, cc, m, n))
        calls.append(dict(ci=ci, rc=rc, cc=cc, m=m, k=k, n=n,
                          ra=int(g.integers(0, NA - m + 1)), ca=int(g.integers(0, NA - k + 1)),
                          rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1))))
    run_batch(mh, ctx, calls, A, B, Cs, Ad, Bd, Cds, NA, NB, NC, p, T, 2)


def test_batched_degenerate_and_errors(mh, ctx):
    torch = torch_cuda()
    p, T, N = 65521, 32, 256
    A, B, C = (parent_host(s, p, N) for s in (941, 942, 943))
    Ad, Bd, Cd = (to_mh(mh, ctx, device_of(X), N, T) for X in (A, B, C))
    assert mh.mh_matmul_modp_batched(ctx, None, 0, p, T, 2, stream_handle()) == 0
    base = dict(C=Cd.data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(), NC=N, NA=N, NB=N,
                rc=0, cc=0, ra=0, ca=0, rb=0, cb=0)
    # empty products are skipped; a real one alongside runs
    calls = [dict(base, m=0, k=5, n=5), dict(base, m=5, k=0, n=5, rc=100),
             dict(base, m=40, k=70, n=33, rc=200, cc=10, ra=3, ca=5, rb=7, cb=9)]
    d = mh.make_descs(calls)
    mh.check(mh.mh_matmul_modp_batched(ctx, d, 3, p, T, 2, stream_handle()))
    want = expected_view(C, A, B, p, 200, 10, 3, 5, 7, 9, 40, 70, 33)
    assert np.array_equal(host_of(to_cart(mh, ctx, Cd, N, T)), want)
    # overlapping output blocks
    d = mh.make_descs([dict(base, m=10, k=10, n=10), dict(base, m=10, k=10, n=10, rc=5, cc=5)])
    assert mh.mh_matmul_modp_batched(ctx, d, 2, p, T, 2, 0) == mh.MH_E_ALIAS
    # an output block over another product's input block
    d = mh.make_descs([dict(base, m=10, k=10, n=10, rc=50),
                       dict(base, A=Cd.data_ptr(), m=10, k=10, n=10, ra=55, rc=100)])
    assert mh.mh_matmul_modp_batched(ctx, d, 2, p, T, 2, 0) == mh.MH_E_ALIAS
    d = mh.make_descs([dict(base, m=10, k=10, n=10, rc=250)])
    assert mh.mh_matmul_modp_batched(ctx, d, 1, p, T, 2, 0) == mh.MH_E_BOUNDS
    assert mh.mh_matmul_modp_batched(ctx, d, 1, 1, T, 2, 0) == mh.MH_E_MODULUS
    assert mh.mh_matmul_modp_batched(ctx, d, -1, p, T, 2, 0) == mh.MH_E_INVALID


@pytest.mark.parametrize("apar", ["0", "1"])
def test_batched_subtract(mh, ctx, monkeypatch, apar):
    # (the A-parent form negates B's per-product panels, as the other form)
    monkeypatch.setenv("MH_BATCH_APARENT", apar)
    p, T, N = 65521, 64, 1024
    g = np.random.default_rng(4242)
    A, B = parent_host(951, p, N), parent_host(952, p, N)
    Cs = [parent_host(953, p, N)]
    Ad, Bd = to_mh(mh, ctx, device_of(A), N, T), to_mh(mh, ctx, device_of(B), N, T)
    Cds = [to_mh(mh, ctx, device_of(Cs[0]), N, T)]
    calls = draw_batch(g, 12, N, N, N, 1, 300)
    descs = mh.make_descs([dict(C=Cds[0].data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(), NC=N,
                                NA=N, NB=N, rc=c["rc"], cc=c["cc"], ra=c["ra"], ca=c["ca"],
                                rb=c["rb"], cb=c["cb"], m=c["m"], k=c["k"], n=c["n"])
                           for c in calls])
    for mode in (mh.MH_MODE_LIMB_I8, mh.MH_MODE_PLAIN_U32):
        mh.check(mh.mh_matmul_modp_batched(ctx, descs, len(calls), p, T,
                                           mode | mh.MH_SUBTRACT, stream_handle()))
        for c in calls:
            oracle_sub(Cs[0], A, B, p, c)
        assert np.array_equal(host_of(to_cart(mh, ctx, Cds[0], N, T)), Cs[0]), mode


def oracle_sub(C, A, B, p, c):
    import oracle
    oracle.matmul_modp_view(C, A, B, p, c["rc"], c["cc"], c["ra"], c["ca"], c["rb"], c["cb"],
                            c["m"], c["k"], c["n"], subtract=True)
