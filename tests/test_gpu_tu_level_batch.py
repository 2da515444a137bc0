"""The 512-product TU-level batch at its full size, against the oracle word by word.

The products of one level of the TU recursion are independent (section 2.2,
Prop. 2.6) and run as one batched call: 512 products with m, k, n = 64 u + r
(u uniform in 1..32, r in 1..63), A and B blocks anywhere in one shared
8192 x 8192 parent each, product i writing C parent i mod 64 at a C offset
disjoint from the other products of that parent (seeded draw,
``seeded_inputs.tu_level_batch(seed=5000)``), p = 65521, T = 64, the limb
form in its default configuration: the launch bench.py times.

Every one of the 64 C parents is compared with the oracle on every word (the
definition applied, product by product, to the Cartesian parent, so words
outside the products' blocks must be unchanged), one parent at a time to keep
host memory near a gigabyte.  The A and B parents must be unchanged.

The batch has 512 products, more than the 64 the batch queue starts with,
so this call also grows the context's queue (and captures its graph) on
the way; a second test grows one context's queue past a graph already
captured (24, then 65, then 200 products), and a third issues batches of
alternating output shapes and moduli back to back, with one host
synchronisation at the end.
"""

import numpy as np
import pytest

import oracle
from seeded_inputs import residues_torch, tu_level_batch
from tests.gpu_util import (device_of, host_of, parent_host, say, stream_handle, to_cart,
                            to_mh, torch_cuda)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_1705_04807_amd as m
    return m


def _descs(mh, calls, Ad, Bd, Cds, NA, NB, NC):
    return mh.make_descs([dict(C=Cds[c["ci"]].data_ptr(), A=Ad.data_ptr(), B=Bd.data_ptr(),
                               NC=NC, NA=NA, NB=NB, rc=c["rc"], cc=c["cc"], ra=c["ra"],
                               ca=c["ca"], rb=c["rb"], cb=c["cb"], m=c["m"], k=c["k"],
                               n=c["n"]) for c in calls])


@pytest.mark.timeout(900)
def test_tu_level_batch_512_products_8192_parents(mh):
    torch = torch_cuda()
    N, T, p, nC = 8192, 64, 65521, 64
    calls = tu_level_batch(seed=5000, count=512, N=N, n_c_parents=nC)
    work = sum(2 * c["m"] * c["k"] * c["n"] for c in calls)
    say("tu batch: 512 products, 2mnk = %.4g" % work)
    ctx = mh.mh_ctx_create(0)
    try:
        def mh_parent(seed):
            X = residues_torch(seed, p, N, N, device="cuda")
            Y = to_mh(mh, ctx, X, N, T)
            torch.cuda.synchronize()
            return X, Y
        Acart, Ad = mh_parent(5001)
        Bcart, Bd = mh_parent(5002)
        A, B = host_of(Acart), host_of(Bcart)
        del Acart, Bcart
        Ad0, Bd0 = Ad.clone(), Bd.clone()
        Cds = []
        for j in range(nC):
            X, Y = mh_parent(5100 + j)
            del X
            Cds.append(Y)
        say("tu batch: parents ready")
        mh.check(mh.mh_matmul_modp_batched(ctx, _descs(mh, calls, Ad, Bd, Cds, N, N, N),
                                           len(calls), p, T, mh.MH_MODE_LIMB_I8,
                                           stream_handle()), "batched")
        torch.cuda.synchronize()
        assert mh.mh_ctx_last_device_error(ctx) == 0
        assert torch.equal(Ad, Ad0) and torch.equal(Bd, Bd0)
        del Ad0, Bd0
        say("tu batch: GPU done")
        for j in range(nC):
            want = host_of(residues_torch(5100 + j, p, N, N, device="cuda"))
            mine = [c for c in calls if c["ci"] == j]
            for c in mine:
                oracle.matmul_modp_view(want, A, B, p, c["rc"], c["cc"], c["ra"], c["ca"],
                                        c["rb"], c["cb"], c["m"], c["k"], c["n"])
            got = host_of(to_cart(mh, ctx, Cds[j], N, T))
            bad = int(np.count_nonzero(got != want))
            say("tu batch: C parent %d (%d products): %d words differ" % (j, len(mine), bad))
            assert bad == 0
            del want, got
    finally:
        mh.mh_ctx_destroy(ctx)
        torch.cuda.empty_cache()


def _draw(g, count, N, nC, smax, used):
    calls = []
    while len(calls) < count:
        m, k, n = (int(g.integers(1, smax + 1)) for _ in range(3))
        ci = int(g.integers(0, nC))
        rc, cc = int(g.integers(0, N - m + 1)), int(g.integers(0, N - n + 1))
        if any(not (rc + m <= r or r + mm <= rc or cc + n <= c or c + nn <= cc)
               for r, c, mm, nn in used[ci]):
            continue
        used[ci].append((rc, cc, m, n))
        calls.append(dict(ci=ci, rc=rc, cc=cc, m=m, k=k, n=n,
                          ra=int(g.integers(0, N - m + 1)), ca=int(g.integers(0, N - k + 1)),
                          rb=int(g.integers(0, N - k + 1)), cb=int(g.integers(0, N - n + 1))))
    return calls


def test_queue_regrowth_after_capture(mh):
    """24, then 65, then 200 products on one context: the queue (64 products at
    first) grows twice after graphs exist, which waits for the context's work,
    destroys the graphs and captures them again."""
    N, T, p, nC = 1024, 64, 65521, 4
    A, B = parent_host(6001, p, N), parent_host(6002, p, N)
    Cs = [parent_host(6100 + j, p, N) for j in range(nC)]
    ctx = mh.mh_ctx_create(0)
    try:
        Ad, Bd = to_mh(mh, ctx, device_of(A), N, T), to_mh(mh, ctx, device_of(B), N, T)
        Cds = [to_mh(mh, ctx, device_of(C), N, T) for C in Cs]
        g = np.random.default_rng(6000)
        used = [[] for _ in range(nC)]
        for count in (24, 65, 200):
            calls = _draw(g, count, N, nC, 72, used)
            say("regrowth: batch of", count)
            mh.check(mh.mh_matmul_modp_batched(ctx, _descs(mh, calls, Ad, Bd, Cds, N, N, N),
                                               count, p, T, mh.MH_MODE_LIMB_I8, stream_handle()))
            for c in calls:
                oracle.matmul_modp_view(Cs[c["ci"]], A, B, p, c["rc"], c["cc"], c["ra"],
                                        c["ca"], c["rb"], c["cb"], c["m"], c["k"], c["n"])
            for j in range(nC):
                assert np.array_equal(host_of(to_cart(mh, ctx, Cds[j], N, T)), Cs[j]), (count, j)
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)


def test_back_to_back_batches_alternating_shapes_and_moduli(mh, monkeypatch):
    """Batches whose kernel configuration (small or large mean output area),
    limb count (p = 65521 or 2^31 - 1) and, at two limbs, GEMM form (A from
    per-product panels or from the parent's: MH_BATCH_APARENT) alternate
    from call to call, issued without a host synchronisation in between; one
    synchronisation at the end, then every C parent against the oracle."""
    torch = torch_cuda()
    N, T = 2048, 64
    P16, P31 = 65521, 2**31 - 1
    # residues mod 65521 are residues mod 2^31 - 1 as well: A and B serve both
    A, B = parent_host(6201, P16, N), parent_host(6202, P16, N)
    C16 = [parent_host(6210 + j, P16, N) for j in range(2)]
    C31 = [parent_host(6220 + j, P31, N) for j in range(2)]
    ctx = mh.mh_ctx_create(0)
    try:
        Ad, Bd = to_mh(mh, ctx, device_of(A), N, T), to_mh(mh, ctx, device_of(B), N, T)
        D16 = [to_mh(mh, ctx, device_of(C), N, T) for C in C16]
        D31 = [to_mh(mh, ctx, device_of(C), N, T) for C in C31]
        torch.cuda.synchronize()
        g = np.random.default_rng(6200)
        plan = []
        for rep in range(3):
            for p, Cs, Ds in ((P16, C16, D16), (P31, C31, D31)):
                # mean output area below 512^2 (64 x 64 blocks), then above it
                for smax, count in ((120, 12), (1400, 3)):
                    monkeypatch.setenv("MH_BATCH_APARENT", str(rep % 2))
                    calls = _draw(g, count, N, 2, smax, [[], []])
                    say("alternating: rep", rep, "p", p, "smax", smax)
                    mh.check(mh.mh_matmul_modp_batched(
                        ctx, _descs(mh, calls, Ad, Bd, Ds, N, N, N), count, p, T,
                        mh.MH_MODE_LIMB_I8, stream_handle()))
                    plan.append((p, Cs, calls))
        torch.cuda.synchronize()
        for p, Cs, calls in plan:
            for c in calls:
                oracle.matmul_modp_view(Cs[c["ci"]], A, B, p, c["rc"], c["cc"], c["ra"],
                                        c["ca"], c["rb"], c["cb"], c["m"], c["k"], c["n"])
        for Cs, Ds in ((C16, D16), (C31, D31)):
            for C, D in zip(Cs, Ds):
                assert np.array_equal(host_of(to_cart(mh, ctx, D, N, T)), C)
        assert mh.mh_ctx_last_device_error(ctx) == 0
    finally:
        mh.mh_ctx_destroy(ctx)
