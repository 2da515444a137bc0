"""Host-side parts of libmh checked on the CPU: exported symbols, index math,
classification, argument validation and the planner, each against the oracle."""

import os
import re

import numpy as np
import pytest

import oracle

mh = pytest.importorskip("paper_1705_04807_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TS = [16, 32, 64, 128]


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mh.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mh_[a-z_0-9]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = header_functions()
    assert len(names) >= 16
    assert sorted(mh.EXPORTS) == names
    for n in names:
        assert hasattr(mh.lib, n), n


def test_null_context_is_rejected():
    for call in (lambda: mh.lib.mh_ctx_kernel_times(None, 0, None, 0, None),
                 lambda: mh.lib.mh_ctx_set_timing(None, 1),
                 lambda: mh.lib.mh_ctx_set_autotune(None, 1),
                 lambda: mh.lib.mh_ctx_destroy(None),
                 lambda: mh.lib.mh_probe_mfma_i8(None, 1000, None, None),
                 lambda: mh.lib.mh_probe_valu_mac(None, 1000, None, None)):
        assert call() == mh.MH_E_INVALID


def test_status_strings():
    for s in range(0, 9):
        assert mh.mh_status_string(s)
    assert mh.mh_status_string(99) == "unknown status"


# ---------------------------------------------------------------- index math

def test_encode_golden_and_oracle():
    for i, j, T, z in [(1000, 1500, 64, 1833500), (100, 200, 32, 30856),
                       (8191, 8191, 64, 67108863)]:
        assert mh.mh_encode(i, j, T) == z
        assert mh.mh_extract(z, T) == (i, j)
    g = np.random.default_rng(5)
    for T in TS:
        for N in (T, 4 * T, 1 << 14):
            for _ in range(200):
                i, j = (int(v) for v in g.integers(0, N, 2))
                z = mh.mh_encode(i, j, T)
                assert z == oracle.mh_encode(i, j, T, N)
                assert mh.mh_extract(z, T) == (i, j)


def test_encode_large_coordinates():
    # 2^18 parents: the dilated-integer encoder against the level walk
    N, T = 1 << 18, 16
    for i, j in [(N - 1, N - 1), (N - 1, 0), (0, N - 1), (123457, 201311)]:
        assert mh.mh_encode(i, j, T) == oracle.mh_encode(i, j, T, N)


# ------------------------------------------------------------ classification

def test_classify_against_brute_force():
    g = np.random.default_rng(7)
    for N, T in [(128, 16), (256, 32), (128, 64), (256, 128)]:
        cases = []
        for _ in range(250):
            r, c = (int(v) for v in g.integers(0, N, 2))
            nr = int(g.integers(1, N - r + 1))
            nc = int(g.integers(1, N - c + 1))
            cases.append((r, c, nr, nc))
        # structured: tiles, quadrants, aligned rectangles, tile-sized but shifted blocks
        for e in (T, 2 * T, 4 * T):
            if e <= N:
                cases += [(0, 0, e, e), (e % N, 0, e, e) if 2 * e <= N else (0, 0, e, e),
                          (T, T, e, e) if T + e <= N else (0, 0, e, e),
                          (0, 0, T, e), (1, 1, T - 1, T - 1), (T - 1, T - 1, 2, 2)]
        for r, c, nr, nc in cases:
            s, f = mh.mh_classify_submatrix(N, T, r, c, nr, nc)
            assert s == 0
            assert f == oracle.classify(N, T, r, c, nr, nc), (N, T, r, c, nr, nc)


def test_classify_errors():
    assert mh.mh_classify_submatrix(64, 8, 0, 0, 8, 8)[0] == mh.MH_E_UNSUPPORTED
    assert mh.mh_classify_submatrix(96, 16, 0, 0, 8, 8)[0] == mh.MH_E_SHAPE
    assert mh.mh_classify_submatrix(64, 16, 60, 0, 8, 8)[0] == mh.MH_E_BOUNDS
    assert mh.mh_classify_submatrix(64, 16, 0, 0, 0, 8)[0] == mh.MH_E_INVALID


# --------------------------------------------------------------- validation

def describe(**kw):
    a = dict(NC=256, rc=0, cc=0, NA=256, ra=0, ca=0, NB=256, rb=0, cb=0, m=64, k=64, n=64,
             p=65521, T=32, mode=0)
    a.update(kw)
    return mh.mh_plan_describe(a["NC"], a["rc"], a["cc"], a["NA"], a["ra"], a["ca"], a["NB"],
                               a["rb"], a["cb"], a["m"], a["k"], a["n"], a["p"], a["T"],
                               a["mode"])


def test_validation_codes():
    assert describe()[0] == mh.MH_OK
    assert describe(T=8)[0] == mh.MH_E_UNSUPPORTED
    assert describe(T=256)[0] == mh.MH_E_UNSUPPORTED
    assert describe(NA=96)[0] == mh.MH_E_SHAPE
    assert describe(NC=16)[0] == mh.MH_E_SHAPE
    assert describe(rc=200)[0] == mh.MH_E_BOUNDS
    assert describe(ca=193, k=64)[0] == mh.MH_E_BOUNDS
    assert describe(cb=-1)[0] == mh.MH_E_BOUNDS
    assert describe(p=1)[0] == mh.MH_E_MODULUS
    assert describe(p=2**31)[0] == mh.MH_E_MODULUS
    assert describe(p=2**31 - 1)[0] == mh.MH_OK
    assert describe(m=-1)[0] == mh.MH_E_INVALID
    assert describe(mode=7)[0] == mh.MH_E_UNSUPPORTED
    # the subtract flag combines with every form; other high bits are refused
    for form in (mh.MH_MODE_AUTO, mh.MH_MODE_PLAIN_U32, mh.MH_MODE_LIMB_I8):
        assert describe(mode=form | mh.MH_SUBTRACT)[0] == mh.MH_OK
        assert describe(mode=form | 0x200)[0] == mh.MH_E_UNSUPPORTED


@pytest.mark.parametrize("p", [2, 3, 251, 65521, (1 << 24) - 3, 67108859])
def test_fp64_form_plan_and_reduction_depth(p):
    s, info = describe(p=p, mode=mh.MH_MODE_FP64, m=200, k=150, n=100)
    assert s == mh.MH_OK and info.mode == mh.MH_MODE_FP64
    assert (info.tile_m, info.tile_n) == (128, 128)
    # depth between reductions: a multiple of the MFMA depth 4 whose worst
    # partial sum (p - 1) + depth * H^2 stays within 2^53, and the largest such
    H = 1 if p == 2 else (p - 1) // 2
    d = info.kblock
    assert d % 4 == 0 and d >= 8
    if d < 2**31 - 4:
        assert (p - 1) + d * H * H <= 2**53
        assert (p - 1) + (d + 4) * H * H > 2**53
    if p == 67108859:
        assert d == 8


def test_parent_size():
    for rows, cols, T, N in [(6000, 5000, 64, 8192), (64, 64, 64, 64), (65, 1, 64, 128),
                             (1, 1, 16, 16), (1000, 1000, 32, 1024), (1, 129, 128, 256),
                             (2**18, 7, 128, 2**18)]:
        assert mh.mh_parent_size(rows, cols, T) == (mh.MH_OK, N), (rows, cols, T)
    assert mh.mh_parent_size(0, 5, 64)[0] == mh.MH_E_INVALID
    assert mh.mh_parent_size(5, 5, 8)[0] == mh.MH_E_UNSUPPORTED
    assert mh.mh_parent_size(2**18 + 1, 5, 64)[0] == mh.MH_E_UNSUPPORTED


def test_elementwise_comparator_plan():
    # no planner: output blocks in the product's own coordinates, no packing
    s, info = describe(mode=mh.MH_MODE_PLAIN_ELEMENTWISE, rc=3, cc=5, ra=7, ca=9, rb=11, cb=13,
                       m=130, k=70, n=65)
    assert s == mh.MH_OK and info.mode == mh.MH_MODE_PLAIN_ELEMENTWISE
    assert (info.tile_m, info.tile_n) == (64, 64)
    assert info.gemm_tasks == 3 * 2 and info.pack_chunks == 0


def test_fp64_form_modulus_limit():
    assert describe(p=67108859, mode=mh.MH_MODE_FP64)[0] == mh.MH_OK
    assert describe(p=(1 << 26) + 15, mode=mh.MH_MODE_FP64)[0] == mh.MH_E_MODULUS
    assert describe(p=2**31 - 1, mode=mh.MH_MODE_FP64 | mh.MH_SUBTRACT)[0] == mh.MH_E_MODULUS
    assert describe(p=2**31 - 1, mode=mh.MH_MODE_LIMB_I8)[0] == mh.MH_OK


def test_limbs_and_kblock():
    for p, L in [(2, 1), (251, 1), (256, 1), (257, 2), (65521, 2), (65536, 2), (65537, 3),
                 ((1 << 24) - 3, 3), (2**31 - 1, 4)]:
        s, info = describe(p=p, mode=mh.MH_MODE_LIMB_I8)
        assert s == 0 and info.limbs == L, p
        # |T_s| <= kblock * L * 2^14 must stay below 2^31
        assert info.kblock * L * 2**14 < 2**31 and info.kblock % 64 == 0
        assert (info.kblock + 64) * L * 2**14 >= 2**31


def test_forced_configuration_table(monkeypatch):
    """MH_LIMB_CFG is honoured for every entry of the configuration table
    that fits the limb count, and ignored beyond it; the GPU parity test of
    the configurations covers exactly this table."""
    from tests.test_gpu_limb_configs import NCFG
    big = dict(NC=2048, NA=2048, NB=2048, m=2048, k=2048, n=2048, mode=mh.MH_MODE_LIMB_I8)
    for cfg in range(NCFG + 4):
        monkeypatch.setenv("MH_LIMB_CFG", str(cfg))
        s, info = describe(p=251, **big)
        assert s == 0
        assert (info.kernel_cfg == cfg) == (cfg < NCFG), cfg
    # L = 4 keeps only the configurations whose accumulators fit
    fits4 = set()
    for cfg in range(NCFG):
        monkeypatch.setenv("MH_LIMB_CFG", str(cfg))
        fits4 |= {cfg} if describe(p=2**31 - 1, **big)[1].kernel_cfg == cfg else set()
    assert {0, 1, 2, 4, 6, 7, 9, 10, 11, 12} == fits4


# ------------------------------------------------------------------ planner

def _leaf_count_brute(T, rc, cc, ra, ca, rb, cb, m, k, n):
    rows = {x for x in range(1, m) if (rc + x) % T == 0 or (ra + x) % T == 0}
    inner = {x for x in range(1, k) if (ca + x) % T == 0 or (rb + x) % T == 0}
    cols = {x for x in range(1, n) if (cc + x) % T == 0 or (cb + x) % T == 0}
    return (len(rows) + 1) * (len(inner) + 1) * (len(cols) + 1)


def _random_product(g, T, maxq=3):
    NC, NA, NB = (T * 2 ** int(g.integers(0, maxq + 1)) for _ in range(3))
    m = int(g.integers(1, min(NC, NA) + 1))
    k = int(g.integers(1, min(NA, NB) + 1))
    n = int(g.integers(1, min(NC, NB) + 1))
    rc, cc = int(g.integers(0, NC - m + 1)), int(g.integers(0, NC - n + 1))
    ra, ca = int(g.integers(0, NA - m + 1)), int(g.integers(0, NA - k + 1))
    rb, cb = int(g.integers(0, NB - k + 1)), int(g.integers(0, NB - n + 1))
    return dict(NC=NC, rc=rc, cc=cc, NA=NA, ra=ra, ca=ca, NB=NB, rb=rb, cb=cb, m=m, k=k, n=n)


@pytest.mark.parametrize("seed", range(12))
def test_planner_leaves_match_recursion(seed):
    g = np.random.default_rng(100 + seed)
    T = int(g.choice([16, 32]))
    P = _random_product(g, T, maxq=2)
    args = [P[x] for x in ("NC", "rc", "cc", "NA", "ra", "ca", "NB", "rb", "cb", "m", "k", "n")]
    s, total, leaves = mh.mh_plan_leaves(*args, T, cap=10**6)
    assert s == 0 and total == len(leaves)
    # the recursion of section 2.2 (oracle) reaches exactly as many base cases
    rec = oracle.recursive_mm(None, P["NC"], P["rc"], P["cc"], None, P["NA"], P["ra"], P["ca"],
                              None, P["NB"], P["rb"], P["cb"], P["m"], P["k"], P["n"], 65521, T,
                              count_only=True)
    assert total == rec == _leaf_count_brute(T, P["rc"], P["cc"], P["ra"], P["ca"], P["rb"],
                                             P["cb"], P["m"], P["k"], P["n"])
    # exact partition of the m x k x n product and containment of every piece
    m, k, n = P["m"], P["k"], P["n"]
    if m * k * n <= 4_000_000:
        cover = np.zeros((m, k, n), np.int32)
        for i0, ni, l0, nl, j0, nj in leaves:
            cover[i0:i0 + ni, l0:l0 + nl, j0:j0 + nj] += 1
        assert (cover == 1).all()
    tile = lambda x: x // T
    for i0, ni, l0, nl, j0, nj in leaves:
        for (r0, nr, c0, nc) in ((P["rc"] + i0, ni, P["cc"] + j0, nj),
                                 (P["ra"] + i0, ni, P["ca"] + l0, nl),
                                 (P["rb"] + l0, nl, P["cb"] + j0, nj)):
            assert tile(r0) == tile(r0 + nr - 1) and tile(c0) == tile(c0 + nc - 1)


def test_planner_nonaligned_8192():
    args = (8192, 64, 33, 8192, 1000, 1500, 8192, 517, 2048, 6000, 3000, 5000)
    s, info = mh.mh_plan_describe(*args, 65521, 64, mh.MH_MODE_LIMB_I8)
    assert s == 0
    assert (info.row_segments, info.inner_segments, info.col_segments) == (188, 94, 157)
    assert info.leaves == 188 * 94 * 157 == 2774504
    assert info.c_tiles == 94 * 79
    assert info.limbs == 2


@pytest.mark.parametrize("mode", [mh.MH_MODE_PLAIN_U32, mh.MH_MODE_LIMB_I8])
@pytest.mark.parametrize("seed", range(8))
def test_gemm_tasks_partition_output_in_whole_tiles(mode, seed):
    g = np.random.default_rng(300 + seed)
    T = int(g.choice(TS))
    P = _random_product(g, T, maxq=3)
    args = [P[x] for x in ("NC", "rc", "cc", "NA", "ra", "ca", "NB", "rb", "cb", "m", "k", "n")]
    s, total, tasks = mh.mh_plan_gemm_tasks(*args, 65521, T, mode, cap=10**6)
    assert s == 0 and total == len(tasks)
    m, n = P["m"], P["n"]
    cover = np.zeros((m, n), np.int32)
    for i0, ni, j0, nj in tasks:
        cover[i0:i0 + ni, j0:j0 + nj] += 1
        # each task's C rows either stay in one tile row or run between tile
        # boundaries (or the block's own edges); the same for columns
        for (o, e, lo, hi) in ((P["rc"] + i0, P["rc"] + i0 + ni, P["rc"], P["rc"] + m),
                               (P["cc"] + j0, P["cc"] + j0 + nj, P["cc"], P["cc"] + n)):
            inside_one = o // T == (e - 1) // T
            whole = (o % T == 0 or o == lo) and (e % T == 0 or e == hi)
            assert inside_one or whole
    assert (cover == 1).all()


def _brute_alias(items):
    """The aliasing rule of a batch, pair by pair: an output block may share a
    word with no other output block and no input block; blocks of parents
    whose storage overlaps with another base or edge count as overlapping."""
    def blocks(it):
        return ((it["C"], it["NC"], it["rc"], it["cc"], it["m"], it["n"]),
                (it["A"], it["NA"], it["ra"], it["ca"], it["m"], it["k"]),
                (it["B"], it["NB"], it["rb"], it["cb"], it["k"], it["n"]))

    def alias(x, y):
        (px, nx, rx, cx, hx, wx), (py, ny, ry, cy, hy, wy) = x, y
        if min(hx, wx, hy, wy) <= 0:
            return False
        if px + 4 * nx * nx <= py or py + 4 * ny * ny <= px:
            return False
        if px != py or nx != ny:
            return True
        return rx < ry + hy and ry < rx + hx and cx < cy + wy and cy < cx + wx

    for i, x in enumerate(items):
        cx = blocks(x)[0]
        for j, y in enumerate(items):
            cy, ay, by = blocks(y)
            if (j != i and alias(cx, cy)) or alias(cx, ay) or alias(cx, by):
                return True
    return False


def test_validate_batch_against_pairwise_rule():
    """mh_validate_batch (the checks of a batched call, host only; its
    aliasing test is a sweep per parent) against the rule applied to every
    pair, on random batches over a few parents, some of them placed so that
    their storage overlaps another parent's."""
    g = np.random.default_rng(17)
    T, p = 64, 65521
    for trial in range(300):
        # parents: (base, N); bases are never dereferenced
        base = 1 << 32
        parents = [(base, 1024), (base + 4 * 1024 * 1024, 512), (base + (8 << 20), 1024)]
        if trial % 5 == 0:  # another parent inside the first one's storage
            parents.append((base + 4096 * 16, 256))
        items = []
        # odd trials: outputs in a parent of their own and smaller blocks, so
        # that disjoint batches are as common as overlapping ones
        sep, div = trial % 2 == 1, 2 if trial % 2 == 0 else 8
        for _ in range(int(g.integers(1, 12))):
            def pick(lo=0, hi=len(parents)):
                return parents[int(g.integers(lo, hi))]
            (C, NC) = pick(2, 3) if sep else pick()
            (A, NA), (B, NB) = (pick(0, 2), pick(0, 2)) if sep else (pick(), pick())
            m = int(g.integers(0, min(NC, NA) // div + 1))
            n = int(g.integers(0, min(NC, NB) // div + 1))
            k = int(g.integers(0, min(NA, NB) // div + 1))
            items.append(dict(C=C, NC=NC, A=A, NA=NA, B=B, NB=NB,
                              rc=int(g.integers(0, NC - m + 1)), cc=int(g.integers(0, NC - n + 1)),
                              ra=int(g.integers(0, NA - m + 1)), ca=int(g.integers(0, NA - k + 1)),
                              rb=int(g.integers(0, NB - k + 1)), cb=int(g.integers(0, NB - n + 1)),
                              m=m, k=k, n=n))
        descs = mh.make_descs(items)
        got = mh.mh_validate_batch(descs, len(items), p, T, mh.MH_MODE_LIMB_I8)
        want = mh.MH_E_ALIAS if _brute_alias(items) else mh.MH_OK
        assert got == want, (trial, items)


def test_validate_batch_errors():
    item = dict(C=1 << 32, NC=1024, A=(1 << 32) + (8 << 20), NA=1024, B=(1 << 32) + (8 << 20),
                NB=1024, rc=0, cc=0, ra=0, ca=0, rb=0, cb=0, m=64, k=64, n=64)
    d = mh.make_descs([item])
    assert mh.mh_validate_batch(d, 1, 65521, 64, mh.MH_MODE_LIMB_I8) == mh.MH_OK
    assert mh.mh_validate_batch(d, 1, 2**31 + 1, 64, 2) == mh.MH_E_MODULUS
    assert mh.mh_validate_batch(d, 1, 65521, 48, 2) == mh.MH_E_UNSUPPORTED
    assert mh.mh_validate_batch(d, 1, 1 << 27, 64, mh.MH_MODE_FP64) == mh.MH_E_MODULUS
    assert mh.mh_validate_batch(None, 1, 65521, 64, 2) == mh.MH_E_INVALID
    bad = mh.make_descs([dict(item, rc=1000)])
    assert mh.mh_validate_batch(bad, 1, 65521, 64, 2) == mh.MH_E_BOUNDS
    two = mh.make_descs([item, dict(item, rc=32, cc=32)])
    assert mh.mh_validate_batch(two, 2, 65521, 64, 2) == mh.MH_E_ALIAS
    apart = mh.make_descs([item, dict(item, rc=64)])
    assert mh.mh_validate_batch(apart, 2, 65521, 64, 2) == mh.MH_OK
