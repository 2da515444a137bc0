"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something other than its own code:
exact library arithmetic (numpy on int64 / Python integers), closed forms,
special cases (GF(2), identity, zero), invariants (associativity, the
Step 1/Step 2 offsets of section 2.2), hand-derived golden vectors and brute
force on tiny inputs.
"""

import itertools
import os

import numpy as np
import pytest

import oracle
from seeded_inputs import residues_np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PRIMES = [2, 3, 5, 251, 65521, 2147483647]


def exact_product(C, A, B, p):
    """(C + A @ B) mod p with Python integers (numpy object arrays): exact for any size."""
    Ao = A.astype(object)
    Bo = B.astype(object)
    return ((C.astype(object) + Ao.dot(Bo)) % p).astype(np.uint32)


def rnd(seed, p, r, c):
    return residues_np(seed, p, r, c)


# ---------------------------------------------------------------- products

@pytest.mark.parametrize("p", PRIMES)
def test_matmul_all_small_shapes_against_exact_integers(oracle_lib, p):
    # every m, k, n <= 6 (k = 0 included), against numpy's exact object-dtype dot
    seed = 7
    for m, k, n in itertools.product(range(1, 7), range(0, 7), range(1, 7)):
        seed += 1
        A = rnd(seed, p, m, k) if k else np.zeros((m, 0), np.uint32)
        B = rnd(seed + 10**6, p, k, n) if k else np.zeros((0, n), np.uint32)
        C = rnd(seed + 2 * 10**6, p, m, n)
        want = exact_product(C, A, B, p) if k else C.copy()
        got = C.copy()
        oracle.matmul_modp(got, np.ascontiguousarray(A), np.ascontiguousarray(B), p)
        assert np.array_equal(got, want), (m, k, n)


@pytest.mark.parametrize("p,m,k,n", [(65521, 37, 300, 41), (2147483647, 23, 129, 31),
                                     (2147483647, 5, 2000, 3)])
def test_matmul_rectangular_against_library(oracle_lib, p, m, k, n):
    A, B, C = rnd(11, p, m, k), rnd(12, p, k, n), rnd(13, p, m, n)
    got = C.copy()
    oracle.matmul_modp(got, A, B, p)
    if p < 2**16:  # products < 2^32 and k < 2^31: int64 matmul is exact
        want = ((C.astype(np.int64) + A.astype(np.int64) @ B.astype(np.int64)) % p)
        assert np.array_equal(got, want.astype(np.uint32))
    assert np.array_equal(got, exact_product(C, A, B, p))


def test_matmul_gf2_is_and_xor(oracle_lib):
    # Over the binary field (the paper's experiments) the product is AND / XOR.
    m, k, n = 19, 33, 17
    A, B, C = rnd(21, 2, m, k), rnd(22, 2, k, n), rnd(23, 2, m, n)
    want = C ^ np.bitwise_xor.reduce(A[:, :, None] & B[None, :, :], axis=1)
    got = C.copy()
    oracle.matmul_modp(got, A, B, 2)
    assert np.array_equal(got, want.astype(np.uint32))


@pytest.mark.parametrize("p", [65521, 2147483647])
def test_matmul_identity_and_zero(oracle_lib, p):
    n = 24
    A = rnd(31, p, n, n)
    I = np.eye(n, dtype=np.uint32)
    Z = np.zeros((n, n), np.uint32)
    got = Z.copy()
    oracle.matmul_modp(got, A, I, p)          # 0 + A.I = A
    assert np.array_equal(got, A)
    got = Z.copy()
    oracle.matmul_modp(got, I, A, p)          # 0 + I.A = A
    assert np.array_equal(got, A)
    C = rnd(32, p, n, n)
    got = C.copy()
    oracle.matmul_modp(got, A, Z, p)          # C + A.0 = C
    assert np.array_equal(got, C)


@pytest.mark.parametrize("p", [65521, 2147483647])
def test_matmul_associativity(oracle_lib, p):
    # (AB)C = A(BC) mod p; a transposed operand or a dropped term breaks it
    A, B, Cm = rnd(41, p, 13, 29), rnd(42, p, 29, 11), rnd(43, p, 11, 17)
    Z = lambda r, c: np.zeros((r, c), np.uint32)
    AB = Z(13, 11); oracle.matmul_modp(AB, A, B, p)
    BC = Z(29, 17); oracle.matmul_modp(BC, B, Cm, p)
    L = Z(13, 17); oracle.matmul_modp(L, AB, Cm, p)
    R = Z(13, 17); oracle.matmul_modp(R, A, BC, p)
    assert np.array_equal(L, R)


def test_matmul_view_matches_subarray(oracle_lib):
    p = 65521
    A, B, C = rnd(51, p, 40, 40), rnd(52, p, 40, 40), rnd(53, p, 40, 40)
    want = C.copy()
    sub = want[3:3 + 7, 5:5 + 9].copy()
    oracle.matmul_modp(sub, np.ascontiguousarray(A[10:17, 1:12]),
                       np.ascontiguousarray(B[20:31, 30:39]), p)
    want[3:10, 5:14] = sub
    got = C.copy()
    oracle.matmul_modp_view(got, A, B, p, 3, 5, 10, 1, 20, 30, 7, 11, 9)
    assert np.array_equal(got, want)


def test_entries_match_full_product(oracle_lib):
    p = 2147483647
    A, B, C = rnd(61, p, 30, 50), rnd(62, p, 50, 20), rnd(63, p, 30, 20)
    full = exact_product(C, A, B, p)
    rows = np.array([0, 29, 7, 13, 29])
    cols = np.array([0, 19, 3, 0, 0])
    got = oracle.matmul_modp_entries(rows, cols, C, A, B, p)
    assert np.array_equal(got, full[rows, cols])


def test_freivalds_accepts_and_rejects(oracle_lib):
    p = 65521
    A, B, C = rnd(71, p, 20, 30), rnd(72, p, 30, 25), rnd(73, p, 20, 25)
    good = exact_product(C, A, B, p)
    x = rnd(74, p, 1, 25)[0]
    assert oracle.freivalds(good, C, A, B, p, x)
    bad = good.copy()
    bad[4, 7] = (bad[4, 7] + 1) % p
    assert not oracle.freivalds(bad, C, A, B, p, x)


# ---------------------------------------------------------------- index

def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([int(v) for v in line.split()])
    return rows


def test_encoder_golden_vectors(oracle_lib):
    for i, j, T, N, z in _golden_rows("mh_index_vectors.txt"):
        assert oracle.mh_encode(i, j, T, N) == z, (i, j, T, N)
        assert oracle.mh_extract(z, T, N) == (i, j)


def _interleave_textbook(i, j, bits):
    # Morton code from binary strings: row bit before column bit, most significant first
    bi, bj = format(i, "0%db" % bits), format(j, "0%db" % bits)
    return int("".join(a + b for a, b in zip(bi, bj)), 2)


@pytest.mark.parametrize("N,T", [(8, 1), (16, 2), (16, 4), (32, 8), (16, 16), (64, 4)])
def test_encoder_bijection_and_closed_forms(oracle_lib, N, T):
    zs = set()
    for i in range(N):
        for j in range(N):
            z = oracle.mh_encode(i, j, T, N)
            zs.add(z)
            assert oracle.mh_extract(z, T, N) == (i, j)
            # independent of the parent size (the Z order of 2^q x 2^q grids nests)
            assert oracle.mh_encode(i, j, T, 2 * N) == z
            # Prop. 2.5: row-major inside the tile, offset from the tile's first index
            sigma = oracle.mh_encode(i - i % T, j - j % T, T, N)
            assert z == sigma + (i % T) * T + (j % T)
            assert sigma % (T * T) == 0
            # tile order is the textbook bit interleave of the tile coordinates
            q = max(1, (N // T - 1).bit_length())
            assert sigma // (T * T) == _interleave_textbook(i // T, j // T, q)
    assert zs == set(range(N * N))
    if T == N:  # no recursion: plain row-major
        assert all(oracle.mh_encode(i, j, T, N) == i * N + j for i in range(N) for j in range(N))


@pytest.mark.parametrize("N,T", [(8, 2), (32, 4), (64, 8)])
def test_step1_step2_offsets(oracle_lib, N, T):
    # Every block of the quadrant recursion: quadrant starts alpha + t lambda/4 and
    # the last entries e_NE = alpha + 2 lambda' - 1, e_SW = alpha + 3 lambda' - 1.
    def walk(r0, c0, edge):
        if edge <= T:
            return
        alpha = oracle.mh_encode(r0, c0, T, N)
        lam = edge * edge
        h = edge // 2
        lq = lam // 4
        starts = [oracle.mh_encode(r0 + (t >> 1) * h, c0 + (t & 1) * h, T, N) for t in range(4)]
        assert starts == [alpha + t * lq for t in range(4)]
        assert oracle.mh_encode(r0 + h - 1, c0 + edge - 1, T, N) == alpha + 2 * lq - 1
        assert oracle.mh_encode(r0 + edge - 1, c0 + h - 1, T, N) == alpha + 3 * lq - 1
        # the block occupies exactly [alpha, alpha + lambda)
        zs = {oracle.mh_encode(r0 + a, c0 + b, T, N) for a in range(edge) for b in range(edge)}
        assert zs == set(range(alpha, alpha + lam))
        for t in range(4):
            walk(r0 + (t >> 1) * h, c0 + (t & 1) * h, h)
    walk(0, 0, N)


@pytest.mark.parametrize("N,T", [(16, 4), (32, 8), (8, 1), (64, 64)])
def test_layout_conversion_against_reshape(oracle_lib, N, T):
    X = rnd(81, 2**31 - 1, N, N)
    mh = oracle.mh_from_cartesian(X, T)
    # independent construction: cut into tiles, order tiles by Z, flatten each row-major
    q = N // T
    tiles = X.reshape(q, T, q, T).transpose(0, 2, 1, 3)
    bits = max(1, (q - 1).bit_length())
    order = sorted(((_interleave_textbook(I, J, bits), I, J) for I in range(q) for J in range(q)))
    want = np.concatenate([tiles[I, J].reshape(-1) for _, I, J in order])
    assert np.array_equal(mh, want)
    assert np.array_equal(oracle.mh_to_cartesian(mh, N, T), X)


# ---------------------------------------------------------------- classifier

def test_classify_golden(oracle_lib):
    for N, T, r, c, nr, nc, flags in _golden_rows("classify_cases.txt"):
        assert oracle.classify(N, T, r, c, nr, nc) == flags, (r, c, nr, nc)


def test_classify_all_blocks_rules(oracle_lib):
    # Every placement in a 16x16 parent with T = 4 against the rules read off the
    # definitions (tile-start and 2^a T sizes; one tile; recursion node).
    N, T = 16, 4
    for r in range(N):
        for c in range(N):
            for nr in range(1, N - r + 1):
                for nc in range(1, N - c + 1):
                    f = oracle.classify(N, T, r, c, nr, nc)
                    pw = lambda x: x % T == 0 and ((x // T) & (x // T - 1)) == 0
                    al = r % T == 0 and c % T == 0 and pw(nr) and pw(nc)
                    co = r // T == (r + nr - 1) // T and c // T == (c + nc - 1) // T
                    qu = nr == nc and pw(nr) and r % nr == 0 and c % nc == 0
                    assert f == (al * 1 | co * 2 | qu * 4), (r, c, nr, nc, f)


# ---------------------------------------------------------------- recursion

def _segments(m, cuts):
    return len({x for x in cuts if 0 < x < m}) + 1


def _leaf_count(T, rc, cc, ra, ca, rb, cb, m, k, n):
    # leaves of the product: the union grid of the three operands' tile cuts
    rows = [x for x in range(1, m) if (rc + x) % T == 0 or (ra + x) % T == 0]
    inner = [x for x in range(1, k) if (ca + x) % T == 0 or (rb + x) % T == 0]
    cols = [x for x in range(1, n) if (cc + x) % T == 0 or (cb + x) % T == 0]
    return _segments(m, rows) * _segments(k, inner) * _segments(n, cols)


@pytest.mark.parametrize("case", range(40))
def test_recursive_mm_matches_definition(oracle_lib, case):
    g = np.random.default_rng(1000 + case)
    T = int(g.choice([1, 2, 4, 8]))
    p = int(g.choice([2, 251, 65521, 2147483647]))
    NC, NA, NB = (T * 2 ** int(g.integers(0, 4 if T > 1 else 5)) for _ in range(3))
    m = int(g.integers(1, min(NC, NA) + 1))
    k = int(g.integers(1, min(NA, NB) + 1))
    n = int(g.integers(1, min(NC, NB) + 1))
    rc, cc = int(g.integers(0, NC - m + 1)), int(g.integers(0, NC - n + 1))
    ra, ca = int(g.integers(0, NA - m + 1)), int(g.integers(0, NA - k + 1))
    rb, cb = int(g.integers(0, NB - k + 1)), int(g.integers(0, NB - n + 1))
    A, B, C = rnd(90 + case, p, NA, NA), rnd(190 + case, p, NB, NB), rnd(290 + case, p, NC, NC)
    want = C.copy()
    oracle.matmul_modp_view(want, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n)
    Cm = oracle.mh_from_cartesian(C, T)
    leaves = oracle.recursive_mm(Cm, NC, rc, cc, oracle.mh_from_cartesian(A, T), NA, ra, ca,
                                 oracle.mh_from_cartesian(B, T), NB, rb, cb, m, k, n, p, T)
    assert np.array_equal(oracle.mh_to_cartesian(Cm, NC, T), want)
    assert leaves == _leaf_count(T, rc, cc, ra, ca, rb, cb, m, k, n)


def test_recursive_mm_aligned_leaf_count(oracle_lib):
    # aligned whole parents: every leaf is a whole tile triple, (N/T)^3 of them
    for N, T in [(64, 8), (128, 32), (256, 32)]:
        assert oracle.recursive_mm(None, N, 0, 0, None, N, 0, 0, None, N, 0, 0, N, N, N,
                                   65521, T, count_only=True) == (N // T) ** 3


def test_recursive_mm_nonaligned_8192_leaf_count(oracle_lib):
    # A 6000x3000 @ (1000,1500), B 3000x5000 @ (517,2048), C 6000x5000 @ (64,33), T = 64
    args = (8192, 64, 33, None, 8192, 1000, 1500, None, 8192, 517, 2048, 6000, 3000, 5000)
    got = oracle.recursive_mm(None, *args[:3], None, *args[4:7], None, *args[8:11],
                              *args[11:], 65521, 64, count_only=True)
    assert got == _leaf_count(64, 64, 33, 1000, 1500, 517, 2048, 6000, 3000, 5000)
    assert got == 188 * 94 * 157


# ---------------------------------------------------------------- limb digits

def _check_digits(x, p, L):
    d, ok = oracle.limb_digits(x, p, L)
    assert ok
    assert all(-128 <= v <= 127 for v in d)
    val = sum(v * 256 ** t for t, v in enumerate(d))
    assert (val - x) % p == 0
    H = 127 * (256 ** L - 1) // 255
    assert val == (x if x <= H else x - p)


def test_limb_digits_exhaustive_65521(oracle_lib):
    p = 65521
    for x in range(0, p, 1):
        _check_digits(x, p, 2)


def test_limb_digits_2p31(oracle_lib):
    p = 2**31 - 1
    H = 127 * (256 ** 4 - 1) // 255
    xs = [0, 1, 127, 128, 255, 256, H - 1, H, H + 1, p - 1, p - 2, 2**31 - 256, 0x80808080 % p]
    xs += [int(v) for v in rnd(99, p, 1, 2000)[0]]
    for x in xs:
        _check_digits(x, p, 4)


def test_limb_digits_need_enough_limbs(oracle_lib):
    # two digits represent the centred window [-32896, 32639]: 65537 > 2^16 does not fit
    _, ok = oracle.limb_digits(32640, 65537, 2)
    assert not ok


# ---------------------------------------------------------------- subtraction

@pytest.mark.parametrize("p", [2, 251, 65521, 2147483647])
def test_subtractive_update(oracle_lib, p):
    A, B, C = rnd(201, p, 17, 40), rnd(202, p, 40, 23), rnd(203, p, 17, 23)
    got = C.copy()
    oracle.matmul_modp_sub(got, A, B, p)
    want = ((C.astype(object) - A.astype(object).dot(B.astype(object))) % p).astype(np.uint32)
    assert np.array_equal(got, want)
    oracle.matmul_modp(got, A, B, p)  # adding the product back restores C
    assert np.array_equal(got, C)
    if p == 2:  # over GF(2) subtraction is addition
        add = C.copy()
        oracle.matmul_modp(add, A, B, p)
        sub = C.copy()
        oracle.matmul_modp_sub(sub, A, B, p)
        assert np.array_equal(add, sub)
