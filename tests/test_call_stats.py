"""Table 1's statistic (base-case calls of the modified product over the
default recursion, section 2.2 performance analysis), host only."""

import numpy as np
import pytest

import oracle
from paper_1705_04807_amd import call_stats as cs


def boxes_brute(m, k, n, T):
    """The default recursion as written: a box m x k x n with some side above T
    splits every such side at its midpoint (first half the ceiling) into up to
    eight boxes; count the boxes that split no further."""
    if m <= T and k <= T and n <= T:
        return 1
    cut = lambda d: [(d + 1) // 2, d // 2] if d > T else [d]
    return sum(boxes_brute(a, b, c, T) for a in cut(m) for b in cut(k) for c in cut(n))


@pytest.mark.parametrize("T", [4, 8, 32])
def test_default_count_is_the_box_recursion(T):
    g = np.random.default_rng(T)
    for _ in range(60):
        m, k, n = (int(v) for v in g.integers(1, 9 * T, size=3))
        assert cs.default_calls(m, k, n, T) == boxes_brute(m, k, n, T), (m, k, n)


def test_default_count_closed_forms():
    T = 32
    for a in range(6):
        for b in range(6):
            assert cs.default_calls(T << a, T << b, T, T) == (1 << a) * (1 << b)
    assert cs.default_pieces(3 * T, T) == 4      # 96 -> 48, 48 -> four pieces of 24
    assert cs.default_pieces(T + 1, T) == 2
    assert cs.default_pieces(1, T) == 1


def test_planner_count_equals_the_oracle_recursion():
    g = np.random.default_rng(17)
    for e in cs.draw_experiments(5, 12, N=256, T=16, placement="anywhere", sizes="tiles"):
        got = cs.planner_calls(e["NC"], e["rc"], e["cc"], e["NA"], e["ra"], e["ca"], e["NB"],
                               e["rb"], e["cb"], e["m"], e["k"], e["n"], 16)
        want = oracle.recursive_mm(None, e["NC"], e["rc"], e["cc"], None, e["NA"], e["ra"],
                                   e["ca"], None, e["NB"], e["rb"], e["cb"], e["m"], e["k"],
                                   e["n"], 65521, 16, count_only=True)
        assert got == want, e


def test_whole_tile_blocks_add_no_calls():
    rows = cs.run(cs.draw_experiments(3, 40, placement="tile", sizes="pow2"))
    assert all(a == b for a, b, _ in rows)


def test_one_row_shift_gives_table1_smallest_increase():
    # C and A blocks both start one row below a tile boundary, everything else
    # on tile boundaries: the two row grids coincide, so rows are cut into 33
    # segments instead of 32, i.e. 1/32 = 3.125 % more calls
    N, T = 2048, 32
    a = cs.planner_calls(N, 1, 0, N, 1, 0, N, 0, 0, 1024, 64, 128, T)
    b = cs.default_calls(1024, 64, 128, T)
    assert (a, b) == (33 * 2 * 4, 32 * 2 * 4)
    assert cs.increase_percent(a, b) == pytest.approx(3.125)


def test_table_shares_sum_to_100():
    rows = cs.run(cs.draw_experiments(9, 50))
    tab = cs.table(rows)
    assert sum(s for _, s in tab) == pytest.approx(100.0)
    assert [i for i, _ in tab] == sorted(i for i, _ in tab)
    assert min(i for i, _ in tab) >= 0.0   # never fewer calls than the default on pow2 sizes


def test_misaligned_grids_double_the_rows():
    # C one row below a boundary, A on one: the two row grids interleave and
    # every tile row splits in two (31 + 1), i.e. 100 % more calls
    N, T = 2048, 32
    a = cs.planner_calls(N, 1, 0, N, 0, 0, N, 0, 0, 1024, 64, 128, T)
    assert a == 2 * cs.default_calls(1024, 64, 128, T)
