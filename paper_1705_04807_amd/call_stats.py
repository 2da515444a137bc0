"""Base-case call counts of the Morton-hybrid sub-matrix product against the
default recursion (the statistic of Table 1, section 2.2 performance analysis).

The paper multiplies random sub-matrices of N = 2048 Morton-hybrid parents
with T' = 32 and reports, per experiment, the percentage by which the
modified algorithm's base-case calls exceed those of the default recursive
algorithm.  Here:

* the modified algorithm's count is the planner's leaf count
  (``mh_plan_describe(...).leaves``): the base cases of the recursion of
  section 2.2 (Steps 1-4), each a product of contained pieces;
* the default algorithm is the plain divide-and-conquer product on the
  sub-matrix dimensions, with this rule (the paper does not print one):
  every dimension of the product m x k x n that exceeds T' is cut at its
  midpoint (first half ceil(d/2)), dimensions of at most T' are kept whole,
  and the recursion stops when all three are at most T'.  Its count is the
  product over the three dimensions of the pieces one dimension is cut into.

Only host code runs (the planner is host-side); no GPU is needed.
"""

from __future__ import annotations

import argparse
import collections
import functools
import json

import numpy as np

from . import MH_MODE_LIMB_I8, MH_OK, mh_plan_describe


@functools.lru_cache(maxsize=None)
def default_pieces(d: int, T: int) -> int:
    """Pieces of one dimension under the default rule: halve while above T."""
    if d <= T:
        return 1
    return default_pieces((d + 1) // 2, T) + default_pieces(d // 2, T)


def default_calls(m: int, k: int, n: int, T: int) -> int:
    return default_pieces(m, T) * default_pieces(k, T) * default_pieces(n, T)


def planner_calls(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, T) -> int:
    s, info = mh_plan_describe(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, 65521, T,
                               MH_MODE_LIMB_I8)
    if s != MH_OK:
        raise ValueError("planner rejected the product (status %d)" % s)
    return int(info.leaves)


def increase_percent(mh_calls: int, default: int) -> float:
    return 100.0 * (mh_calls - default) / default


PLACEMENTS = ("anywhere", "tile", "mixed")
SIZES = ("pow2", "tiles")


def draw_experiments(seed: int, count: int, N: int = 2048, T: int = 32,
                     placement: str = "mixed", sizes: str = "pow2"):
    """Random products S_C += S_A . S_B on N x N parents.

    Each dimension is a whole number of tiles (the paper's ratios imply it):
    T' times a power of two from 1 to N/(2T') ("pow2", where the default rule
    cuts exact tiles) or T' times any integer in that range ("tiles").  Each
    starting row and column is drawn uniformly from the positions that keep
    the block inside its parent: any position ("anywhere", so blocks are
    usually scattered), tile boundaries only ("tile": unions of whole tiles),
    or, per coordinate with even odds, one or the other ("mixed")."""
    if placement not in PLACEMENTS:
        raise ValueError("placement must be one of %s" % (PLACEMENTS,))
    if sizes not in SIZES:
        raise ValueError("sizes must be one of %s" % (SIZES,))
    g = np.random.default_rng(seed)
    umax = N // (2 * T)

    def dim():
        if sizes == "pow2":
            return T << int(g.integers(0, umax.bit_length()))
        return T * int(g.integers(1, umax + 1))

    def start(d):
        on_tiles = placement == "tile" or (placement == "mixed" and g.integers(0, 2) == 0)
        step = T if on_tiles else 1
        return step * int(g.integers(0, (N - d) // step + 1))

    out = []
    for _ in range(count):
        m, k, n = dim(), dim(), dim()
        out.append(dict(NC=N, NA=N, NB=N, m=m, k=k, n=n, rc=start(m), cc=start(n),
                        ra=start(m), ca=start(k), rb=start(k), cb=start(n)))
    return out


def run(experiments, T: int = 32):
    """Per experiment: (planner calls, default calls, % increase)."""
    rows = []
    for e in experiments:
        a = planner_calls(e["NC"], e["rc"], e["cc"], e["NA"], e["ra"], e["ca"], e["NB"],
                          e["rb"], e["cb"], e["m"], e["k"], e["n"], T)
        b = default_calls(e["m"], e["k"], e["n"], T)
        rows.append((a, b, increase_percent(a, b)))
    return rows


def table(rows, decimals: int = 2):
    """Table 1's first two columns: distinct % increases and the share of
    experiments showing each, sorted by increase."""
    hist = collections.Counter(round(r[2], decimals) for r in rows)
    n = max(len(rows), 1)
    return [(inc, 100.0 * c / n) for inc, c in sorted(hist.items())]


def summary(rows):
    inc = np.array([r[2] for r in rows], dtype=np.float64)
    return dict(experiments=len(rows), mean_increase=float(inc.mean()) if len(inc) else 0.0,
                median_increase=float(np.median(inc)) if len(inc) else 0.0,
                max_increase=float(inc.max()) if len(inc) else 0.0,
                min_increase=float(inc.min()) if len(inc) else 0.0,
                distinct=len(set(np.round(inc, 2))))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--experiments", type=int, default=468)
    ap.add_argument("--seed", type=int, default=1705)
    ap.add_argument("--N", type=int, default=2048)
    ap.add_argument("--T", type=int, default=32)
    ap.add_argument("--placement", choices=PLACEMENTS, default="mixed")
    ap.add_argument("--sizes", choices=SIZES, default="pow2")
    ap.add_argument("--top", type=int, default=25, help="rows of the histogram to print")
    ap.add_argument("--json", action="store_true")
    a = ap.parse_args(argv)
    rows = run(draw_experiments(a.seed, a.experiments, a.N, a.T, a.placement, a.sizes), a.T)
    tab = table(rows)
    if a.json:
        print(json.dumps(dict(summary=summary(rows), table=tab)))
        return
    print("%% increase in base-case calls  |  %% of experiments   (N=%d, T'=%d, %d experiments,"
          " placement %s, sizes %s)" % (a.N, a.T, len(rows), a.placement, a.sizes))
    for inc, share in sorted(tab, key=lambda t: -t[1])[:a.top]:
        print("%10.2f  |  %5.1f" % (inc, share))
    print(json.dumps(summary(rows)))


if __name__ == "__main__":
    main()
