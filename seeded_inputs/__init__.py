"""Seeded synthetic inputs shared by the tests, the bench and the oracle's callers.

This module holds no arithmetic of the method (no products, no reductions
of products, no layout code): it only turns a seed and a counter into a
residue, so that the HIP path and the CPU oracle can be fed identical
matrices without either importing the other.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written from its published
definition.  Output number ``c`` (c = 0, 1, 2, ...) of the generator seeded
with ``s`` is ``mix(s + (c + 1) * GAMMA)`` where ``mix`` is the published
variant-13 finaliser.  Being a pure function of the counter, any element of
any matrix can be regenerated on its own (the tests use that to rebuild
single rows and columns of 8192 x 8192 parents without holding them).

A matrix entry at Cartesian position (i, j) of a parent with row length
``ld`` uses counter ``i * ld + j``; the value is the 64-bit output reduced
mod p, whose bias from exact uniformity is below p / 2**64 <= 2**-33.
Values are generated in Cartesian order, so they do not depend on the
storage layout.

Two implementations are provided and tested to agree bit for bit: numpy
on the host, and torch int64 tensors (host or device) for large parents.
"""

from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# Seeds of the standard workloads: 1000 * workload + operand (A=1, B=2, C=3).
A_OP, B_OP, C_OP = 1, 2, 3


def workload_seed(workload: int, operand: int) -> int:
    return 1000 * workload + operand


def splitmix64_scalar(seed: int, counter: int) -> int:
    """Output number ``counter`` of SplitMix64 seeded with ``seed`` (pure Python)."""
    z = (seed + (counter + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_np(seed: int, counters: np.ndarray) -> np.ndarray:
    """Vectorised SplitMix64 outputs for an array of counters (uint64, wrapping)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + (c + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def residues_np(seed: int, p: int, rows: int, cols: int, ld: int | None = None,
                row0: int = 0, col0: int = 0) -> np.ndarray:
    """uint32 array [rows, cols] holding entries (row0+i, col0+j) of the seeded parent.

    ``ld`` is the row length of the parent the counters refer to (default: cols).
    """
    ld = cols if ld is None else ld
    out = np.empty((rows, cols), dtype=np.uint32)
    jj = np.arange(col0, col0 + cols, dtype=np.uint64)
    # row blocks keep temporaries near 64 MB
    step = max(1, (1 << 23) // max(cols, 1))
    for r in range(0, rows, step):
        re = min(rows, r + step)
        ii = np.arange(row0 + r, row0 + re, dtype=np.uint64)[:, None]
        with np.errstate(over="ignore"):
            ctr = ii * np.uint64(ld) + jj[None, :]
        out[r:re] = (splitmix64_np(seed, ctr) % np.uint64(p)).astype(np.uint32)
    return out


def _lsr(x, s: int):
    """Logical right shift of a torch int64 tensor."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def _wrap64(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def residues_torch(seed: int, p: int, rows: int, cols: int, ld: int | None = None,
                   device="cpu", row0: int = 0, col0: int = 0):
    """Same values as :func:`residues_np`, as a torch int32 tensor holding uint32 bits.

    Uses int64 tensors with two's-complement wrap-around for the 64-bit
    SplitMix64 state; the reduction mod p of an unsigned 64-bit value is done
    from its two 32-bit halves so that no intermediate exceeds 2**63.
    """
    import torch

    ld = cols if ld is None else ld
    out = torch.empty((rows, cols), dtype=torch.int32, device=device)
    jj = torch.arange(col0, col0 + cols, dtype=torch.int64, device=device)
    two32_mod_p = (1 << 32) % p
    step = max(1, (1 << 24) // max(cols, 1))
    for r in range(0, rows, step):
        re = min(rows, r + step)
        ii = torch.arange(row0 + r, row0 + re, dtype=torch.int64, device=device)[:, None]
        c = ii * ld + jj[None, :]
        z = (c + 1) * _wrap64(GAMMA) + _wrap64(seed)
        z = (z ^ _lsr(z, 30)) * _wrap64(M1)
        z = (z ^ _lsr(z, 27)) * _wrap64(M2)
        z = z ^ _lsr(z, 31)
        hi = _lsr(z, 32)
        lo = z & 0xFFFFFFFF
        v = ((hi % p) * two32_mod_p + lo) % p
        out[r:re] = v.to(torch.int32)  # values < 2**31 for p <= 2**31 - 1
    return out


def residues_scalar(seed: int, p: int, i: int, j: int, ld: int) -> int:
    return splitmix64_scalar(seed, i * ld + j) % p


def tu_level_batch(seed: int = 5000, count: int = 512, N: int = 8192, n_c_parents: int = 64,
                   unit: int = 64, max_units: int = 32):
    """Shapes and offsets of `count` independent products of one TU recursion level.

    For each product and each of m, k, n independently: size = unit * u + r
    with u uniform in 1..max_units and r uniform in 1..unit-1.  A and B
    blocks lie anywhere in one shared N x N parent each (read-only overlap
    allowed); product i writes C parent i mod n_c_parents, its C offset
    redrawn until disjoint from the earlier blocks of that parent.  Draws
    come from SplitMix64 seeded with `seed`, in a fixed order.
    """
    ctr = [0]

    def draw(lo: int, hi: int) -> int:  # uniform integer in [lo, hi]
        v = splitmix64_scalar(seed, ctr[0])
        ctr[0] += 1
        return lo + v % (hi - lo + 1)

    used = [[] for _ in range(n_c_parents)]
    calls = []
    for i in range(count):
        m, k, n = (unit * draw(1, max_units) + draw(1, unit - 1) for _ in range(3))
        ci = i % n_c_parents
        while True:
            rc, cc = draw(0, N - m), draw(0, N - n)
            if all(rc + m <= r or r + mm <= rc or cc + n <= c or c + nn <= cc
                   for r, c, mm, nn in used[ci]):
                break
        used[ci].append((rc, cc, m, n))
        calls.append(dict(ci=ci, rc=rc, cc=cc, m=m, k=k, n=n, ra=draw(0, N - m),
                          ca=draw(0, N - k), rb=draw(0, N - k), cb=draw(0, N - n)))
    return calls
