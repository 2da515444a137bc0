"""CPU oracle for C := C + A.B mod p on Morton-hybrid operands.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the bench's CPU
baseline leg may use it; the product library never does.  It shares no code
with the HIP path.  The arithmetic lives in ``mh_oracle.c`` (plain C,
OpenMP); this module compiles it with gcc on first use and wraps it with
ctypes over numpy arrays.

Functions with no pin of their own: none (every routine here is checked
against brute force, closed forms or library routines in tests/).
"""

from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# MH_SANITIZE=1: the AddressSanitizer / UndefinedBehaviorSanitizer build of
# build_sanitized.py, for host-only sanitizer runs of the CPU tests.
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")

ALIGNED, CONTAINED, QUADRANT = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (always when ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if os.environ.get("MH_SANITIZE") == "1":
            if not os.path.exists(_LIB_SAN):
                raise ImportError("MH_SANITIZE=1 but oracle/liboracle_san.so is not built "
                                  "(python oracle/build_sanitized.py)")
            L = ct.CDLL(_LIB_SAN)
        else:
            if not os.path.exists(_LIB):
                build()
            L = ct.CDLL(_LIB)
        P = ct.c_void_p
        I64 = ct.c_int64
        U32 = ct.c_uint32
        U64 = ct.c_uint64
        L.oracle_matmul_modp.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, U32, ct.c_int]
        L.oracle_matmul_modp.restype = None
        L.oracle_matmul_modp_sub.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, U32, ct.c_int]
        L.oracle_matmul_modp_sub.restype = None
        L.oracle_matmul_modp_entries.argtypes = [P, P, P, I64, P, I64, P, I64, P, I64, I64,
                                                 U32, ct.c_int]
        L.oracle_matmul_modp_entries.restype = None
        L.oracle_freivalds.argtypes = [P, P, I64, P, I64, P, I64, I64, I64, I64, U32, P,
                                       ct.c_int]
        L.oracle_freivalds.restype = ct.c_int
        L.oracle_mh_encode.argtypes = [U64, U64, U64, U64]
        L.oracle_mh_encode.restype = U64
        L.oracle_mh_extract.argtypes = [U64, U64, U64, ct.POINTER(U64), ct.POINTER(U64)]
        L.oracle_mh_extract.restype = None
        L.oracle_mh_from_cartesian.argtypes = [P, P, I64, I64, I64]
        L.oracle_mh_from_cartesian.restype = None
        L.oracle_mh_to_cartesian.argtypes = [P, I64, P, I64, I64]
        L.oracle_mh_to_cartesian.restype = None
        L.oracle_classify.argtypes = [I64, I64, I64, I64, I64, I64]
        L.oracle_classify.restype = U32
        L.oracle_recursive_mm.argtypes = [P, I64, I64, I64, P, I64, I64, I64, P, I64, I64, I64,
                                          I64, I64, I64, U32, I64, ct.c_int]
        L.oracle_recursive_mm.restype = U64
        L.oracle_limb_digits.argtypes = [U32, U32, ct.c_int, P]
        L.oracle_limb_digits.restype = ct.c_int
        _lib = L
    return _lib


def _u32(a: np.ndarray) -> np.ndarray:
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"], "uint32 C-contiguous array expected"
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def matmul_modp(C: np.ndarray, A: np.ndarray, B: np.ndarray, p: int,
                nthreads: int | None = None) -> None:
    """In place: C <- (C + A @ B) mod p on 2-D uint32 arrays (the definition)."""
    _u32(C), _u32(A), _u32(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2 and C.shape == (m, n)
    lib().oracle_matmul_modp(_ptr(C), n, _ptr(A), k, _ptr(B), n, m, k, n, p,
                             nthreads or default_threads())


def matmul_modp_sub(C: np.ndarray, A: np.ndarray, B: np.ndarray, p: int,
                    nthreads: int | None = None) -> None:
    """In place: C <- (C - A @ B) mod p on 2-D uint32 arrays."""
    _u32(C), _u32(A), _u32(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2 and C.shape == (m, n)
    lib().oracle_matmul_modp_sub(_ptr(C), n, _ptr(A), k, _ptr(B), n, m, k, n, p,
                                 nthreads or default_threads())


def matmul_modp_view(C: np.ndarray, A: np.ndarray, B: np.ndarray, p: int,
                     rc: int, cc: int, ra: int, ca: int, rb: int, cb: int,
                     m: int, k: int, n: int, nthreads: int | None = None,
                     subtract: bool = False) -> None:
    """In place on whole Cartesian parents: C[rc:rc+m, cc:cc+n] += A[ra.., ca..] B[rb.., cb..]
    (or -= with subtract)."""
    _u32(C), _u32(A), _u32(B)
    if m <= 0 or n <= 0:
        return
    ldc, lda, ldb = C.shape[1], A.shape[1], B.shape[1]
    assert rc + m <= C.shape[0] and cc + n <= ldc
    assert ra + m <= A.shape[0] and ca + k <= lda
    assert rb + k <= B.shape[0] and cb + n <= ldb
    base = lambda X, r, c, ld: ct.c_void_p(X.ctypes.data + 4 * (r * ld + c))
    fn = lib().oracle_matmul_modp_sub if subtract else lib().oracle_matmul_modp
    fn(base(C, rc, cc, ldc), ldc, base(A, ra, ca, lda), lda, base(B, rb, cb, ldb), ldb, m, k, n,
       p, nthreads or default_threads())


def matmul_modp_entries(rows, cols, C: np.ndarray, A: np.ndarray, B: np.ndarray, p: int,
                        nthreads: int | None = None) -> np.ndarray:
    """(C + A @ B) mod p at the listed (row, col) entries only; C is not modified.

    A is m x k and B is k x n (any uint32 2-D arrays, C-contiguous)."""
    _u32(C), _u32(A), _u32(B)
    ri = np.ascontiguousarray(rows, dtype=np.int64)
    cj = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(ri.shape[0], dtype=np.uint32)
    k = A.shape[1]
    assert B.shape[0] == k
    lib().oracle_matmul_modp_entries(_ptr(out), _ptr(ri), _ptr(cj), ri.shape[0], _ptr(C),
                                     C.shape[1], _ptr(A), A.shape[1], _ptr(B), B.shape[1], k,
                                     p, nthreads or default_threads())
    return out


def freivalds(Cnew, Cold, A, B, p: int, x: np.ndarray, nthreads: int | None = None) -> bool:
    """True if Cnew.x == Cold.x + A.(B.x) mod p for the given residue vector x."""
    for a in (Cnew, Cold, A, B):
        _u32(a)
    x = _u32(np.ascontiguousarray(x, dtype=np.uint32))
    m, k = A.shape
    n = B.shape[1]
    return bool(lib().oracle_freivalds(_ptr(Cnew), _ptr(Cold), n, _ptr(A), k, _ptr(B), n,
                                       m, k, n, p, _ptr(x), nthreads or default_threads()))


def mh_encode(i: int, j: int, T: int, N: int) -> int:
    return int(lib().oracle_mh_encode(i, j, T, N))


def mh_extract(z: int, T: int, N: int) -> tuple[int, int]:
    i, j = ct.c_uint64(), ct.c_uint64()
    lib().oracle_mh_extract(z, T, N, ct.byref(i), ct.byref(j))
    return int(i.value), int(j.value)


def mh_from_cartesian(src: np.ndarray, T: int) -> np.ndarray:
    _u32(src)
    N = src.shape[0]
    assert src.shape == (N, N)
    dst = np.empty(N * N, dtype=np.uint32)
    lib().oracle_mh_from_cartesian(_ptr(dst), _ptr(src), N, N, T)
    return dst


def mh_to_cartesian(src_mh: np.ndarray, N: int, T: int) -> np.ndarray:
    _u32(src_mh)
    assert src_mh.size == N * N
    dst = np.empty((N, N), dtype=np.uint32)
    lib().oracle_mh_to_cartesian(_ptr(dst), N, _ptr(src_mh), N, T)
    return dst


def classify(N: int, T: int, row: int, col: int, rows: int, cols: int) -> int:
    return int(lib().oracle_classify(N, T, row, col, rows, cols))


def recursive_mm(C_mh, NC, rc, cc, A_mh, NA, ra, ca, B_mh, NB, rb, cb, m, k, n, p, T,
                 count_only: bool = False) -> int:
    """The paper's modified product on Morton-hybrid buffers (in place on C_mh).

    Returns the number of base-case calls."""
    if count_only:
        nul = ct.c_void_p(0)
        return int(lib().oracle_recursive_mm(nul, NC, rc, cc, nul, NA, ra, ca, nul, NB, rb, cb,
                                             m, k, n, p, T, 1))
    _u32(C_mh), _u32(A_mh), _u32(B_mh)
    return int(lib().oracle_recursive_mm(_ptr(C_mh), NC, rc, cc, _ptr(A_mh), NA, ra, ca,
                                         _ptr(B_mh), NB, rb, cb, m, k, n, p, T, 0))


def limb_digits(x: int, p: int, L: int) -> tuple[list[int], bool]:
    d = (ct.c_int8 * L)()
    ok = lib().oracle_limb_digits(x, p, L, ct.cast(d, ct.c_void_p))
    return [int(v) for v in d], bool(ok)
