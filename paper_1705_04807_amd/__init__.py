"""Python binding of libmh (include/mh.h): argument marshalling only.

Every function keeps the C name and argument order of the C ABI.  Device
pointers are plain integers (``tensor.data_ptr()`` of torch int32 tensors
used as raw uint32 storage); streams are ``hipStream_t`` handles as
integers (``torch.cuda.current_stream().cuda_stream``), 0 for the null
stream.  Status codes are returned as ints; :func:`check` turns a non-zero
status into an exception.

The library is loaded from this directory (``libmh.so``, built by
``build.py``).  There is no fallback: if the library is missing, importing
the binding raises.
"""

from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MH_SANITIZE=1 selects the build whose host code runs under AddressSanitizer
# and UndefinedBehaviorSanitizer (build_sanitized.py; CPU-only test runs).
LIB_PATH = os.path.join(_HERE, "libmh_san.so" if os.environ.get("MH_SANITIZE") == "1"
                        else "libmh.so")

MH_OK = 0
MH_E_INVALID = 1
MH_E_SHAPE = 2
MH_E_BOUNDS = 3
MH_E_MODULUS = 4
MH_E_ALIAS = 5
MH_E_UNSUPPORTED = 6
MH_E_NOMEM = 7
MH_E_DEVICE = 8

MH_ALIGNED = 1
MH_CONTAINED = 2
MH_QUADRANT = 4

MH_MODE_AUTO = 0
MH_MODE_PLAIN_U32 = 1
MH_MODE_LIMB_I8 = 2
MH_MODE_FP64 = 3
MH_MODE_PLAIN_ELEMENTWISE = 4
MH_SUBTRACT = 0x100

MH_K_LAYOUT_FROM = 0
MH_K_LAYOUT_TO = 1
MH_K_PACK = 2
MH_K_GEMM_PLAIN = 3
MH_K_GEMM_LIMB = 4
MH_K_BATCHED = 5
MH_K_GEMM_F64 = 6
MH_K_COUNT = 7

MH_BATCH_FORM_EARLY_C = 1  # mh_ctx_last_batch_config forms
MH_BATCH_FORM_A_PARENT = 2

# Every symbol declared in include/mh.h.
EXPORTS = (
    "mh_ctx_create", "mh_ctx_destroy", "mh_status_string", "mh_ctx_last_device_error",
    "mh_ctx_set_timing", "mh_ctx_kernel_time", "mh_encode", "mh_extract",
    "mh_classify_submatrix", "mh_layout_from_cartesian", "mh_layout_to_cartesian",
    "mh_matmul_modp", "mh_matmul_modp_batched", "mh_plan_describe", "mh_plan_leaves",
    "mh_plan_gemm_tasks", "mh_ctx_set_autotune", "mh_ctx_tune_lookup", "mh_ctx_tune_cache_save",
    "mh_ctx_tune_cache_load", "mh_parent_size", "mh_layout_from_cartesian_padded",
    "mh_layout_to_cartesian_padded", "mh_ctx_kernel_times", "mh_probe_mfma_i8",
    "mh_probe_valu_mac", "mh_ctx_set_workspace_limit", "mh_ctx_workspace_info",
    "mh_matmul_modp_noalloc", "mh_ctx_last_batch_config", "mh_validate_batch",
)


class MhError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (%d)" % (what or "libmh", mh_status_string(status), status))


class mh_mm_desc(ct.Structure):
    _fields_ = [("C", ct.c_void_p), ("A", ct.c_void_p), ("B", ct.c_void_p),
                ("NC", ct.c_int64), ("NA", ct.c_int64), ("NB", ct.c_int64),
                ("rc", ct.c_int64), ("cc", ct.c_int64), ("ra", ct.c_int64),
                ("ca", ct.c_int64), ("rb", ct.c_int64), ("cb", ct.c_int64),
                ("m", ct.c_int64), ("k", ct.c_int64), ("n", ct.c_int64)]


class mh_plan_info(ct.Structure):
    _fields_ = [("row_segments", ct.c_int64), ("inner_segments", ct.c_int64),
                ("col_segments", ct.c_int64), ("leaves", ct.c_int64), ("c_tiles", ct.c_int64),
                ("gemm_tasks", ct.c_int64), ("pack_chunks", ct.c_int64), ("mode", ct.c_int32),
                ("in_place", ct.c_int32), ("tile_m", ct.c_int32), ("tile_n", ct.c_int32),
                ("limbs", ct.c_int32), ("kblock", ct.c_int32), ("kernel_cfg", ct.c_int32)]


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 and
    # libhsa-runtime64 (same sonames as ROCm's).  Loading torch first makes
    # libmh bind to those copies, so device pointers and streams from torch
    # are valid in libmh; loading libmh first would bring in a second runtime
    # that cannot open the device once torch has.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmh.so is not built (run paper_1705_04807_amd/build.py): " + LIB_PATH)
    L = ct.CDLL(LIB_PATH)
    P, I32, I64, U32, U64 = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_uint64
    sig = {
        "mh_ctx_create": ([ct.POINTER(P), ct.c_int], ct.c_int),
        "mh_ctx_destroy": ([P], ct.c_int),
        "mh_status_string": ([ct.c_int], ct.c_char_p),
        "mh_ctx_last_device_error": ([P], ct.c_int),
        "mh_ctx_set_timing": ([P, ct.c_int], ct.c_int),
        "mh_ctx_set_workspace_limit": ([P, U64], ct.c_int),
        "mh_ctx_workspace_info": ([P, ct.POINTER(U64), ct.POINTER(U64)], ct.c_int),
        "mh_ctx_kernel_time": ([P, ct.c_int, ct.POINTER(ct.c_double), ct.POINTER(I64), ct.c_int],
                               ct.c_int),
        "mh_ctx_kernel_times": ([P, ct.c_int, ct.POINTER(ct.c_double), I64, ct.POINTER(I64)],
                                ct.c_int),
        "mh_probe_mfma_i8": ([P, I32, ct.POINTER(ct.c_double), P], ct.c_int),
        "mh_probe_valu_mac": ([P, I32, ct.POINTER(ct.c_double), P], ct.c_int),
        "mh_ctx_set_autotune": ([P, ct.c_int], ct.c_int),
        "mh_ctx_tune_lookup": ([P, U32, I32, I64, I64, I64, ct.POINTER(I32)], ct.c_int),
        "mh_ctx_tune_cache_save": ([P, ct.c_char_p], ct.c_int),
        "mh_ctx_tune_cache_load": ([P, ct.c_char_p, ct.POINTER(I32)], ct.c_int),
        "mh_encode": ([U64, U64, U32], U64),
        "mh_extract": ([U64, U32, ct.POINTER(U64), ct.POINTER(U64)], None),
        "mh_classify_submatrix": ([I64, I32, I64, I64, I64, I64, ct.POINTER(U32)], ct.c_int),
        "mh_layout_from_cartesian": ([P, P, P, I64, I64, I32, P], ct.c_int),
        "mh_layout_to_cartesian": ([P, P, I64, P, I64, I32, P], ct.c_int),
        "mh_parent_size": ([I64, I64, I32, ct.POINTER(I64)], ct.c_int),
        "mh_layout_from_cartesian_padded": ([P, P, I64, P, I64, I64, I64, I32, P], ct.c_int),
        "mh_layout_to_cartesian_padded": ([P, P, I64, I64, I64, P, I64, I32, P], ct.c_int),
        "mh_matmul_modp": ([P, P, I64, I64, I64, P, I64, I64, I64, P, I64, I64, I64, I64, I64,
                            I64, U32, I32, I32, P], ct.c_int),
        "mh_matmul_modp_noalloc": ([P, P, I64, I64, I64, P, I64, I64, I64, P, I64, I64, I64, I64,
                                    I64, I64, U32, I32, I32, P], ct.c_int),
        "mh_matmul_modp_batched": ([P, ct.POINTER(mh_mm_desc), I32, U32, I32, I32, P], ct.c_int),
        "mh_ctx_last_batch_config": ([P, ct.POINTER(I32), ct.POINTER(I32), ct.POINTER(I32)],
                                     ct.c_int),
        "mh_validate_batch": ([ct.POINTER(mh_mm_desc), I32, U32, I32, I32], ct.c_int),
        "mh_plan_describe": ([I64] * 12 + [U32, I32, I32, ct.POINTER(mh_plan_info)], ct.c_int),
        "mh_plan_leaves": ([I64] * 12 + [I32, ct.POINTER(I64), I64, ct.POINTER(I64)], ct.c_int),
        "mh_plan_gemm_tasks": ([I64] * 12 + [U32, I32, I32, ct.POINTER(I64), I64,
                                             ct.POINTER(I64)], ct.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def check(status: int, what: str = "") -> None:
    if status != MH_OK:
        raise MhError(status, what)


# ------------------------------------------------------------------ context

def mh_ctx_create(hip_device: int = 0) -> int:
    h = ct.c_void_p()
    check(lib.mh_ctx_create(ct.byref(h), hip_device), "mh_ctx_create")
    return h.value


def mh_ctx_destroy(ctx: int) -> int:
    return lib.mh_ctx_destroy(ctx)


def mh_status_string(status: int) -> str:
    return lib.mh_status_string(status).decode()


def mh_ctx_last_device_error(ctx: int) -> int:
    return lib.mh_ctx_last_device_error(ctx)


def mh_ctx_set_workspace_limit(ctx: int, nbytes: int) -> int:
    return lib.mh_ctx_set_workspace_limit(ctx, nbytes)


def mh_ctx_workspace_info(ctx: int) -> tuple[int, int, int]:
    """Returns (status, limit in bytes (0 = none), bytes held)."""
    lim, held = ct.c_uint64(), ct.c_uint64()
    s = lib.mh_ctx_workspace_info(ctx, ct.byref(lim), ct.byref(held))
    return s, lim.value, held.value


def mh_ctx_set_timing(ctx: int, enable: bool) -> int:
    return lib.mh_ctx_set_timing(ctx, 1 if enable else 0)


def mh_ctx_kernel_time(ctx: int, kernel: int, reset: bool = False) -> tuple[float, int]:
    ms = ct.c_double()
    n = ct.c_int64()
    check(lib.mh_ctx_kernel_time(ctx, kernel, ct.byref(ms), ct.byref(n), 1 if reset else 0),
          "mh_ctx_kernel_time")
    return ms.value, n.value


def mh_probe_mfma_i8(ctx: int, iters: int, stream: int) -> float:
    """Sustained int8 MFMA operations per second of the context's device
    (random register operands, no memory traffic; see include/mh.h)."""
    pops = ct.c_double()
    check(lib.mh_probe_mfma_i8(ctx, iters, ct.byref(pops), stream), "mh_probe_mfma_i8")
    return pops.value


def mh_probe_valu_mac(ctx: int, iters: int, stream: int) -> float:
    """Sustained 96-bit multiply-accumulates per second of the plain form's
    instruction pair (see include/mh.h)."""
    macs = ct.c_double()
    check(lib.mh_probe_valu_mac(ctx, iters, ct.byref(macs), stream), "mh_probe_valu_mac")
    return macs.value


def mh_ctx_kernel_times(ctx: int, kernel: int, cap: int = 4096) -> list[float]:
    """Durations (ms) of the recorded launches of one kernel class, in launch order."""
    buf = (ct.c_double * max(cap, 1))()
    n = ct.c_int64()
    check(lib.mh_ctx_kernel_times(ctx, kernel, buf, cap, ct.byref(n)), "mh_ctx_kernel_times")
    return [buf[i] for i in range(min(cap, n.value))]


def mh_ctx_set_autotune(ctx: int, mode: int) -> int:
    return lib.mh_ctx_set_autotune(ctx, mode)


def mh_ctx_tune_lookup(ctx: int, p: int, T: int, m: int, k: int, n: int) -> int:
    c = ct.c_int32()
    check(lib.mh_ctx_tune_lookup(ctx, p, T, m, k, n, ct.byref(c)), "mh_ctx_tune_lookup")
    return c.value


def mh_ctx_tune_cache_save(ctx: int, path: str) -> int:
    return lib.mh_ctx_tune_cache_save(ctx, path.encode())


def mh_ctx_tune_cache_load(ctx: int, path: str) -> tuple[int, int]:
    """Returns (status, entries loaded)."""
    n = ct.c_int32()
    s = lib.mh_ctx_tune_cache_load(ctx, path.encode(), ct.byref(n))
    return s, n.value


# ---------------------------------------------------------------- host math

def mh_encode(i: int, j: int, T: int) -> int:
    return int(lib.mh_encode(i, j, T))


def mh_extract(z: int, T: int) -> tuple[int, int]:
    i, j = ct.c_uint64(), ct.c_uint64()
    lib.mh_extract(z, T, ct.byref(i), ct.byref(j))
    return int(i.value), int(j.value)


def mh_classify_submatrix(N: int, T: int, row: int, col: int, rows: int, cols: int):
    """Returns (status, flags)."""
    f = ct.c_uint32()
    s = lib.mh_classify_submatrix(N, T, row, col, rows, cols, ct.byref(f))
    return s, int(f.value)


# ------------------------------------------------------------------ device

def mh_layout_from_cartesian(ctx, dst_mh: int, src: int, ld_src: int, N: int, T: int,
                             stream: int = 0) -> int:
    return lib.mh_layout_from_cartesian(ctx, dst_mh, src, ld_src, N, T, stream)


def mh_layout_to_cartesian(ctx, dst: int, ld_dst: int, src_mh: int, N: int, T: int,
                           stream: int = 0) -> int:
    return lib.mh_layout_to_cartesian(ctx, dst, ld_dst, src_mh, N, T, stream)


def mh_parent_size(rows: int, cols: int, T: int):
    """Returns (status, N)."""
    n = ct.c_int64(0)
    s = lib.mh_parent_size(rows, cols, T, ct.byref(n))
    return s, n.value


def mh_layout_from_cartesian_padded(ctx, dst_mh: int, N: int, src: int, ld_src: int, rows: int,
                                    cols: int, T: int, stream: int = 0) -> int:
    return lib.mh_layout_from_cartesian_padded(ctx, dst_mh, N, src, ld_src, rows, cols, T, stream)


def mh_layout_to_cartesian_padded(ctx, dst: int, ld_dst: int, rows: int, cols: int, src_mh: int,
                                  N: int, T: int, stream: int = 0) -> int:
    return lib.mh_layout_to_cartesian_padded(ctx, dst, ld_dst, rows, cols, src_mh, N, T, stream)


def mh_matmul_modp(ctx, C: int, NC: int, rc: int, cc: int, A: int, NA: int, ra: int, ca: int,
                   B: int, NB: int, rb: int, cb: int, m: int, k: int, n: int, p: int, T: int,
                   mode: int = MH_MODE_AUTO, stream: int = 0) -> int:
    return lib.mh_matmul_modp(ctx, C, NC, rc, cc, A, NA, ra, ca, B, NB, rb, cb, m, k, n, p, T,
                              mode, stream)


def mh_matmul_modp_noalloc(ctx, C: int, NC: int, rc: int, cc: int, A: int, NA: int, ra: int,
                           ca: int, B: int, NB: int, rb: int, cb: int, m: int, k: int, n: int,
                           p: int, T: int, mode: int = MH_MODE_AUTO, stream: int = 0) -> int:
    return lib.mh_matmul_modp_noalloc(ctx, C, NC, rc, cc, A, NA, ra, ca, B, NB, rb, cb, m, k, n,
                                      p, T, mode, stream)


def make_descs(items) -> ct.Array:
    """Array of mh_mm_desc from dicts/tuples with the struct's field names."""
    arr = (mh_mm_desc * len(items))()
    for d, it in zip(arr, items):
        for key, val in (it.items() if isinstance(it, dict) else it):
            setattr(d, key, val)
    return arr


def mh_matmul_modp_batched(ctx, descs, count: int, p: int, T: int,
                           mode: int = MH_MODE_AUTO, stream: int = 0) -> int:
    return lib.mh_matmul_modp_batched(ctx, descs, count, p, T, mode, stream)


# ----------------------------------------------------------------- planner

def mh_validate_batch(descs, count: int, p: int, T: int, mode: int = MH_MODE_AUTO) -> int:
    return lib.mh_validate_batch(descs, count, p, T, mode)


def mh_ctx_last_batch_config(ctx) -> tuple[int, int, int, int]:
    """(status, cfg, limbs, forms) of the last batched graph the context launched."""
    cfg, limbs, forms = ct.c_int32(-1), ct.c_int32(0), ct.c_int32(0)
    s = lib.mh_ctx_last_batch_config(ctx, ct.byref(cfg), ct.byref(limbs), ct.byref(forms))
    return s, cfg.value, limbs.value, forms.value


def mh_plan_describe(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, p, T, mode=MH_MODE_AUTO):
    """Returns (status, mh_plan_info)."""
    info = mh_plan_info()
    s = lib.mh_plan_describe(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, p, T, mode,
                             ct.byref(info))
    return s, info


def mh_plan_leaves(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, T, cap: int):
    """Returns (status, total, [(i0, ni, l0, nl, j0, nj), ...] up to cap)."""
    buf = (ct.c_int64 * (6 * max(cap, 1)))()
    cnt = ct.c_int64()
    s = lib.mh_plan_leaves(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, T, buf, cap,
                           ct.byref(cnt))
    got = min(cap, cnt.value)
    return s, cnt.value, [tuple(buf[6 * q:6 * q + 6]) for q in range(got)]


def mh_plan_gemm_tasks(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, p, T, mode, cap: int):
    """Returns (status, total, [(i0, ni, j0, nj), ...] up to cap)."""
    buf = (ct.c_int64 * (4 * max(cap, 1)))()
    cnt = ct.c_int64()
    s = lib.mh_plan_gemm_tasks(NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n, p, T, mode, buf,
                               cap, ct.byref(cnt))
    got = min(cap, cnt.value)
    return s, cnt.value, [tuple(buf[4 * q:4 * q + 4]) for q in range(got)]
