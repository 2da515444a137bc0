"""Throughput of C := C + A.B mod p on Morton-hybrid operands (one MI355X).

One step = one whole product through the C ABI (planner, limb packing,
int8 MFMA GEMM and the mod-p epilogue) with the operands already resident in
HBM in Morton-hybrid layout.  Prints one JSON line:
  value  = modular GOPS (2mnk / s) of the timed steps, whole job;
  roofline = the dominant kernel (the limb GEMM) against the int8 MFMA peak,
             its average duration taken from HIP events the library records
             on the stream it launches on; beside the published peak,
             sustained_peak = the int8 MFMA rate the device keeps up under
             its power limit (mh_probe_mfma_i8, after the timed region);
  plain  = the plain uint32 kernel on the same workload (the comparator);
  fp64   = the FP64-MFMA form on the same workload, when p < 2^26;
  cpu_baseline = the CPU oracle (triple loop, 128-bit accumulators) on a
             bounded sample of output rows of the same workload.
The default run (the 8192^3 product) adds one key per other workload of the
metric, each with the same fields (value, ms_per_step, config, roofline,
plain, fp64 where p < 2^26, cpu_baseline on a smaller sample), timed after
the headline: aligned_4096cube_p65521, nonaligned_8192parents_p65521 and
batched_512_tu_level_p65521 (the batched graph, a loop of single calls and
the plain form's batch).  --no-extras leaves them out.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
       python bench.py --copy-calibration   (plain 1 GiB device copy, three times:
                                             the reference for scaling HBM counters)

roofline.traffic comes from the committed rocprofv3 counter summary under
profiles/ (a "traffic-record:" line); it is used only when that record names
the same kernel configuration, workload and kernel source hash as this run,
and is null otherwise.
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "modular GOPS (2mnk/s) for C+=A·B mod p, MFMA/batched vs plain, bit-exact"
INT8_PEAK_TOPS = 5000.0   # MI355X dense int8 MFMA, 5.0 POP/s
FP64_PEAK_TFLOPS = 78.6   # MI355X dense fp64 MFMA
PROBE_ITERS = 40000       # mh_probe_mfma_i8: 8 x 40000 MFMAs per wave, about 7 ms a launch
VALU_PROBE_ITERS = 8192   # mh_probe_valu_mac: 16 x 8192 per lane, about 7 ms a launch
# Plain kernel: one multiply-accumulate = v_mad_u64_u32 + v_addc_co_u32, two
# full-rate VALU instructions; 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz / 2.
PLAIN_PEAK_TMACS = 256 * 4 * 16 * 2.4e9 / 2 / 1e12
FP64_MAX_P = (1 << 26) - 1
P31 = 2**31 - 1

WORKLOADS = {
    # 8192^3 aligned product at the large prime: four 8-bit limbs, one k-block
    "modp_8192cube_p2^31-1_T64": dict(N=8192, T=64, p=P31, m=8192, k=8192, n=8192,
                                      off=(0, 0, 0, 0, 0, 0), seeds=(4001, 4002, 4003)),
    # one GPU's share of the 8192^3 product split 4 x 2 over eight GPUs: the
    # 2048 x 4096 block of C at (2048, 4096), all of k (no exchange needed)
    "modp_8192cube_shard_2048x4096_p2^31-1_T64": dict(
        N=8192, T=64, p=P31, m=2048, k=8192, n=4096,
        off=(2048, 4096, 2048, 0, 0, 4096), seeds=(4001, 4002, 4003)),
    # 4096^3 aligned product at p = 65521: two limbs
    "modp_4096cube_p65521_T64": dict(N=4096, T=64, p=65521, m=4096, k=4096, n=4096,
                                     off=(0, 0, 0, 0, 0, 0), seeds=(2001, 2002, 2003)),
    # non-aligned rectangular blocks of 8192^2 parents
    "modp_nonaligned_8192parents_p65521_T64": dict(
        N=8192, T=64, p=65521, m=6000, k=3000, n=5000,
        off=(64, 33, 1000, 1500, 517, 2048), seeds=(3001, 3002, 3003)),
    # the same blocks with the paper's truncation size T' = 32 and with 16
    "modp_nonaligned_8192parents_p65521_T32": dict(
        N=8192, T=32, p=65521, m=6000, k=3000, n=5000,
        off=(64, 33, 1000, 1500, 517, 2048), seeds=(3001, 3002, 3003)),
    "modp_nonaligned_8192parents_p65521_T16": dict(
        N=8192, T=16, p=65521, m=6000, k=3000, n=5000,
        off=(64, 33, 1000, 1500, 517, 2048), seeds=(3001, 3002, 3003)),
}
# 512 uneven independent products of one TU recursion level, one batched call
BATCHED = "batched_512_tu_level_8192parents_p65521_T64"
DEFAULT = "modp_8192cube_p2^31-1_T64"
# keys of the default line beside the headline: the other workloads of the metric
EXTRA_SINGLE = (("aligned_4096cube_p65521", "modp_4096cube_p65521_T64"),
                ("nonaligned_8192parents_p65521", "modp_nonaligned_8192parents_p65521_T64"))
EXTRA_BATCHED = "batched_512_tu_level_p65521"
INT8_UNIT = "TOP/s"  # int8 multiply-add operations (two per multiply-accumulate)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_1705_04807_amd/csrc/mh_gemm_limb.hip",
                  "paper_1705_04807_amd/csrc/mh_device.h",
                  "paper_1705_04807_amd/csrc/mh_internal.h")
BATCHED_SOURCES = KERNEL_SOURCES + ("paper_1705_04807_amd/csrc/mh_pack.hip",
                                    "paper_1705_04807_amd/csrc/mh_batched.hip")


def kernel_source_hash(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def with_sustained(roof: dict, sustained):
    """Adds the measured ceiling beside the published peak (which stays the
    roofline's peak)."""
    if sustained:
        roof["sustained_peak"] = sustained
        roof["frac_sustained"] = roof["achieved"] / sustained
        roof["sustained_note"] = ("sustained_peak = int8 MFMA rate this device keeps up on "
                                  "random register operands with no memory traffic "
                                  "(mh_probe_mfma_i8): the published peak assumes the full "
                                  "clock, which the device lowers under this load")
    return roof


def recorded_traffic(kernel: str, cfg: int, workload: str, src: str):
    """HBM bytes per launch (fetch + write) from a matching traffic-record, else None."""
    pat = re.compile(r"traffic-record:\s+kernel=(\S+)\s+cfg=(\S+)\s+workload=(\S+)\s+src=(\S+)"
                     r"\s+fetch_bytes=(\d+)\s+write_bytes=(\d+)")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*"))):
        try:
            text = open(path).read()
        except OSError:
            continue
        for m in pat.finditer(text):
            if (m.group(1), m.group(2), m.group(3), m.group(4)) == (kernel, str(cfg), workload, src):
                return int(m.group(5)) + int(m.group(6))
    return None


def copy_calibration() -> None:
    """A plain device copy of 1 GiB, three times (reads 1 GiB, writes 1 GiB each)."""
    import torch
    n = 1 << 28
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": 4 * n}), flush=True)


def cpu_threads() -> int:
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(A_dev, B_dev, W, budget_s=12.0):
    """Oracle on a bounded sample of output rows; returns the cpu_baseline object."""
    import numpy as np
    import torch

    import oracle

    p, m, k, n = W["p"], W["m"], W["k"], W["n"]
    rc, cc, ra, ca, rb, cb = W["off"]
    nt = cpu_threads()
    Bh = B_dev[rb:rb + k, cb:cb + n].contiguous().cpu().numpy().view(np.uint32)
    Bh = np.ascontiguousarray(Bh)

    def run(rows, threads=nt):
        Ah = np.ascontiguousarray(
            A_dev[ra:ra + rows, ca:ca + k].contiguous().cpu().numpy().view(np.uint32))
        Ch = np.zeros((rows, n), np.uint32)
        t0 = time.perf_counter()
        oracle.matmul_modp(Ch, Ah, Bh, p, nthreads=threads)
        return time.perf_counter() - t0

    probe = max(1, min(m, nt))
    t = run(probe)
    rows = int(min(m, max(probe, budget_s / max(t, 1e-6) * probe)))
    rows = max(probe, (rows // nt) * nt) if rows >= nt else rows
    t = run(rows) if rows != probe else t
    gops = 2.0 * rows * n * k / t / 1e9
    # the same loop on one thread, over a sample sized to about a fifth of the budget
    rows1 = max(1, min(m, int(budget_s / 5 * gops * 1e9 / nt / (2.0 * n * k))))
    t1 = run(rows1, 1)
    return {"value": gops, "unit": "GOPS", "cores": nt, "kind": "oracle", "cpu": cpu_model(),
            "sample": "%d of %d output rows (all %d columns, k=%d), %.1f s" % (rows, m, n, k, t),
            "single_thread": {"value": 2.0 * rows1 * n * k / t1 / 1e9, "unit": "GOPS",
                              "sample": "%d output rows, %.1f s" % (rows1, t1)}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_workload(args, mh, name, steps, warmup, cpu_budget):
    """One product of workload `name` (operands resident in HBM, Morton-hybrid
    layout): the limb form timed over `steps` steps after `warmup` (the first
    warm-up call tunes the configuration), then the plain comparator, the
    FP64 form where p < 2^26, and the CPU oracle on a bounded sample.
    Returns the fields of one bench line (the headline or an extra key)."""
    import torch

    from seeded_inputs import residues_torch

    W = WORKLOADS[name]
    N, T, p, m, k, n = W["N"], W["T"], W["p"], W["m"], W["k"], W["n"]
    rc, cc, ra, ca, rb, cb = W["off"]
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    ctx = mh.mh_ctx_create(0)

    log("generating %s" % name)
    cart = {}
    parents = {}
    for key, seed in zip("ABC", W["seeds"]):
        X = residues_torch(seed, p, N, N, device="cuda")
        cart[key] = X
        Y = torch.empty(N * N, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        mh.check(mh.mh_layout_from_cartesian(ctx, Y.data_ptr(), X.data_ptr(), N, N, T, sh))
        parents[key] = Y
    torch.cuda.synchronize()
    stream.synchronize()

    def step(mode):
        mh.check(mh.mh_matmul_modp(ctx, parents["C"].data_ptr(), N, rc, cc,
                                   parents["A"].data_ptr(), N, ra, ca, parents["B"].data_ptr(), N,
                                   rb, cb, m, k, n, p, T, mode, sh), "mh_matmul_modp")

    work = 2.0 * m * n * k
    s, info = mh.mh_plan_describe(N, rc, cc, N, ra, ca, N, rb, cb, m, k, n, p, T,
                                  mh.MH_MODE_LIMB_I8)
    mh.check(s)
    L = info.limbs

    # ---- limb MFMA form; the first warm-up call tunes the kernel
    # configuration for this shape (untimed)
    if not args.no_autotune:
        mh.check(mh.mh_ctx_set_autotune(ctx, 2))
    log("%s: warmup %d" % (name, warmup))
    for _ in range(max(warmup, 1)):
        step(mh.MH_MODE_LIMB_I8)
    stream.synchronize()
    torch.cuda.synchronize()
    mh.mh_ctx_set_timing(ctx, True)
    for kk in range(mh.MH_K_COUNT):
        mh.mh_ctx_kernel_time(ctx, kk, reset=True)
    log("%s: timing %d steps" % (name, steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(mh.MH_MODE_LIMB_I8)
    stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gemm_each = mh.mh_ctx_kernel_times(ctx, mh.MH_K_GEMM_LIMB)
    gemm_ms, gemm_n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_GEMM_LIMB, reset=True)
    tuned = mh.mh_ctx_tune_lookup(ctx, p, T, m, k, n)
    kernel_cfg = tuned if tuned >= 0 else info.kernel_cfg
    pack_ms, pack_n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_PACK, reset=True)
    mh.mh_ctx_set_timing(ctx, False)
    ms_per_step = elapsed / steps * 1e3
    value = work * steps / elapsed / 1e9
    gemm_avg = gemm_ms / max(gemm_n, 1)
    int8_tops = L * L * work / (gemm_avg * 1e-3) / 1e12
    log("%s: limb %.3f ms/step, gemm %.3f ms, pack %.3f ms"
        % (name, ms_per_step, gemm_avg, pack_ms / max(pack_n, 1)))

    # ---- plain uint32 kernel (comparator)
    plain = None
    if args.plain_steps > 0:
        step(mh.MH_MODE_PLAIN_U32)
        stream.synchronize()
        mh.mh_ctx_set_timing(ctx, True)
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(mh.MH_MODE_PLAIN_U32)
        stream.synchronize()
        pe = time.perf_counter() - t0
        pg_ms, pg_n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_GEMM_PLAIN, reset=True)
        mh.mh_ctx_kernel_time(ctx, mh.MH_K_PACK, reset=True)
        mh.mh_ctx_set_timing(ctx, False)
        pgemm = pg_ms / max(pg_n, 1)
        tmacs = work / 2 / (pgemm * 1e-3) / 1e12
        plain = {"value": work * args.plain_steps / pe / 1e9, "unit": "GOPS",
                 "ms_per_step": pe / args.plain_steps * 1e3, "gemm_ms": pgemm,
                 "roofline": {"bound": "alu", "achieved": tmacs, "peak": PLAIN_PEAK_TMACS,
                              "unit": "T multiply-accumulates/s",
                              "frac": tmacs / PLAIN_PEAK_TMACS, "kernel": "k_gemm_plain"}}
        plain["limb_speedup"] = value / plain["value"]
        log("%s: plain %.3f ms/step" % (name, plain["ms_per_step"]))

    # ---- FP64-MFMA form (primes below 2^26 only)
    fp64 = None
    if args.fp64_steps > 0 and p <= FP64_MAX_P:
        step(mh.MH_MODE_FP64)
        stream.synchronize()
        mh.mh_ctx_set_timing(ctx, True)
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            step(mh.MH_MODE_FP64)
        stream.synchronize()
        fe = time.perf_counter() - t0
        fg_ms, fg_n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_GEMM_F64, reset=True)
        fp_ms, fp_n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_PACK, reset=True)
        mh.mh_ctx_set_timing(ctx, False)
        fgemm = fg_ms / max(fg_n, 1)
        ftf = work / (fgemm * 1e-3) / 1e12
        fp64 = {"value": work * args.fp64_steps / fe / 1e9, "unit": "GOPS",
                "ms_per_step": fe / args.fp64_steps * 1e3, "gemm_ms": fgemm,
                "pack_ms": fp_ms / max(fp_n, 1) if fp_n else 0.0,
                "roofline": {"bound": "mfma", "achieved": ftf, "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": ftf / FP64_PEAK_TFLOPS,
                             "kernel": "k_gemm_f64"}}
        fp64["limb_speedup"] = value / fp64["value"]
        log("%s: fp64 %.3f ms/step, gemm %.3f ms" % (name, fp64["ms_per_step"], fgemm))
    assert mh.mh_ctx_last_device_error(ctx) == 0

    cpu = None
    if not args.no_cpu_baseline:
        log("%s: cpu baseline" % name)
        cpu = cpu_baseline(cart["A"], cart["B"], W, budget_s=cpu_budget)
    mh.mh_ctx_destroy(ctx)
    del cart, parents
    torch.cuda.empty_cache()
    return {
        "value": value, "unit": "GOPS", "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step,
        "config": {"workload": name, "m": m, "k": k, "n": n, "p": p, "T": T,
                   "parents": N, "offsets_c_a_b": list(W["off"]), "limbs": L,
                   "mode": "limb_i8", "tile": [info.tile_m, info.tile_n]},
        "roofline": {"bound": "mfma", "achieved": int8_tops, "peak": INT8_PEAK_TOPS,
                     "unit": INT8_UNIT, "frac": int8_tops / INT8_PEAK_TOPS,
                     "traffic": recorded_traffic("k_gemm_limb", kernel_cfg, name,
                                                 kernel_source_hash()),
                     "kernel": "k_gemm_limb", "kernel_cfg": kernel_cfg,
                     "kernel_src": kernel_source_hash(), "kernel_ms": gemm_avg,
                     "kernel_ms_min": min(gemm_each) if gemm_each else None,
                     "kernel_ms_median": (sorted(gemm_each)[len(gemm_each) // 2]
                                          if gemm_each else None),
                     "note": "achieved = int8 multiply-add operations (L^2 * 2mnk) per launch "
                             "/ average launch time, in tera-operations per second; traffic = "
                             "HBM bytes per launch from FETCH_SIZE and WRITE_SIZE, "
                             "copy-calibrated"},
        "pack_ms": pack_ms / max(pack_n, 1),
        "plain": plain,
        "fp64": fp64,
        "cpu_baseline": cpu,
    }


def probes(args, mh):
    """Measured ceilings, after every timed region: the sustained int8 MFMA
    rate and the plain form's multiply-accumulate issue rate (None, None
    with --no-probe)."""
    if args.no_probe:
        return None, None
    import torch
    stream = torch.cuda.Stream()
    ctx = mh.mh_ctx_create(0)
    log("sustained multiply-accumulate probe")
    smacs = max(mh.mh_probe_valu_mac(ctx, VALU_PROBE_ITERS, stream.cuda_stream)
                for _ in range(3)) / 1e12
    log("sustained int8 MFMA probe")
    sint8 = max(mh.mh_probe_mfma_i8(ctx, PROBE_ITERS, stream.cuda_stream)
                for _ in range(3)) / 1e12
    mh.mh_ctx_destroy(ctx)
    return sint8, smacs


def with_plain_sustained(plain, smacs):
    if plain and smacs and "roofline" in plain:
        r = plain["roofline"]
        r.update({"sustained_peak": smacs, "frac_sustained": r["achieved"] / smacs,
                  "sustained_note": "sustained_peak = issue rate of the same multiply-accumulate "
                                    "pair with no memory traffic (mh_probe_valu_mac)"})
    return plain


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + [BATCHED])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="timed steps of the FP64-MFMA form (only for p < 2^26)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the sustained-rate probes (mh_probe_mfma_i8, mh_probe_valu_mac)")
    ap.add_argument("--no-extras", action="store_true",
                    help="the default run measures only the 8192^3 product, without the "
                         "4096^3, non-aligned and 512-product batch workloads beside it")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--ablation", action="store_true",
                    help="plain kernel through the planner against the elementwise comparator "
                         "(per-element Morton-hybrid encoding, no planner) on --workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="built-in kernel configuration instead of tuning during warm-up")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X and has "
              "no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1705_04807_amd as mh
    torch.cuda.set_device(0)

    if args.ablation:
        ablation(args, mh)
        return

    extras = {}
    if args.workload == BATCHED:
        head = batched_workload(args, mh, args.steps, args.warmup, 12.0)
    else:
        head = single_workload(args, mh, args.workload, args.steps, args.warmup, 12.0)
        if args.workload == DEFAULT and not args.no_extras:
            # the other workloads of the metric, each with its own roofline and
            # CPU baseline (smaller samples), after the headline's timed region
            for key, name in EXTRA_SINGLE:
                extras[key] = single_workload(args, mh, name, args.steps, args.warmup, 4.0)
            extras[EXTRA_BATCHED] = batched_workload(args, mh, args.steps, args.warmup, 4.0)
    sint8, smacs = probes(args, mh)
    for part in [head] + list(extras.values()):
        with_sustained(part["roofline"], sint8)
        with_plain_sustained(part.get("plain"), smacs)

    out = {"metric": METRIC, "value": head["value"], "unit": "GOPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8",
           "data": "synthetic", "config": head["config"], "roofline": head["roofline"]}
    for key, val in head.items():
        if key not in out and key not in ("steps", "warmup", "unit"):
            out[key] = val
    out.update(extras)
    print(json.dumps(out), flush=True)


def ablation(args, mh):
    """Problems P1/P2 of section 2.1 on the GPU: one kernel, two ways of reaching the
    operands.  Prints one JSON line (not the throughput line)."""
    import torch

    from seeded_inputs import residues_torch

    W = WORKLOADS[args.workload]
    N, T, p, m, k, n = W["N"], W["T"], W["p"], W["m"], W["k"], W["n"]
    rc, cc, ra, ca, rb, cb = W["off"]
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    ctx = mh.mh_ctx_create(0)
    parents = {}
    for key, seed in zip("ABC", W["seeds"]):
        X = residues_torch(seed, p, N, N, device="cuda")
        Y = torch.empty(N * N, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        mh.check(mh.mh_layout_from_cartesian(ctx, Y.data_ptr(), X.data_ptr(), N, N, T, sh))
        parents[key] = Y
    stream.synchronize()
    work = 2.0 * m * n * k

    def step(mode):
        mh.check(mh.mh_matmul_modp(ctx, parents["C"].data_ptr(), N, rc, cc,
                                   parents["A"].data_ptr(), N, ra, ca, parents["B"].data_ptr(), N,
                                   rb, cb, m, k, n, p, T, mode, sh), "mh_matmul_modp")

    def timed(mode, kernel):
        step(mode)
        stream.synchronize()
        mh.mh_ctx_set_timing(ctx, True)
        for kk in range(mh.MH_K_COUNT):
            mh.mh_ctx_kernel_time(ctx, kk, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(mode)
        stream.synchronize()
        el = time.perf_counter() - t0
        g_ms, g_n = mh.mh_ctx_kernel_time(ctx, kernel, reset=True)
        p_ms, p_n = mh.mh_ctx_kernel_time(ctx, mh.MH_K_PACK, reset=True)
        mh.mh_ctx_set_timing(ctx, False)
        return {"ms_per_step": el / args.steps * 1e3, "gemm_ms": g_ms / max(g_n, 1),
                "pack_ms": p_ms / max(p_n, 1) if p_n else 0.0,
                "value": work * args.steps / el / 1e9, "unit": "GOPS"}

    log("ablation: planner path")
    planner = timed(mh.MH_MODE_PLAIN_U32, mh.MH_K_GEMM_PLAIN)
    log("ablation: elementwise comparator")
    elementwise = timed(mh.MH_MODE_PLAIN_ELEMENTWISE, mh.MH_K_GEMM_PLAIN)
    assert mh.mh_ctx_last_device_error(ctx) == 0
    mh.mh_ctx_destroy(ctx)
    print(json.dumps({"ablation": "planner_vs_elementwise", "workload": args.workload,
                      "T": W["T"], "p": W["p"], "m": W["m"], "k": W["k"], "n": W["n"],
                      "offsets_c_a_b": list(W["off"]), "steps": args.steps,
                      "planner": planner, "elementwise": elementwise,
                      "planner_speedup": elementwise["ms_per_step"] / planner["ms_per_step"]}),
          flush=True)


def batched_workload(args, mh, steps, warmup, cpu_budget):
    """One step = one mh_matmul_modp_batched call over the 512 products of one
    TU recursion level; beside it a loop of single mh_matmul_modp calls and
    the plain form's batch (products one after another).  Returns the fields
    of one bench line."""
    import torch

    from seeded_inputs import residues_torch, tu_level_batch

    N, T, p, nC = 8192, 64, 65521, 64
    calls = tu_level_batch(seed=5000, count=512, N=N, n_c_parents=nC)
    work = float(sum(2 * c["m"] * c["k"] * c["n"] for c in calls))
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    ctx = mh.mh_ctx_create(0)
    log("batched: generating %d parents" % (nC + 2))

    def parent(seed):
        X = residues_torch(seed, p, N, N, device="cuda")
        Y = torch.empty(N * N, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        mh.check(mh.mh_layout_from_cartesian(ctx, Y.data_ptr(), X.data_ptr(), N, N, T, sh))
        stream.synchronize()
        return X, Y

    Acart, A = parent(5001)
    Bcart, B = parent(5002)
    Cs = [parent(5100 + j)[1] for j in range(nC)]
    descs = mh.make_descs([dict(C=Cs[c["ci"]].data_ptr(), A=A.data_ptr(), B=B.data_ptr(),
                                NC=N, NA=N, NB=N, rc=c["rc"], cc=c["cc"], ra=c["ra"],
                                ca=c["ca"], rb=c["rb"], cb=c["cb"], m=c["m"], k=c["k"],
                                n=c["n"]) for c in calls])

    def batched(mode):
        mh.check(mh.mh_matmul_modp_batched(ctx, descs, len(calls), p, T, mode, sh), "batched")

    def looped(mode):
        for c in calls:
            mh.check(mh.mh_matmul_modp(ctx, Cs[c["ci"]].data_ptr(), N, c["rc"], c["cc"],
                                       A.data_ptr(), N, c["ra"], c["ca"], B.data_ptr(), N,
                                       c["rb"], c["cb"], c["m"], c["k"], c["n"], p, T, mode, sh))

    def timed(fn, nsteps, kernels=()):
        stream.synchronize()
        mh.mh_ctx_set_timing(ctx, True)
        for kk in range(mh.MH_K_COUNT):
            mh.mh_ctx_kernel_time(ctx, kk, reset=True)
        t0 = time.perf_counter()
        for _ in range(nsteps):
            fn()
        stream.synchronize()
        el = time.perf_counter() - t0
        ks = {kk: mh.mh_ctx_kernel_time(ctx, kk, reset=True) for kk in kernels}
        mh.mh_ctx_set_timing(ctx, False)
        return el / nsteps, ks

    if not args.no_autotune:
        mh.check(mh.mh_ctx_set_autotune(ctx, 2))
    log("batched: warmup %d" % warmup)
    for _ in range(max(warmup, 1)):
        batched(mh.MH_MODE_LIMB_I8)
    t_b, ks = timed(lambda: batched(mh.MH_MODE_LIMB_I8), steps, (mh.MH_K_BATCHED,))
    graph_ms = ks[mh.MH_K_BATCHED][0] / max(ks[mh.MH_K_BATCHED][1], 1)
    s, batch_cfg, L, forms = mh.mh_ctx_last_batch_config(ctx)
    mh.check(s)
    value = work / t_b / 1e9
    log("batched: %.3f ms/step (graph %.3f ms, configuration %d, forms %d)"
        % (t_b * 1e3, graph_ms, batch_cfg, forms))
    looped(mh.MH_MODE_LIMB_I8)
    t_l, _ = timed(lambda: looped(mh.MH_MODE_LIMB_I8), 2)
    log("batched: looped %.3f ms" % (t_l * 1e3))
    plain = None
    if args.plain_steps > 0:
        batched(mh.MH_MODE_PLAIN_U32)
        t_p, _ = timed(lambda: batched(mh.MH_MODE_PLAIN_U32), max(args.plain_steps, 3))
        plain = {"value": work / t_p / 1e9, "unit": "GOPS", "ms_per_step": t_p * 1e3,
                 "steps": max(args.plain_steps, 3), "limb_speedup": value / (work / t_p / 1e9)}
        log("batched: plain %.3f ms" % (t_p * 1e3))
    assert mh.mh_ctx_last_device_error(ctx) == 0
    int8_tops = L * L * work / (graph_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        log("batched: cpu baseline")
        c0 = max(calls, key=lambda c: c["m"] * c["n"] * c["k"])
        W = dict(p=p, m=c0["m"], k=c0["k"], n=c0["n"],
                 off=(c0["rc"], c0["cc"], c0["ra"], c0["ca"], c0["rb"], c0["cb"]))
        cpu = cpu_baseline(Acart.view(N, N), Bcart.view(N, N), W, budget_s=cpu_budget)
        cpu["sample"] = "largest product of the batch: " + cpu["sample"]
    mh.mh_ctx_destroy(ctx)
    del Acart, Bcart, A, B, Cs
    torch.cuda.empty_cache()
    src = kernel_source_hash(BATCHED_SOURCES)
    return {
        "value": value, "unit": "GOPS", "steps": steps, "warmup": warmup,
        "ms_per_step": t_b * 1e3,
        "config": {"workload": BATCHED, "products": len(calls), "work_2mnk": work, "p": p,
                   "T": T, "parents": N, "c_parents": nC, "limbs": L, "mode": "limb_i8",
                   "form": "persistent pack + GEMM in one HIP graph"},
        "roofline": {"bound": "mfma", "achieved": int8_tops, "peak": INT8_PEAK_TOPS,
                     "unit": INT8_UNIT, "frac": int8_tops / INT8_PEAK_TOPS,
                     "traffic": recorded_traffic("batched_graph", batch_cfg, BATCHED, src),
                     "kernel": "batched graph (k_pack_limb_batched + k_gemm_limb_batched)",
                     "kernel_cfg": batch_cfg, "kernel_src": src, "kernel_ms": graph_ms,
                     "kernel_forms": {"early_c": bool(forms & mh.MH_BATCH_FORM_EARLY_C),
                                      "a_parent": bool(forms & mh.MH_BATCH_FORM_A_PARENT)},
                     "note": "achieved = int8 multiply-add operations of the whole batch "
                             "(L^2 * sum 2mnk) / graph time, in tera-operations per second; "
                             "traffic = HBM bytes per graph launch (both pack kernels and the "
                             "GEMM) from FETCH_SIZE and WRITE_SIZE, copy-calibrated"},
        "looped": {"value": work / t_l / 1e9, "unit": "GOPS", "ms_per_step": t_l * 1e3,
                   "steps": 2},
        "plain": plain,
        "cpu_baseline": cpu,
    }


if __name__ == "__main__":
    main()
