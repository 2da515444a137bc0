"""Build libmh_san.so: libmh with its host code (planner, classification,
index math, context, batch queue) under AddressSanitizer and
UndefinedBehaviorSanitizer.  The device code is built as usual: the
sanitizers apply to the host side only.  With MH_SANITIZE=1 the binding
loads this library instead of libmh.so; the run is described in
oracle/build_sanitized.py.  For CPU-only runs of the host tests.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build as base  # noqa: E402  (the regular build's flags and sources)

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-g"]
OUT = os.path.join(HERE, "libmh_san.so")
BUILD = os.path.join(HERE, "_build_san")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    r = subprocess.run(["hipcc", *base.CXXFLAGS, *SAN, "-c", src, "-o", obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = base.sources()
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), len(os.sched_getaffinity(0)))) as ex:
        objs = list(ex.map(_compile, srcs))
    r = subprocess.run(["hipcc", f"--offload-arch={base.ARCH}", "-shared", "-fPIC", *objs,
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                        "-fsanitize=undefined", "-shared-libsan", "-o", OUT,
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    return OUT


if __name__ == "__main__":
    print(build())
