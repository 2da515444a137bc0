"""Build liboracle_san.so: the oracle with AddressSanitizer and
UndefinedBehaviorSanitizer, for host-only sanitizer runs of the CPU test
suite.  Compiled with the ROCm LLVM clang, so that one sanitizer runtime
(clang's) serves both this library and the sanitized host code of libmh
(paper_1705_04807_amd/build_sanitized.py) in one process.

    python oracle/build_sanitized.py
    python paper_1705_04807_amd/build_sanitized.py
    MH_SANITIZE=1 ASAN_OPTIONS=detect_leaks=0 \\
      LD_PRELOAD=$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so) \\
      python -m pytest tests -m "not gpu"

With MH_SANITIZE=1 the oracle wrapper loads this library instead of
liboracle.so.  Host code only: nothing here runs on a GPU.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CLANG = "/opt/rocm/llvm/bin/clang"
LLVM_LIB = "/opt/rocm/llvm/lib"


def build() -> str:
    out = os.path.join(HERE, "liboracle_san.so")
    subprocess.check_call([
        CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-shared", "-fPIC",
        "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
        os.path.join(HERE, "mh_oracle.c"), "-o", out,
        "-L" + LLVM_LIB, "-Wl,-rpath," + LLVM_LIB])
    return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)
