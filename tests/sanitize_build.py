"""AddressSanitizer and UndefinedBehaviorSanitizer on the host code: builds
the library with its host pass instrumented (device code is compiled as
usual) and the C oracle instrumented, then runs the CPU test suite against
both builds (MDPNOP_LIB and ORACLE_LIB select them; the sanitizer runtime is
preloaded into the interpreter, leak detection is off because the
interpreter itself keeps memory until exit).

Test infrastructure (it builds and runs the oracle), kept beside the tests.

Usage: python tests/sanitize_build.py [pytest arguments]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from paper_2509_01416_amd import build as B  # noqa: E402

OUT = os.path.join(B.CSRC, "_build_asan")
LIB = os.path.join(ROOT, "paper_2509_01416_amd", "libmdpnop_asan.so")
ORACLE_SRC = os.path.join(ROOT, "oracle", "si_oracle.c")
ORACLE_LIB = os.path.join(ROOT, "oracle", "libsi_oracle_asan.so")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
       "-fno-sanitize-recover=undefined"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build() -> None:
    os.makedirs(OUT, exist_ok=True)
    host_san = [a for f in SAN for a in ("-Xarch_host", f)]

    def one(src):
        obj = os.path.join(OUT, src + ".o")
        cmd = [B.HIPCC, *B.COMMON, "-g", *host_san, "-c", os.path.join(B.CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        _run(cmd)
        return obj
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(one, B._sources()))
    _run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *host_san,
          "-shared-libsan", "-o", LIB, *objs])
    _run([CLANG, "-O1", "-g", "-std=c99", "-fPIC", "-shared", *SAN, "-shared-libsan",
          "-o", ORACLE_LIB, ORACLE_SRC, "-lm"])


def runtime() -> str:
    libs = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not libs:
        raise RuntimeError("no clang AddressSanitizer runtime found")
    return libs[0]


def main(argv) -> int:
    build()
    # the sanitizer runtime goes first in the child's preload list; whatever
    # the environment already preloads stays after it
    preload = ":".join(p for p in (runtime(), os.environ.get("LD_PRELOAD", "")) if p)
    env = dict(os.environ, MDPNOP_LIB=LIB, ORACLE_LIB=ORACLE_LIB, LD_PRELOAD=preload,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu",
           "-p", "no:cacheprovider", *argv]
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
