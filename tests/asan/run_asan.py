#!/usr/bin/env python3
"""Build the library with AddressSanitizer on its host code (device code unchanged) and run the
host-only ABI driver against it. Used by tests/test_host_asan.py; no GPU is needed or touched.
Prints the driver's output; exit status 0 when the driver passes with no sanitizer report."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2502_21013_amd import build as B  # noqa: E402

OUT = os.path.join(ROOT, "_build", "asan")
LLVM = os.environ.get("ROCM_LLVM", "/opt/rocm/llvm/bin")


def main() -> int:
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libptsolve_asan.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    cmd = [hipcc, *B.HIPCC_FLAGS, *san, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2502_21013_amd", "csrc"), *B.sources(), "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stdout + r.stderr)
        return 2
    drv = os.path.join(OUT, "abi_host_driver")
    cmd = [os.path.join(LLVM, "clang"), "-fsanitize=address", "-fno-omit-frame-pointer", "-g", "-std=c11",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_host_driver.c"),
           "-L", OUT, "-lptsolve_asan", "-Wl,-rpath," + OUT, "-o", drv]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stdout + r.stderr)
        return 3
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=7",
               LSAN_OPTIONS="suppressions=" + os.path.join(HERE, "lsan.supp"))
    r = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout + r.stderr)
    return r.returncode


if __name__ == "__main__":
    sys.exit(main())
