"""The library's host code (plan validation, layout, tables, launch-bounds check, error paths)
under AddressSanitizer: tests/asan/run_asan.py builds libptsolve with -fsanitize=address on the
host side only and runs a C driver through the host-only entry points of the ABI. No GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_host_paths_are_clean_under_asan():
    script = os.path.join(ROOT, "tests", "asan", "run_asan.py")
    if not os.path.exists(script):
        pytest.skip("sanitizer driver not present")
    r = subprocess.run([sys.executable, script], capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert "AddressSanitizer" not in r.stdout and "LeakSanitizer" not in r.stdout
