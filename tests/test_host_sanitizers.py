"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU needed): python -m paper_2604_20731_amd.build --sanitize builds the
host side of every library source with both sanitizers, links the
csrc/abi_check.cpp driver and runs it.  The driver walks every argument and
configuration error path of include/crv.h and requires the documented status
from each; any sanitizer report (leaks included) fails the run."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_abi_error_paths_clean_under_asan_and_ubsan():
    if not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    res = subprocess.run([sys.executable, "-m", "paper_2604_20731_amd.build", "--sanitize"],
                         cwd=ROOT, capture_output=True, text=True, timeout=1150)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert res.returncode == 0, out[-3000:]
    assert "abi_check: all checks passed" in out
    assert "Sanitizer" not in out
