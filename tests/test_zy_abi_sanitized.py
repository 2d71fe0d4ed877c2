"""The C ABI driven end to end from C (tests/abi_driver.c) against the
library built with AddressSanitizer and UBSan on its host code
(`python -m paper_2506_06494_amd.build --sanitize`): every call returns its
documented status and the sanitisers report nothing.  Skipped when the
sanitised build is absent."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "paper_2506_06494_amd", "abi_driver_san")


def test_abi_driver_under_host_sanitizers(tmp_path):
    if not os.path.exists(DRIVER):
        pytest.skip("sanitised build not present")
    env = dict(os.environ)
    # the HIP runtime keeps process-lifetime allocations: leak reports off
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([DRIVER, str(tmp_path)], env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout)
    print(r.stderr[-4000:])
    assert r.returncode == 0
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
