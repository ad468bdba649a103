"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host side only; device code as usual): tests/sanitize/host_driver.cpp calls
every entry point of the C ABI on a small seeded scene and through its error
paths, linked against libxm_hostsan.so (both built by __graft_entry__.build(),
paper_2502_04640_amd/build.py build_hostsan).  The sanitizers abort the driver
on their first finding; the driver exits nonzero when a status or invariant
check fails."""
import os
import subprocess

import pytest

from conftest import ROOT, progress

pytestmark = pytest.mark.gpu

DRIVER = os.path.join(ROOT, "tests", "sanitize", "xm_hostsan_driver")


def test_c_abi_under_host_sanitizers():
    if not os.path.exists(DRIVER):
        pytest.skip("host-sanitizer driver not built (paper_2502_04640_amd.build.build_hostsan)")
    progress("case: C ABI under host ASan + UBSan")
    env = dict(os.environ)
    # the HIP runtime's own allocations are not the library's: no leak report
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([DRIVER], env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout[-6000:])
    print(r.stderr[-6000:])
    assert r.returncode == 0, f"driver exit status {r.returncode}"
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
