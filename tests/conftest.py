import os
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# One line per GPU test start and end (and per progress note of a long test)
# in gpurun_out/pytest_progress.log: a run whose stdout is captured still
# shows that it is alive.
PROGRESS = os.path.join(ROOT, "gpurun_out", "pytest_progress.log")


def progress(msg):
    try:
        os.makedirs(os.path.dirname(PROGRESS), exist_ok=True)
        with open(PROGRESS, "a") as f:
            f.write(f"{time.strftime('%H:%M:%S')} {msg}\n")
    except OSError:
        pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_runtest_logstart(nodeid, location):
    if "test_gpu" in nodeid or "test_zz" in nodeid:
        progress(f"start {nodeid}")


def pytest_runtest_logfinish(nodeid, location):
    if "test_gpu" in nodeid or "test_zz" in nodeid:
        progress(f"end {nodeid}")
