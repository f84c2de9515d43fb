import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


def pytest_sessionfinish(session, exitstatus):
    """A process that ran GPU tests ends right after pytest has reported,
    without interpreter teardown: the HIP runtime bundled with torch and the
    library built by the system compiler are torn down in an order this
    suite does not control, and a segmentation fault was seen there once all
    GPU tests had passed."""
    if "torch" in sys.modules and getattr(sys.modules["torch"], "cuda", None) is not None:
        try:
            ran_gpu = sys.modules["torch"].cuda.is_initialized()
        except Exception:
            ran_gpu = False
        if ran_gpu:
            session.config._h2_exit_status = int(exitstatus)


def pytest_unconfigure(config):
    status = getattr(config, "_h2_exit_status", None)
    if status is not None:
        sys.stdout.flush()
        sys.stderr.flush()
        os._exit(status)
