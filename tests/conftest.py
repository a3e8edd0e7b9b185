import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size workloads")


def pytest_runtest_setup(item):
    # name the case before any GPU work starts, so a run that dies inside a
    # kernel still says which case it was (pytest captures stderr, so the
    # name also goes to the file RADULS_CASE_LOG names, when set)
    if item.get_closest_marker("gpu") is not None:
        line = f"[gpu-case] {item.nodeid}\n"
        sys.__stderr__.write(line)
        sys.__stderr__.flush()
        path = os.environ.get("RADULS_CASE_LOG")
        if path:
            with open(path, "a") as f:
                f.write(line)
                f.flush()
                os.fsync(f.fileno())
