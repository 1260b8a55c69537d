import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running test")


def _flush_print(*a):
    print(*a, flush=True)


@pytest.fixture(autouse=True)
def _name_the_case(request):
    # Print the test's name before it runs so that a run that dies on the GPU
    # still names the case that was running.
    if request.node.get_closest_marker("gpu") is not None:
        _flush_print("\n[case]", request.node.nodeid)
    yield
