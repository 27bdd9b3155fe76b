import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built liblbpf.so")
    config.addinivalue_line("markers", "slow: long CPU run of the oracle")


@pytest.fixture(autouse=True)
def _announce(request):
    # Name the case before it touches the GPU, so a lost box still says which.
    if request.node.get_closest_marker("gpu"):
        print("\n[gpu-case] %s" % request.node.nodeid, flush=True)
    yield
