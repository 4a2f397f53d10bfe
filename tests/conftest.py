import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    # The oracle is test infrastructure: build it once per session if it is missing.
    lib = os.path.join(ROOT, "oracle", "liborc.so")
    if not os.path.exists(lib):
        from oracle import build as ob
        ob.build()


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    return oracle
