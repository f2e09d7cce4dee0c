import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU run")


@pytest.fixture(scope="session", autouse=True)
def _built_inputs():
    """The oracle and the bed generator are plain C/C++ built on first use."""
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    gen = os.path.join(ROOT, "paper_2501_05300_amd", "libbedgen.so")
    if not os.path.exists(gen):
        from paper_2501_05300_amd import build as B
        B.build_bedgen()
    yield
