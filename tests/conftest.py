import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libpm.so")
    config.addinivalue_line("markers", "slow: large CPU case")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    """Build the input generator and the oracle if nothing is built yet."""
    from paper_1912_08453_amd import _build
    if not os.path.exists(_build.GEN_LIB):
        _build.build_gen()
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build(force=False)
    yield
