import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
# MCLBM_ORACLE_DIR lets a mutation run point the pins at a planted-mistake copy
sys.path.insert(0, os.environ.get("MCLBM_ORACLE_DIR", os.path.join(ROOT, "oracle")))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: oracle physics runs that take more than ~20 s on CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle
