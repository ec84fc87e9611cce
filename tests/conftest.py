import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def synth():
    """One GPU context (1 GiB torch workspace) shared by the GPU tests."""
    import paper_2504_18943_amd as m
    s = m.Synthesizer(device=0, workspace_bytes=1 << 30)
    yield s
    s.close()
