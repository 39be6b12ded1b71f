import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def ora():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def fb():
    """The HIP library binding; GPU tests only."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_1157_amd import fewbody
    return fewbody


@pytest.fixture
def plans(fb):
    """The library's plan table, restored after the test."""
    saved = {n: fb.get_plan(n) for n in [0] + list(range(2, 17))}
    yield fb
    for n, (m, w, g) in saved.items():
        fb.set_plan(n, m, w, g)
