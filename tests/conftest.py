import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="session")
def ietilib():
    """The built C-ABI library (built in-tree once if it is missing)."""
    from paper_2501_04340_amd import ietidp
    if not os.path.exists(ietidp.library_path()):
        from paper_2501_04340_amd import build
        build.build()
    return ietidp.load_library()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
