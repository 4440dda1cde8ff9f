import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def small_geom():
    """A 24^3 scan scaled from the 64^3 one (fast oracle runs)."""
    from workloads import Geometry
    return Geometry(24, 24, 24, 4.0, 4.0, 4.0, 48, 36, 3.2, 3.2, 1000.0, 1500.0, 8)
