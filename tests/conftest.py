import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        from oracle import build
        build.build()
    oracle.set_threads(min(8, os.cpu_count() or 1))
    return oracle


def rel_l1(a: np.ndarray, b: np.ndarray, scale_floor: float = 0.0) -> np.ndarray:
    """Per-variable relative L1 distance sum|a-b| / sum|b| over the cells."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    num = np.abs(a - b).sum(axis=1)
    den = np.abs(b).sum(axis=1)
    return num / np.maximum(den, scale_floor)
