import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# ---- helpers shared by the tests (no arithmetic of the method here) ---------------

def to_int(limbs) -> int:
    """Little-endian u32 limbs -> Python int (Python's own bignum arithmetic)."""
    limbs = np.asarray(limbs, dtype=np.uint32)
    return int.from_bytes(limbs.astype("<u4").tobytes(), "little")


def from_int(x: int, n: int) -> np.ndarray:
    """Python int (0 <= x < 2^(32n)) -> n little-endian u32 limbs."""
    assert 0 <= x < (1 << (32 * n)) or n == 0
    return np.frombuffer(x.to_bytes(4 * n, "little"), dtype="<u4").astype(np.uint32)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle
