import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-only check")


@pytest.fixture(scope="session", autouse=True)
def _torch_device_first():
    """GPU sessions: let torch create its HIP context before the library's
    first call, so torch's cached device count is taken on a clean start."""
    try:
        import torch
    except Exception:  # pragma: no cover
        yield
        return
    if torch.cuda.is_available():
        torch.cuda.init()
        torch.zeros(1, device="cuda")
        torch.cuda.synchronize()
    yield
