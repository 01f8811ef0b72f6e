import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _torch_runtime_first(request):
    """With GPU tests selected, start torch's HIP runtime before the
    library's (torch ships its own runtime beside the one the library links;
    started in that order, as bench.py does, both see the device, while
    torch started after many library calls has reported no GPU)."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        import torch
        if torch.cuda.is_available():
            torch.empty(1, device="cuda:0")
            torch.cuda.synchronize()
    yield
