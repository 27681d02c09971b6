import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: statistical oracle checks that take tens of seconds")


@pytest.fixture(scope="session")
def torch_threads():
    import torch
    torch.set_num_threads(max(1, min(8, os.cpu_count() or 1)))
    return torch
