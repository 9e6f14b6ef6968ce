import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running test")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """Skip-free GPU fixture: a gpu-marked test on a machine without a GPU fails loudly."""
    if not _gpu_available():
        pytest.fail("gpu test selected but no GPU is visible")
    from paper_2104_12916_amd import qpgpu
    qpgpu.lib()
    return qpgpu
