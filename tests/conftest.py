import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(autouse=True)
def _release_cached_device_memory():
    """Before each test, hand the device memory that earlier tests' tensors
    left in torch's caching allocator back to the device: the solves of the
    large lattices size their columns in flight from the free device memory.
    Does nothing unless a GPU test has already initialised the device."""
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        import gc
        gc.collect()
        torch.cuda.empty_cache()
    yield
