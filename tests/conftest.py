import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libvie")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


@pytest.fixture(scope="module", autouse=True)
def _hand_device_memory_back():
    """After each test module: destroy the library contexts that only cyclic
    garbage still holds (a pytest.raises frame keeps its test's locals), then
    return torch's cached device memory to the device.  The full-size modules
    bind workspaces of up to 239 GB through torch; kept in its cache, that
    memory would leave the HIP runtime's own allocations (queues, scratch,
    FFT plans) of every later module only the remainder of the 288 GB."""
    yield
    import gc
    gc.collect()
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
