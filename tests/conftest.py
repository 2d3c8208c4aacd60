import gc
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # tuned launch shapes go to a file of this run, not the user's cache
    import tempfile
    os.environ.setdefault("COLA_TUNE_CACHE",
                          os.path.join(tempfile.mkdtemp(prefix="cola_tune_"), "hop_tune.txt"))
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(autouse=True)
def _release_device_memory(request):
    """After each GPU test: drop its tensors and hand torch's cached device memory back, so
    the library's own allocations in the next test (tens of GB at 48^3 x 96) find it."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    gc.collect()
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
