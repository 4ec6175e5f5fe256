import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    if not gpu_available():
        pytest.skip("no GPU visible")
    import torch
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _collect_plans(request):
    # Plans, pools and batches held by reference cycles (pytest.raises keeps
    # the test frame alive through the exception's traceback) are destroyed
    # when the test ends, not at whatever later allocation triggers the
    # garbage collector.
    yield
    if request.node.get_closest_marker("gpu") is not None:
        import gc
        gc.collect()
