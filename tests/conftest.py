import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Names every GPU test on stderr before it touches the device."""
    if request.node.get_closest_marker("gpu") is not None:
        sys.__stderr__.write(f"\n[gpu case] {request.node.nodeid}\n")
        sys.__stderr__.flush()
    yield


@pytest.fixture(scope="session")
def device():
    import torch
    import paper_1907_09529_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()  # raises when the HIP library is missing: no fallback path exists
    torch.cuda.set_device(0)
    return torch.device("cuda:0")
