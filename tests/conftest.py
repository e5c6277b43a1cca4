import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library binding; skips when no GPU is visible."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_21379_amd import binding
    return binding.lib()


@pytest.fixture(autouse=True)
def _announce(request):
    """Name the case on the real stderr (not captured) before it runs, so the
    last line printed identifies the test if a GPU step never returns."""
    if request.node.get_closest_marker("gpu"):
        sys.__stderr__.write(f"\n[gpu-case] {request.node.nodeid}\n")
        sys.__stderr__.flush()
    yield
