import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds on the CPU")


_HIP_UP = False


@pytest.fixture(autouse=True)
def _torch_hip_context_first(request):
    """Before the first GPU test, bring up torch's HIP context (and wait for the
    device) so that the library's first runtime call finds it initialised, as
    it does under the benchmark and the smoke test."""
    global _HIP_UP
    if not _HIP_UP and request.node.get_closest_marker("gpu") is not None:
        import torch
        if torch.cuda.is_available():
            torch.empty(1, device="cuda")
            torch.cuda.synchronize()
        _HIP_UP = True
    yield
