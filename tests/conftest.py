import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True)
def _release_device_cache(request):
    """After each GPU test, give the library's idle cached device blocks back,
    so that one test's scratch does not crowd the next test's tensors."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    mod = sys.modules.get("paper_2102_02989_amd.rsgdf")
    if mod is not None and getattr(mod, "_lib", None) is not None:
        mod.release_cache()
