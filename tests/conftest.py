import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU statistical test")


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")


def pytest_runtest_logstart(nodeid, location):
    """Name every GPU case on stderr before it runs (flushed), so a run that ends the box
    still says which case was running."""
    if "gpu" in nodeid:
        sys.__stderr__.write(f"\n[start] {nodeid}\n")
        sys.__stderr__.flush()


def pytest_collection_modifyitems(config, items):
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="needs a GPU")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
