import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: oracle checks that take more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a device; skip them loudly when there is none so that a
    # CPU run never mistakes a skipped kernel test for a passing one.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no HIP device in this process")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
