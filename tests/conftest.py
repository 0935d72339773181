import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def _gpu_present() -> bool:
    # no HIP call and no torch during collection: the GPU tests load libpms
    # (system ROCm) themselves, and the torch wheel bundles a second HIP
    # runtime under the same soname
    return os.path.exists("/dev/kfd") and os.path.exists("/dev/dri")


def pytest_collection_modifyitems(config, items):
    if _gpu_present():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    from oracle import oracle as _o
    if not os.path.exists(_o.library_path()):
        _o.build()
    return oracle
