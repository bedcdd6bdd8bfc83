import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(autouse=True)
def _device_checks(request):
    """With a device-check build of the library (GS2D_LIB naming libgs2d_checked.so),
    every GPU test ends by asserting that no kernel check failed in any open context."""
    yield
    if "gpu" not in request.keywords:
        return
    ras = sys.modules.get("paper_2506_00970_amd.rasterizer")
    if ras is None:
        return
    from paper_2506_00970_amd import _lib

    if not (_lib.load().gs2d_build_info() & _lib.BUILD_DEVICE_CHECKS):
        return
    for r in list(ras.LIVE):
        if r._ctx is not None:
            bits = r.counts()["device_checks"]
            assert bits == 0, f"device checks failed: bits {bits:#x}"


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle.build()
    return oracle
