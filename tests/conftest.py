import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _rfsim_built():
    # the forward-model helper is plain C; build it once if this checkout has not yet
    from paper_2603_22496_amd.phantom import _LIB, build_rfsim
    if not os.path.exists(_LIB):
        build_rfsim(force=False)
    yield
