import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (dense eigen-decompositions or many samples)")


@pytest.fixture(autouse=True)
def _library_options_back_to_defaults():
    """The library's kernel-selection options are process-wide: a test that
    sets one leaves the next test the defaults again (only when the binding
    was loaded; nothing is imported here)."""
    yield
    L = sys.modules.get("paper_2306_09559_amd._lib")
    if L is not None:
        for opt, value in ((L.OPT_PLANE_SWEEP, L.SWEEP_AUTO), (L.OPT_SWEEP_RANK, 0), (L.OPT_HOP_SLAB, 1),
                           (L.OPT_LINK_BUF, 1), (L.OPT_SWEEP_CHUNKS, 0)):
            L.set_option(opt, value)
