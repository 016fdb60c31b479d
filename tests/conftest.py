import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


def _ensure_library():
    lib = os.path.join(ROOT, "paper_2502_07754_amd", "libmsp.so")
    if not os.path.exists(lib):
        from paper_2502_07754_amd import build
        build.build()
    return lib


@pytest.fixture(scope="session")
def libmsp_path():
    return _ensure_library()


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0; GPU tests fail (not skip) when it cannot load."""
    import torch
    _ensure_library()
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2502_07754_amd as msp
    msp.load_library()
    torch.cuda.set_device(0)
    return msp
