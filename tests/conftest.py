import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def hsd_ctx():
    """One device context for all GPU tests (skips when no GPU is visible)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_06340_amd as hsd
    ctx = hsd.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="session")
def hooks_ctx():
    """(library, context handle) of the test-hooks build of the library, for
    the GPU tests that call its hooks (skips when no GPU is visible)."""
    import ctypes
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_06340_amd import _lib
    L = _lib.load_test_hooks()
    h = ctypes.c_void_p()
    assert L.hsd_init(0, 0, ctypes.byref(h)) == 0, L.hsd_last_error()
    yield L, h
    L.hsd_finalize(h)


def golden_path(name):
    return os.path.join(ROOT, "tests", "golden", name)
