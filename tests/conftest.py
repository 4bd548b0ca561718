import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # GPU tests cannot run without a GPU; make that explicit instead of erroring
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture
def live(request):
    """Context manager that lets a long test's progress lines (and the library's own
    HODBF_LOG messages on stderr) reach the terminal while pytest captures output."""
    import contextlib

    capman = request.config.pluginmanager.getplugin("capturemanager")

    @contextlib.contextmanager
    def ctx():
        if capman is None:
            yield
            return
        with capman.global_and_fixture_disabled():
            yield

    return ctx
