import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def ensure_library():
    """Path of the built HIP library; builds it first only if it is missing."""
    from paper_2307_04528_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2307_04528_amd.build import build
        build()
    return _lib.LIB_PATH
