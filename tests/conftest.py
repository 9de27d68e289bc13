import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the GPU)")
    config.addinivalue_line("markers", "slow: large CPU-only case")


def _ensure_native():
    """Build the in-tree libraries once if they are missing (CPU-only runs)."""
    lib = os.path.join(ROOT, "paper_1507_05086_amd", "libcc.so")
    if not os.path.exists(lib):
        import importlib.util
        path = os.path.join(ROOT, "paper_1507_05086_amd", "build.py")
        spec = importlib.util.spec_from_file_location("_cc_build", path)
        ccbuild = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(ccbuild)  # not through the package: that would load libcc.so
        ccbuild.build()


_ensure_native()
