import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_library():
    lib = os.path.join(ROOT, "paper_2010_12478_amd", "libregscan.so")
    if not os.path.exists(lib):
        import importlib.util   # build.py by path: the package needs the library to import
        spec = importlib.util.spec_from_file_location(
            "_regscan_build", os.path.join(ROOT, "paper_2010_12478_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()


_ensure_library()
