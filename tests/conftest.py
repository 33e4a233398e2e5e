import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (gfx950) and the HIP library")
    lib = os.environ.get("TWOFOLD_ORACLE_LIB")
    if lib:
        # the oracle's pins run against another build of it (planted-mistake
        # copies, tests/test_oracle_mutants.py)
        from oracle import build as oracle_build
        oracle_build.build = lambda force=False, quiet=True: lib
    bounds_py = os.environ.get("TWOFOLD_BOUNDS_PY")
    if bounds_py:
        # the bound pins run against another copy of oracle/bounds.py
        # (planted-mistake copies, tests/test_oracle_mutants.py)
        import importlib.util

        import oracle
        spec = importlib.util.spec_from_file_location("oracle.bounds", bounds_py)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        sys.modules["oracle.bounds"] = mod
        oracle.bounds = mod


def _have_gpu():
    if os.environ.get("TWOFOLD_ORACLE_LIB") or os.environ.get("TWOFOLD_BOUNDS_PY"):
        return False  # CPU-only runs of the oracle's pins
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _have_gpu():
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
