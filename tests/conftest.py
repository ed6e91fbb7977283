import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")
    # The generator and the oracle are plain C built with gcc; build them if
    # this checkout has not been built yet (cheap, CPU only).
    for mod in ("synth", "oracle"):
        lib = os.path.join(ROOT, mod, f"lib{mod}.so")
        if not os.path.exists(lib):
            import importlib
            importlib.import_module(f"{mod}.build").build()


@pytest.fixture(scope="session")
def root():
    return ROOT
