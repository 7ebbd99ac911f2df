import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def _ensure_built():
    """Build the CPU-side libraries only if nothing is built yet."""
    import synth
    import oracle
    if not os.path.exists(synth._LIB_PATH):
        synth.build()
    if not all(os.path.exists(p) for p in oracle.lib_paths()):
        oracle.build()


_ensure_built()
