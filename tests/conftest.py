import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libraries():
    """Build the CPU-side libraries (oracle, generator) if they are missing."""
    from oracle import LIB_PATH, build as obuild
    if not os.path.exists(LIB_PATH):
        obuild.build()
    from paper_2510_15095_amd import build as pbuild
    from paper_2510_15095_amd.workload import _LIB_PATH
    if not os.path.exists(_LIB_PATH):
        pbuild.build_workload()
    yield
