import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _ensure_host_libs():
    """The host-only C libraries (input generator, oracle) are built with gcc
    when nothing is built yet; the HIP library is never built here."""
    import oracle
    import workload
    if not os.path.exists(workload._LIB_PATH):
        workload.build()
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build()


_ensure_host_libs()
