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


def _ensure_libs():
    """Builds what is not built yet (input generator and oracle with gcc, the
    decomposer with hipcc); a library that exists is loaded as it is."""
    import oracle
    import workload
    if not os.path.exists(workload._LIB_PATH):
        workload.build()
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build()
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_mpld_build", os.path.join(ROOT, "paper_2303_14335_amd", "build.py"))
    mbuild = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mbuild)
    if not os.path.exists(mbuild.LIB):
        mbuild.build()


_ensure_libs()


@pytest.fixture(scope="session")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 device"
    import paper_2303_14335_amd as mp
    c = mp.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()
