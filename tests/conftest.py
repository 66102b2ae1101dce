import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on cuda:0)")
    config.addinivalue_line("markers", "slow: long CPU run (oracle pins that march to a steady state)")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Build the CPU oracle once per session if it is missing."""
    from oracle import build as obuild
    if not os.path.exists(obuild.LIB):
        obuild.build()
    yield


@pytest.fixture(scope="session", autouse=True)
def _library_built():
    """Build libcplb.so (hipcc cross-compiles for gfx950 without a GPU) once
    per session if a fresh checkout lacks it; a GPU run never builds."""
    from paper_2402_15752_amd import build as lbuild
    if not os.path.exists(lbuild.LIB) and os.path.exists("/opt/rocm/bin/hipcc"):
        import torch
        if not torch.cuda.is_available():
            lbuild.build()
    yield
