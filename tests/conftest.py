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
    config.addinivalue_line("markers", "slow: longer CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def device_table(orc):
    """The oracle's acceptance table in the library's device layout: Ising
    keeps the rows of even k and the columns of even dk ([N+1][5]); Potts and
    the multimagnetic table are laid out alike already."""
    return orc.T[::2, ::2] if orc.model == 0 else orc.T


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()
