import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def small_mesh():
    import casegen as cg
    return cg.config_mesh(cg.CONFIGS["small"])


@pytest.fixture(scope="session")
def small_case(small_mesh):
    import casegen as cg
    return cg.make_case(small_mesh, cg.CONFIGS["small"])


@pytest.fixture(scope="session")
def jitter_mesh():
    import casegen as cg
    return cg.box_mesh(40.0, 30.0, 20.0, 10.0, jitter=0.2, seed=7)
