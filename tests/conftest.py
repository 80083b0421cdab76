import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large inputs; minutes of CPU time")


def pytest_collection_modifyitems(config, items):
    # GPU tests are collected after the CPU tests of the same run.
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def sg():
    import scenegen
    scenegen.build(force=False)
    return scenegen


@pytest.fixture(scope="session")
def starnt():
    """The product binding; builds libstarnt.so first when it is missing."""
    import os
    lib = os.path.join(ROOT, "paper_2606_16747_amd", "libstarnt.so")
    if not os.path.exists(lib):
        # the build script is loaded by its path: importing it through the
        # package would run __init__, which needs the library
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_starnt_build", os.path.join(ROOT, "paper_2606_16747_amd", "build.py"))
        b = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(b)
        b.build()
    import paper_2606_16747_amd as m
    return m


@pytest.fixture(scope="session")
def gpu(starnt):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    return torch.device("cuda:0")
