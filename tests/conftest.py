import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def vgx():
    """The ctypes binding; GPU tests need it and a visible device."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2302_03343_amd.vgx as binding
    return binding


@pytest.fixture(scope="session")
def c1_grid():
    from synth import synthetic_pdf_grid
    return synthetic_pdf_grid()


@pytest.fixture(scope="session")
def pdf_ctx(vgx, c1_grid):
    h = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    yield h
    vgx.pdf_destroy(h)


def report(msg):
    """Flush a line naming the GPU case before it runs."""
    print(msg, flush=True)
