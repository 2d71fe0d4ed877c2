import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def tiny():
    """Tiny cantilever (4x4 cross-section, 16 long), its oracle model and the
    oracle precompute with 4 cubature samples per vertex."""
    from oracle import correction as oc, fem
    from paper_2506_06494_amd import inputs
    sc = inputs.tiny_beam()
    mdl = fem.model_from_scene(sc)
    tab = oc.precompute(mdl, S=4, n_cand=64, seed=0)
    return sc, mdl, tab
