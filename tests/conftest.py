import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def weights_path(tmp_path_factory):
    """The seeded benchmark model (seed 0) written to a temporary weights file."""
    from paper_2604_07276_amd import synth
    p = tmp_path_factory.mktemp("weights") / "dpa1_seed0.bin"
    synth.make_weights(str(p), seed=0)
    return str(p)


@pytest.fixture(scope="session")
def oracle_model(weights_path):
    from oracle import dpa1_oracle
    return dpa1_oracle.load_model(weights_path)
