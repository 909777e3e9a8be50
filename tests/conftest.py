import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU checks")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def fe_pot(orc):
    from paper_1107_2619_amd import inputs

    return orc.Potential(inputs.perturbed_potential("fe_fs", 1))


@pytest.fixture(scope="session")
def fec_pot(orc):
    from paper_1107_2619_amd import inputs

    return orc.Potential(inputs.perturbed_potential("fec_eam", 4))


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
