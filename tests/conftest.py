import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU case")


@pytest.fixture(scope="session")
def geom():
    from paper_2102_08862_amd import synth
    synth.build()
    return synth.geometry()


@pytest.fixture(scope="session")
def ocfg(geom):
    import oracle
    oracle.build()
    return oracle.Config(row_x=geom[0])
