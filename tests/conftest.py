import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long statistical or end-to-end test")


@pytest.fixture(scope="session")
def sw_params():
    from paper_2103_10449_amd.inputs import SW_SILICON
    return dict(SW_SILICON)
