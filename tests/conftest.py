import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(autouse=True)
def _automatic_launch_plans():
    """Launch-plan overrides a test sets (emri.set_tuning) end with it."""
    yield
    E = sys.modules.get("paper_2311_17174_amd.emri")
    if E is not None:
        E.set_tuning()
