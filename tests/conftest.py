import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X")
    config.addinivalue_line("markers", "slow: minutes of CPU work")


@pytest.fixture(scope="session")
def tiny_scene():
    import scenegen as sg
    return sg.make_scene("tiny", seed=0)


@pytest.fixture(scope="session")
def tiny_rays(tiny_scene):
    import scenegen as sg
    return sg.sample_rays(tiny_scene, sg.WORKLOADS["tiny"]["rays"], seed=0)
