import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def weights_dir(tmp_path_factory):
    d = os.environ.get("TD_WEIGHTS_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        return d
    return str(tmp_path_factory.mktemp("tdw"))


@pytest.fixture(scope="session")
def weights(weights_dir):
    from synth.models import cached_weights

    def get(config, seed=0):
        return cached_weights(config, weights_dir, seed)
    return get
