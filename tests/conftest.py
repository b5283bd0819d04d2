import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")


@pytest.fixture(scope="session")
def model_cache():
    """Seeded synthetic systems, built once per session."""
    from synth import make_model
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = make_model(name)
        return cache[name]
    return get
