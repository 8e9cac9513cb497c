import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def problem_cache():
    """Session cache of generated problems keyed by (name, seed)."""
    import synth

    cache = {}

    def get(name, seed=None):
        key = (name, seed)
        if key not in cache:
            cache[key] = synth.make_problem(name, seed)
        return cache[key]

    return get
