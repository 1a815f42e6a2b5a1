import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def field_cache():
    """Seeded synthetic fields, generated once per session."""
    from paper_1412_1498_amd import synth
    cache = {}

    def get(dims, amp, seed):
        key = (tuple(dims), float(amp), int(seed))
        if key not in cache:
            cache[key] = synth.random_gauge_field(dims, amp, seed).numpy()
        return cache[key].copy()
    return get
