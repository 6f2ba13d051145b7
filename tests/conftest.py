import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU-only check")


_CACHE = {}


def workload(name, seed=0, **kw):
    """Seeded workloads are deterministic; cache them per test session."""
    from workloads import make_workload
    key = (name, seed, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = make_workload(name, seed=seed, **kw)
    return _CACHE[key]


_ORC = {}


def oracle_run(name, seed=0, **kw):
    from oracle import oracle as O
    key = (name, seed, tuple(sorted(kw.items())))
    if key not in _ORC:
        _ORC[key] = O.run_pipeline(workload(name, seed, **kw))
    return _ORC[key]


# small variants of the three plain workloads that the oracle finishes in seconds
SMALL = {
    "shadow_128": {},
    "refl_96": dict(W=96, H=96),
    "mixed_128x72": dict(W=128, H=72, n_meshes=48),
}


def small(name, seed=0):
    base = {"shadow_128": "shadow_128", "refl_96": "refl_1024", "mixed_128x72": "mixed_1080p"}[name]
    return base, SMALL[name]


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(1234)
