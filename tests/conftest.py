import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: minutes-scale CPU test")


@pytest.fixture(scope="session")
def tiny_mesh():
    from paper_1906_08125_amd import workloads as w
    return w.config_tiny().mesh()


@pytest.fixture(scope="session")
def plates_mesh():
    """Periodic parallel plates, no tip: 4 x 4 x 8 cubes of 0.5 nm."""
    from paper_1906_08125_amd import workloads as w
    return w.kuhn_tip_mesh(4, 4, 8, 0.5)


@pytest.fixture(scope="session")
def small_tip_mesh():
    """3 x 3 x 4 cubes (216 tets before removal) with a one-cell tip."""
    from paper_1906_08125_amd import workloads as w
    return w.kuhn_tip_mesh(3, 3, 4, 0.5, 0.5, 1.0)


def golden(name):
    """The named fixture of tests/golden/: {key: [fields]} from its
    whitespace-separated lines ('#' starts a comment)."""
    import os
    out = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, *v = line.split()
                out[k] = v
    return out
