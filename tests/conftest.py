import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C-ABI)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O

    O.lib()
    return O


@pytest.fixture(scope="session")
def inputs():
    from paper_2504_00340_amd import inputs as I

    return I


@pytest.fixture(scope="session")
def c1_oracle(oracle_mod, inputs):
    """Config 1 run through the oracle once per session: (config, Oracle, dose, final state)."""
    c = inputs.config1()
    o = oracle_mod.Oracle(c["grid"], c["phys"])
    dose, fin = o.run(c["beam"], c["rho"])
    return c, o, dose, fin


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
