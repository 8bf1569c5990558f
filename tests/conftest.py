import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle check")


def read_golden(name):
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line)
    return rows


def paper_value(key):
    for row in read_golden("paper_values.txt"):
        k, v = [s.strip() for s in row.split("=")]
        if k == key:
            return float(v)
    raise KeyError(key)


@pytest.fixture(scope="session")
def small_problem():
    import oracle
    import tc_inputs
    cfg = tc_inputs.CONFIGS["small"]
    P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
    return P, cfg


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(1234))
