import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    # the oracle's element and vertex loops on the host cores (same results for any count)
    import oracle
    oracle.set_threads(min(16, os.cpu_count() or 1))


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_spd(r, n=3, cond=6.0):
    """Random SPD matrix with eigenvalues in [1, cond] (scaled), float64."""
    A = r.normal(size=(n, n))
    Qm, _ = np.linalg.qr(A)
    ev = np.exp(r.uniform(0, np.log(cond), size=n))
    return (Qm * ev) @ Qm.T
