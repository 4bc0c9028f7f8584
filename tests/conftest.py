import copy
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def tiny():
    import workloads
    from oracle.fmm import Setup
    wl = workloads.tiny_chain()
    C = wl.orbitals()
    return wl, C, Setup(wl.system, wl.params)


def with_params(wl, **kw):
    p = copy.copy(wl.params)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def small_sheet(lmax=2, depth=3):
    """C24H12-like flake (n=2 hexagonal flake), s+p basis, 2-D tree."""
    import workloads
    wl = workloads.graphene_flake(n=2, lmax=lmax, nocc=12, depth=depth)
    return wl


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
