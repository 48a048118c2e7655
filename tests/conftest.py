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
def op0():
    """Oracle operator of workload 0 (2 x 2 plates in 0.5 wavelength boxes)."""
    from oracle.system import OracleOperator
    from synth import make_workload
    return OracleOperator(make_workload(0))


@pytest.fixture(scope="session")
def dense0(op0):
    """Dense Galerkin brute force for workload 0, rows of element 0 only."""
    from oracle.galerkin import efie_dense
    wl = op0.wl
    return efie_dense(op0.geo, wl.elem_center(), wl.k, wl.eta, rows=range(op0.nb))
