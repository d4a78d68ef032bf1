import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")


def cell_dict(nh, tgas, tdust, y_h2, y_e, n_euv=0.0, n_fuv=0.0, z=1.0, eir=None):
    """SoA dict for cells given scalars or arrays (inputs built like the
    workload generator: internal energy from the gas temperature)."""
    from paper_2604_21438_amd.workloads import internal_energy
    arrs = np.broadcast_arrays(*[np.atleast_1d(np.asarray(x, np.float64)) for x in
                                 (nh, tgas, tdust, y_h2, y_e, n_euv, n_fuv, z)])
    nh, tgas, tdust, y_h2, y_e, n_euv, n_fuv, z = [np.ascontiguousarray(a.copy()) for a in arrs]
    d = dict(nh=nh, n_euv=n_euv, n_fuv=n_fuv, zmet=z, y_h2=y_h2, y_e=y_e,
             eint=internal_energy(nh, y_h2, y_e, tgas), tdust=tdust)
    if eir is None:  # the CMB's field (the value FIXED IR holds), evolved from there
        from paper_2604_21438_amd.workloads import A_RAD, C_RED, T_CMB
        eir = A_RAD * T_CMB ** 4 / C_RED
    d["eir"] = np.ascontiguousarray(np.broadcast_to(np.asarray(eir, np.float64), nh.shape).copy())
    return d


@pytest.fixture(scope="session")
def golden():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as f:
        return json.load(f)
