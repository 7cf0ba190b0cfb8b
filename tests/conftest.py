import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def oracle_from_case(case, nthreads=None, **over):
    """Build an OracleSim for a workload dict (paper_1503_08406_amd.workloads).
    The float32 input fields are passed as float64, so both sides of a parity
    check see identical numbers."""
    import oracle
    opts = dict(case["opts"])
    opts.update(over)
    if nthreads is None:
        nthreads = min(8, len(os.sched_getaffinity(0)))
    p = oracle.make_params(case["nx"], case["ny"], H=case["H"], bc_kind=case["bc_kind"],
                           T_wall=case["T_wall"], Ra=case["Ra"], Da=case["Da"],
                           Pr=case["Pr"], Ste=case["Ste"], nthreads=nthreads, **opts)
    K = None if case["K"] is None else case["K"].astype(np.float64)
    F = None if case["Feps"] is None else case["Feps"].astype(np.float64)
    return oracle.OracleSim(p, case["eps"].astype(np.float64), K, F)


def front_rows(fl):
    """Per-row position of the first f_l = 0.5 crossing scanned from x = 0,
    linearly interpolated, measured from the wall one lattice unit left of the
    first node (0 when the row has no crossing)."""
    fl = np.asarray(fl, dtype=np.float64)
    out = np.zeros(fl.shape[0])
    for r in range(fl.shape[0]):
        row = fl[r]
        s0 = row[0] >= 0.5
        idx = np.nonzero((row >= 0.5) != s0)[0]
        if idx.size == 0:
            continue
        i = idx[0]
        a, b = row[i - 1], row[i]
        out[r] = (i - 1) + (a - 0.5) / (a - b) + 1.0
    return out
