"""GPU tests of the discrete adjoint (dmrt_record / dmrt_adjoint): gradients
of a functional of the final T and f_l fields with respect to per-cell
log K and porosity, against central finite differences of the FP64 oracle
on tiny grids (conduction melting; convection melting with nodes melting
during the run; a liquid cavity with strong buoyancy freezing at the cold
wall), with the contract's relative error bound of 1e-3."""
import sys

import numpy as np
import pytest

from conftest import oracle_from_case
from paper_1503_08406_amd import workloads as W

pytestmark = pytest.mark.gpu

FD_TOL = 1e-3  # relative to the largest FD gradient component


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(kind):
    """Tiny melting problems with random porosity and log-normal permeability."""
    nx, ny = 16, 12
    rng = np.random.default_rng({"conduction": 21, "convection": 22, "liquid": 23}[kind])
    eps = rng.uniform(0.35, 0.6, (ny, nx))
    if kind == "conduction":
        H = float(ny)
        K = 1e-2 * H * H * np.exp(0.5 * rng.standard_normal((ny, nx)))
        case = W.make_case("adj_conduction", nx, ny, [1, 2, 2, 2], [1.0, 0, 0, 0], Ra=0.0,
                           Da=1e-2, Pr=1.0, Ste=1.0, eps=eps, K=K, T_init=-0.06, T_s=-0.02,
                           T_l=0.02, alpha_l=0.05, convective=0)
        steps = 80
    elif kind == "liquid":
        # liquid cavity with strong buoyancy, freezing at the cold wall: the
        # permeability acts on T and f_l through the flow
        H = 16.0
        K = 1.0 * H * H * np.exp(0.5 * rng.standard_normal((ny, nx)))
        case = W.make_case("adj_liquid", nx, ny, [1, 1, 2, 2], [1.0, 0, 0, 0], Ra=3e3, Da=1.0,
                           Pr=1.0, Ste=1.0, eps=eps, K=K, H=H, T_init=0.45, T_s=0.38, T_l=0.42,
                           convective=1, Ma=0.3)
        steps = 200
    else:
        H = 64.0
        K = 5e-3 * H * H * np.exp(0.5 * rng.standard_normal((ny, nx)))
        case = W.make_case("adj_convection", nx, ny, [1, 1, 2, 2], [1.0, 0, 0, 0], Ra=2e4,
                           Da=5e-3, Pr=1.0, Ste=1.0, eps=eps, K=K, H=H, T_init=0.375, T_s=0.38,
                           T_l=0.42, convective=1)
        steps = 120
    wT = rng.standard_normal((ny, nx)).astype(np.float32)
    wf = rng.standard_normal((ny, nx)).astype(np.float32)
    return case, steps, wT, wf


def _oracle_functional(case, steps, wT, wf, eps, K):
    c = dict(case)
    c["eps"], c["K"] = eps, K
    o = oracle_from_case(c, nthreads=1)
    o.step(steps)
    F = o.fields()
    return float(np.sum(wT.astype(np.float64) * F["T"]) + np.sum(wf.astype(np.float64) * F["fl"]))


def _fd_gradients(case, steps, wT, wf, h_k=1e-5, h_e=1e-6):
    eps0 = case["eps"].astype(np.float64)
    K0 = case["K"].astype(np.float64)
    gk = np.zeros(eps0.shape)
    ge = np.zeros(eps0.shape)
    for idx in np.ndindex(eps0.shape):
        for sgn in (1, -1):
            K = K0.copy()
            K[idx] *= np.exp(sgn * h_k)
            gk[idx] += sgn * _oracle_functional(case, steps, wT, wf, eps0, K) / (2 * h_k)
            e = eps0.copy()
            e[idx] += sgn * h_e
            ge[idx] += sgn * _oracle_functional(case, steps, wT, wf, e, K0) / (2 * h_e)
    return gk, ge


@pytest.mark.parametrize("kind", ["conduction", "convection", "liquid"])
def test_adjoint_matches_oracle_finite_differences(kind):
    from paper_1503_08406_amd.dmrt import Solver
    case, steps, wT, wf = _case(kind)
    s = Solver(case, fl_tol=1e-7)
    s.record(steps)
    F = s.fields()
    assert (F["fl"] > 0).sum() >= 10 and ((F["fl"] > 0) & (F["fl"] < 1)).sum() > 0
    gk, ge = s.adjoint(wT, wf)
    _say(kind, "GPU gradients done; liquid", int((F["fl"] > 0).sum()))
    fk, fe = _fd_gradients(case, steps, wT, wf)
    ek = np.abs(gk - fk).max() / max(np.abs(fk).max(), 1e-30)
    ee = np.abs(ge - fe).max() / max(np.abs(fe).max(), 1e-30)
    _say(kind, "max |dL/dlogK| %.3e err %.2e; max |dL/deps| %.3e err %.2e"
         % (np.abs(fk).max(), ek, np.abs(fe).max(), ee))
    assert ee <= FD_TOL
    if kind == "conduction":
        assert np.abs(gk).max() == 0.0  # no flow: permeability does not enter
    else:
        assert np.abs(fk).max() > 0 and ek <= FD_TOL
    # the state of the handle is unchanged by the adjoint
    F2 = s.fields()
    for k in F:
        assert np.array_equal(F[k], F2[k])
