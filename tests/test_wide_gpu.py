"""The largest lattices: when an f array passes 4 GB the step kernels
address memory with 64-bit offsets instead of 32-bit buffer offsets.  A
periodic 10496 x 10304 lattice (f arrays of 4.3 GB, 16 GB of state) holding
a state with period 64 in x and y evolves exactly as the 64 x 64 periodic
lattice of one period: every 64 x 64 block of the large result equals the
small result bit for bit, for the default model, the sigma/k_e variants and
the source before streaming.  The small lattice itself is checked against
the oracle."""
import sys

import numpy as np
import pytest

from parity_util import pair
from paper_1503_08406_amd import workloads as W

pytestmark = pytest.mark.gpu

N, RX, RY = 64, 164, 161  # period, repeats in x and y: 10496 x 10304


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases(**opts):
    rng = np.random.default_rng(31)
    eps = rng.uniform(0.3, 0.7, (N, N))
    K = 2e-3 * 64 * 64 * np.exp(0.3 * rng.standard_normal((N, N)))
    o = dict(T_init=0.4, T_s=0.38, T_l=0.42, convective=1)
    o.update(opts)
    mk = lambda nx, ny, e, k: W.make_case("periodic", nx, ny, [0] * 4, [0] * 4, Ra=2e5, Da=2e-3,
                                          Pr=1.0, Ste=0.8, eps=e, K=k, H=64, **o)
    return mk(N, N, eps, K), mk(N * RX, N * RY, np.tile(eps, (RY, RX)), np.tile(K, (RY, RX)))


def _blocks(a):
    return a.reshape(RY, N, RX, N)


@pytest.mark.parametrize("var", [
    {}, dict(sigma_mode=1, cps_ratio=0.93, cm_ratio=1.2, ke_mode=1, ks_ratio=2.0, km_ratio=3.0),
    dict(latent_mode=1, fl_maxit=400)], ids=["default", "sigma_ke", "r2"])
def test_wide_lattice_equals_its_period(oracle_mod, var):
    from paper_1503_08406_amd.dmrt import Solver
    L = oracle_mod.lattice()
    small, big = _cases(**var)
    f, g, fl = W.random_state(N, N, 9, L["w9"], L["w5"])
    # R2 sweeps to FP32 stationarity (its FP32 residual accumulates, see
    # the R2 step test); R1 stops at 1e-7
    tol = 1e-9 if var.get("latent_mode") else 1e-7
    s, o = pair(small, gpu_over=dict(fl_tol=tol))
    s.set_state(f, g, fl)
    o.set_state(f.astype(float), g.astype(float), fl.astype(float))
    s.step(3)
    o.step(3)
    Fs, Fo = s.fields(), o.fields()
    assert np.abs(Fs["fl"] - Fo["fl"]).max() < 2e-5 and np.abs(Fs["T"] - Fo["T"]).max() < 2e-5
    _say("wide", var, "building", big["nx"], "x", big["ny"])
    b = Solver(big, fl_tol=tol)
    b.set_state(np.tile(f, (1, RY, RX)), np.tile(g, (1, RY, RX)), np.tile(fl, (RY, RX)))
    b.step(3)
    Fb = b.fields()
    b.close()
    for k in Fs:
        blk = _blocks(Fb[k])
        assert np.array_equal(blk, np.broadcast_to(Fs[k][None, :, None, :], blk.shape)), k
    _say("wide", var, "all", RX * RY, "blocks equal")
