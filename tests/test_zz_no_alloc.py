"""dmrt_diag_noalloc (the diagnostics entry point for callers that cannot
allocate device memory) against dmrt_diag, through the C ABI: identical
results on two calls in a row, the second on a smaller lattice, and a clear
error for a lattice beyond the fixed scratch array."""
import sys

import numpy as np
import pytest

from paper_1503_08406_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    for k in a:
        assert a[k] == b[k], (k, a[k], b[k])


def test_noalloc_diag_equals_diag_on_two_lattices(oracle_mod):
    from paper_1503_08406_amd.dmrt import Solver
    big = Solver(W.cavity(nx=300, ny=200, Ra=2e5, Da=5e-3, Ste=0.5, T_init=0.2), graph_steps=8)
    big.step(600)
    L = oracle_mod.lattice()
    case = W.make_case("rand", 70, 37, [1, 1, 2, 2], [0.9, 0.1, 0, 0], Ra=2e5, Da=2e-3, Pr=1.0,
                       Ste=0.8, eps=0.45, H=64, T_init=0.4, T_s=0.38, T_l=0.42, convective=1)
    small = Solver(case)
    f, g, fl = W.random_state(70, 37, 9, L["w9"], L["w5"])
    small.set_state(f, g, fl)
    small.step(12)
    _say("no-alloc diag: 300x200 cavity")
    a1, b1 = big.diag_noalloc(), big.diag()
    assert a1["active"] > 100 and a1["u_max"] > 0
    _same(a1, b1)
    _say("no-alloc diag: 70x37 random state (smaller, second call)")
    a2, b2 = small.diag_noalloc(), small.diag()
    assert a2["active"] > 0
    _same(a2, b2)
    big.step(10)
    _same(big.diag_noalloc(), big.diag())
    big.close()
    small.close()


def test_noalloc_diag_rejects_a_lattice_beyond_its_scratch():
    from paper_1503_08406_amd.dmrt import DmrtError, DMRT_ESIZE, Solver
    _say("no-alloc diag: 4096x4224 lattice (beyond the fixed scratch)")
    s = Solver(W.cavity(nx=4096, ny=4224, steps=0))
    with pytest.raises(DmrtError) as ei:
        s.diag_noalloc()
    assert ei.value.code == DMRT_ESIZE and "scratch" in str(ei.value)
    d = s.diag()  # the allocating entry point still serves it
    assert d["nonfinite"] == 0
    s.close()
