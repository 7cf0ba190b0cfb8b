"""GPU parity of the moving-interface and pressure-level cases (the oracle
pins of tests/test_oracle_pins.py run through the HIP library), and of the
on-demand diagnostics reductions against sums formed from oracle fields."""
import math
import sys

import numpy as np
import pytest

from conftest import oracle_from_case
from parity_util import assert_diag_close, assert_fields_close, oracle_diag, pair
from paper_1503_08406_amd import workloads as W
import test_oracle_pins as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_slab_flow_along_moving_front_matches_oracle_and_brinkman():
    """The melting slab with buoyancy parallel to the front (Sec. 4.1 with
    convection, Eqs. 2, 4-6, 29): GPU fields against the oracle at the
    contract tolerances at five times over a few node-melting periods, and
    the GPU's u_y near the moving front against the quasi-steady Brinkman-
    Forchheimer balance at the oracle pin's bound."""
    case, p = P.slab_flow_case()
    s, o = pair(case, gpu_over=dict(fl_tol=1e-7))
    d = o.derived
    Feps = 1.75 / math.sqrt(175 * p["phi"] ** 3)
    x = np.arange(p["nx"])
    for t in p["times"]:
        _say("slab flow, step", t)
        s.step(t - s.time)
        o.step(t - o.time)
        Fg, Fo = s.fields(), o.fields()
        e = assert_fields_close(Fg, Fo, label="slab flow %d" % t)
        _say("  errors", {k: float("%.3g" % v) for k, v in e.items()})
        fl, uy = Fg["fl"][0].astype(np.float64), Fg["uy"][0].astype(np.float64)
        xs = int(np.argmax(fl == 0))
        assert xs == int(np.argmax(Fo["fl"][0] == 0))
        ua = P.brinkman_profile(x, Fg["T"][0].astype(np.float64), fl, d, p["phi"], Feps,
                                float(xs))(x[:xs])[0]
        err = np.abs(uy[:xs] - ua) / np.abs(ua).max()
        assert err[xs // 2:].max() < 5e-3 and err.max() < 4e-2, (err[xs // 2:].max(), err.max())
        assert np.abs(Fg["ux"]).max() < 1e-6


def test_pressure_level_does_not_change_the_flow_on_gpu(oracle_mod):
    """The melting, convecting cavity of the pressure-level pin started at
    liquid density 1 and 1.02: each run against the oracle at the contract
    tolerances, and the two GPU runs against each other (FP32 stores the
    deviations from the rest weights, so the shifted run rounds differently:
    1e-4 of max |u|)."""
    c, T, fl = P.gauge_case()
    L = oracle_mod.lattice()
    out = []
    for rho in (1.0, 1.02):
        _say("pressure level, density", rho)
        s, o = pair(c, gpu_over=dict(fl_tol=1e-7))
        f, g, f_l = P.gauge_state(L["w9"], L["w5"], T, fl, rho)
        s.set_state(f.astype(np.float32), g.astype(np.float32), f_l.astype(np.float32))
        o.set_state(f, g, f_l)
        s.step(1500)
        o.step(1500)
        Fg, Fo = s.fields(), o.fields()
        assert_fields_close(Fg, Fo, label="density %g" % rho)
        dg, do = s.diag(), oracle_diag(c, Fo)
        assert_diag_close(dg, do, label="density %g" % rho)
        out.append((Fg, dg))
        s.close()
    (A, da), (B, db) = out
    umax = max(np.abs(A["ux"]).max(), np.abs(A["uy"]).max())
    du = max(np.abs(A["ux"] - B["ux"]).max(), np.abs(A["uy"] - B["uy"]).max())
    _say("GPU pressure-level difference of u: %.3e of max |u|" % (du / umax))
    assert du <= 1e-4 * umax
    assert abs((db["mass"] - da["mass"]) / da["active"] - 0.02) < 1e-5


def test_closed_box_keeps_its_density_on_gpu(oracle_mod):
    """A liquid at rest at density 1.013 in a closed box stays at rest with
    its mass (the pin's case)."""
    n, rho = 6, 1.013
    c = W.make_case("box_rest", n, n + 1, [2, 2, 2, 2], [0] * 4, Ra=0, Da=1e-2, Pr=1, Ste=1,
                    eps=0.6, T_init=0.5, T_s=0.1, T_l=0.2, convective=1)
    from paper_1503_08406_amd.dmrt import Solver
    s = Solver(c)
    w9, w5 = oracle_mod.lattice()["w9"], oracle_mod.lattice()["w5"]
    f = np.broadcast_to(w9[:, None, None] * rho, (9, n + 1, n)).astype(np.float32)
    g = np.broadcast_to(w5[:, None, None] * 0.5, (5, n + 1, n)).astype(np.float32)
    s.set_state(f, g, np.ones((n + 1, n), np.float32))
    m0 = s.diag()["mass"]
    s.step(500)
    F, d = s.fields(), s.diag()
    assert np.abs(F["ux"]).max() == 0 and np.abs(F["uy"]).max() == 0
    assert abs(d["mass"] - m0) <= 1e-6 * m0 and abs(m0 / (n * (n + 1)) - rho) < 1e-6


def test_forced_closed_box_matches_oracle(oracle_mod):
    """A closed box of liquid at uniform temperature above the reference (a
    buoyancy force normal to the top and bottom walls), started from the
    hydrostatic density: the wall extrapolation as read lets a through-flow
    of about phi G develop (the force impulse of one step), on both sides
    alike; GPU against the oracle at the contract tolerances."""
    nx, ny, phi, T = 8, 16, 0.5, 0.9
    c = W.make_case("hydro", nx, ny, [2, 2, 2, 2], [0] * 4, Ra=1e4, Da=1e-2, Pr=1, Ste=1,
                    eps=phi, Feps=0.0, H=float(ny), T_init=T, T_s=0.1, T_l=0.2, T0=0.0,
                    convective=1, Ma=0.1)
    s, o = pair(c)
    G = o.derived["gbeta"] * T
    L = oracle_mod.lattice()
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    rho = 1 + 3 * phi * G * (y - (ny - 1) / 2)
    f = np.stack([L["w9"][i] * rho - 1.5 * L["w9"][i] * L["e9"][i, 1] * phi * G for i in range(9)])
    g = L["w5"][:, None, None] * T * np.ones((5, ny, nx))
    fl = np.ones((ny, nx))
    s.set_state(f.astype(np.float32), g.astype(np.float32), fl.astype(np.float32))
    o.set_state(f, g, fl)
    for t in (200, 4000):
        s.step(t - s.time)
        o.step(t - o.time)
        Fg, Fo = s.fields(), o.fields()
        assert_fields_close(Fg, Fo, label="forced box %d" % t)
        _say("forced closed box, step %d: mean u_y / (phi G) GPU %.4f oracle %.4f"
             % (t, Fg["uy"].mean() / (phi * G), Fo["uy"].mean() / (phi * G)))


# ------------------------------------------------------------ diagnostics
def test_diag_matches_oracle_on_random_states(oracle_mod):
    """dmrt_diag after 12 steps from random mixed states (each boundary
    layout) against the same reductions of the oracle's fields."""
    from test_parity_gpu import BCS, _random_case
    L = oracle_mod.lattice()
    for bc in BCS:
        nx, ny = 70, 37
        case = _random_case(nx, ny, bc)
        f, g, fl = W.random_state(nx, ny, 9, L["w9"], L["w5"])
        s, o = pair(case, gpu_over=dict(fl_tol=1e-7))
        s.set_state(f, g, fl)
        o.set_state(f.astype(float), g.astype(float), fl.astype(float))
        s.step(12)
        o.step(12)
        e = assert_diag_close(s.diag(), oracle_diag(case, o.fields()), label=bc)
        _say("diag random", bc, {k: float("%.2g" % v) for k, v in e.items()})
        s.close()


def test_diag_matches_oracle_on_freezing_cavity():
    """dmrt_diag on the convecting cavity that freezes at its cold wall
    (nodes leave the flow while it runs), at four times."""
    case = W.make_case("freezing", 100, 72, [1, 1, 2, 2], [1.0, 0.0, 0.0, 0.0], Ra=1e5, Da=5e-3,
                       Pr=1.0, Ste=0.5, eps=0.45, H=72, T_init=0.8, T_s=0.48, T_l=0.52,
                       convective=1)
    s, o = pair(case)
    for k in range(4):
        s.step(750)
        o.step(750)
        e = assert_diag_close(s.diag(), oracle_diag(case, o.fields()), label="freezing %d" % s.time)
        _say("diag freezing", s.time, {q: float("%.2g" % v) for q, v in e.items()})


def test_diag_matches_oracle_on_full_size_cavity():
    """dmrt_diag of the 1024x1024 cavity after 2000 steps (graph replay, as
    benchmarked) against the oracle's whole-lattice reductions
    (tests/golden/cavity_1024_2000_diag.npz)."""
    import os
    from paper_1503_08406_amd.dmrt import Solver
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "cavity_1024_2000_diag.npz"))
    s = Solver(W.cavity(nx=1024, ny=1024, steps=2000), graph_steps=64)
    s.step(int(gold["steps"]))
    do = {k: float(gold[k]) for k in gold.files}
    do["active"] = int(gold["active"])
    e = assert_diag_close(s.diag(), do, label="cavity 1024")
    _say("diag cavity 1024", {q: float("%.2g" % v) for q, v in e.items()})
