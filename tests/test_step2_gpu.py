"""Two time steps per launch (steps_per_launch = 2, the k_step2 kernel)
against one step per launch: the same per-node arithmetic, so the same bits,
for every boundary layout, for lattices narrower and wider than one tile of
62 columns, for row counts that leave a ragged last tile (and lattices of
fewer rows than a tile), with melting, freezing and convection, with odd
step counts (a last single step) and with graph replay (also graphs of an
odd number of two-step launches)."""
import sys

import numpy as np
import pytest

from paper_1503_08406_amd import workloads as W

pytestmark = pytest.mark.gpu

BCS = {
    "periodic": ([0, 0, 0, 0], [0, 0, 0, 0]),
    "walls_x": ([1, 2, 0, 0], [0.9, 0, 0, 0]),
    "box": ([1, 1, 2, 2], [0.9, 0.1, 0, 0]),
    "mixed": ([2, 1, 1, 2], [0, 0.05, 0.7, 0]),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b, label):
    for k in a:
        assert np.array_equal(a[k], b[k]), (label, k, float(np.abs(a[k] - b[k]).max()))


def _pair(case, **over):
    from paper_1503_08406_amd.dmrt import Solver
    return Solver(case, steps_per_launch=1, **over), Solver(case, steps_per_launch=2, **over)


def _compare(s1, s2, label):
    _same(s1.fields(), s2.fields(), label + " fields")
    f1, g1 = s1.populations()
    f2, g2 = s2.populations()
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2), label + " populations"
    assert s1.time == s2.time


@pytest.mark.parametrize("bc", list(BCS))
@pytest.mark.parametrize("shape", [(70, 37), (62, 16), (63, 17), (124, 9), (5, 7)])
def test_two_steps_per_launch_equal_single_steps_on_random_states(oracle_mod, bc, shape):
    nx, ny = shape
    kinds, tw = BCS[bc]
    L = oracle_mod.lattice()
    case = W.make_case("rand", nx, ny, kinds, tw, Ra=2e5, Da=2e-3, Pr=1.0, Ste=0.8, eps=0.45,
                       H=64, T_init=0.4, T_s=0.38, T_l=0.42, convective=1)
    f, g, fl = W.random_state(nx, ny, 9, L["w9"], L["w5"])
    s1, s2 = _pair(case)
    for s in (s1, s2):
        s.set_state(f, g, fl)
    for n in (2, 1, 4, 9):
        _say("two-step", bc, shape, n)
        s1.step(n)
        s2.step(n)
        _compare(s1, s2, "%s %s after %d" % (bc, shape, s1.time))


@pytest.mark.parametrize("graph_steps", [0, 6, 8])
def test_two_steps_per_launch_on_a_melting_cavity(graph_steps):
    """Convection melting with moving interface (150 x 77: two tiles and a
    ragged third across, a ragged last tile row), plain launches and graphs
    of 3 and 4 two-step launches; odd totals."""
    case = W.cavity(nx=150, ny=77, Ra=3e5, Da=5e-3, Ste=0.5, T_init=0.2)
    s1, s2 = _pair(case, graph_steps=graph_steps)
    for n in (300, 301, 99):
        s1.step(n)
        s2.step(n)
        _compare(s1, s2, "cavity gs %d after %d" % (graph_steps, s1.time))
    assert (s1.fields()["fl"] > 0).sum() > 100


def test_two_steps_per_launch_on_a_freezing_cavity_and_degenerate_lattices():
    cases = [
        W.make_case("freezing", 100, 72, [1, 1, 2, 2], [1.0, 0.0, 0.0, 0.0], Ra=1e5, Da=5e-3,
                    Pr=1.0, Ste=0.5, eps=0.45, H=72, T_init=0.8, T_s=0.48, T_l=0.52,
                    convective=1),
        W.make_case("one", 1, 1, [0] * 4, [0] * 4, Ra=1e4, Da=1e-2, Pr=1, Ste=1, eps=0.5, H=8,
                    T_init=0.5, T_s=0.1, T_l=0.2),
        W.make_case("line", 1, 9, [1, 1, 2, 2], [1.0, 0.0, 0, 0], Ra=1e4, Da=1e-2, Pr=1, Ste=1,
                    eps=0.5, H=8, T_init=0.5, T_s=0.1, T_l=0.2),
        W.make_case("solid", 67, 5, [1, 2, 0, 0], [-0.5, 0, 0, 0], Ra=1e4, Da=1e-2, Pr=1, Ste=1,
                    eps=0.5, H=8, T_init=-1.0, T_s=0.1, T_l=0.2),
        W.make_case("liquid", 65, 9, [1, 1, 2, 2], [1.0, 0.5, 0, 0], Ra=1e5, Da=1e-2, Pr=1,
                    Ste=1, eps=0.9, H=9, T_init=0.8, T_s=0.1, T_l=0.2),
        W.conduction_slab(nx=130, ny=4),
        W.corner(n=96),
    ]
    for case in cases:
        _say("two-step", case["name"])
        s1, s2 = _pair(case, graph_steps=8)
        for n in (101, 300):
            s1.step(n)
            s2.step(n)
            _compare(s1, s2, "%s after %d" % (case["name"], s1.time))


def test_two_steps_per_launch_full_size_cavity_window():
    """The benchmark's 1024 x 1024 cavity: 2000 steps with graph replay in
    both modes give the same bits."""
    case = W.cavity(nx=1024, ny=1024, steps=2000)
    s1, s2 = _pair(case, graph_steps=64)
    s1.step(2000)
    s2.step(2000)
    _same(s1.fields(), s2.fields(), "cavity 1024")


@pytest.mark.parametrize("bc", list(BCS))
def test_per_array_addressing_gives_the_same_bits(oracle_mod, bc):
    """The two-step kernel with one buffer resource per array (addressing 1,
    the form for arrays that do not fit one 4 GB window) against the default
    single resource over the state's window and against one step per
    launch, on random mixed states."""
    from paper_1503_08406_amd.dmrt import Solver
    nx, ny = 70, 37
    kinds, tw = BCS[bc]
    L = oracle_mod.lattice()
    case = W.make_case("rand", nx, ny, kinds, tw, Ra=2e5, Da=2e-3, Pr=1.0, Ste=0.8, eps=0.45,
                       H=64, T_init=0.4, T_s=0.38, T_l=0.42, convective=1)
    f, g, fl = W.random_state(nx, ny, 11, L["w9"], L["w5"])
    s1, s2 = _pair(case)
    s3 = Solver(case, steps_per_launch=2, addressing=1)
    assert s3.launch_steps == 2
    for s in (s1, s2, s3):
        s.set_state(f, g, fl)
    for n in (2, 1, 4, 9):
        _say("addressing", bc, n)
        for s in (s1, s2, s3):
            s.step(n)
        _compare(s1, s2, "%s window after %d" % (bc, s1.time))
        _compare(s1, s3, "%s per array after %d" % (bc, s1.time))


def test_two_steps_per_launch_on_a_wide_lattice_with_rows_interleaved_over_dies(oracle_mod):
    """A lattice of 48 or more tiles per row (3000 nodes wide) takes the
    launch that interleaves tile rows over the dies: random states and a
    melting run give the bits of one step per launch, and a recorded run
    (two-step launches that also store the state between) ends at the same
    state."""
    from paper_1503_08406_amd.dmrt import Solver
    L = oracle_mod.lattice()
    kinds, tw = BCS["box"]
    case = W.make_case("wide", 3000, 37, kinds, tw, Ra=2e5, Da=2e-3, Pr=1.0, Ste=0.8, eps=0.45,
                       H=37, T_init=0.4, T_s=0.38, T_l=0.42, convective=1)
    f, g, fl = W.random_state(3000, 37, 13, L["w9"], L["w5"])
    s1, s2 = _pair(case)
    for s in (s1, s2):
        s.set_state(f, g, fl)
    for n in (2, 1, 4):
        s1.step(n)
        s2.step(n)
        _compare(s1, s2, "wide after %d" % s1.time)
    melt = W.cavity(nx=3000, ny=30, Ra=3e5, Da=5e-3, Ste=0.5, T_init=0.37)
    s1, s2 = _pair(melt, graph_steps=8)
    s3 = Solver(melt, record_mode=2)
    s1.step(201)
    s2.step(201)
    s3.record(201)
    _compare(s1, s2, "wide cavity")
    _same(s1.fields(), s3.fields(), "wide cavity recorded")
    assert (s1.fields()["fl"] > 0).sum() > 2 * 30  # past the wall column


@pytest.mark.parametrize("nx", [496, 3968])
def test_two_steps_per_launch_with_rotated_tile_groups(oracle_mod, nx):
    """Rows of tiles a multiple of 8 long (8 tiles: 496 nodes; 64 tiles:
    3968 nodes, also with the rows interleaved over the dies) take each
    die's tiles in rotated groups: random states and a melting run give the
    bits of one step per launch."""
    L = oracle_mod.lattice()
    kinds, tw = BCS["walls_x"]
    ny = 23
    case = W.make_case("rot", nx, ny, kinds, tw, Ra=2e5, Da=2e-3, Pr=1.0, Ste=0.8, eps=0.45,
                       H=ny, T_init=0.4, T_s=0.38, T_l=0.42, convective=1)
    f, g, fl = W.random_state(nx, ny, 17, L["w9"], L["w5"])
    s1, s2 = _pair(case)
    for s in (s1, s2):
        s.set_state(f, g, fl)
    for n in (2, 1, 4):
        _say("rotated groups", nx, n)
        s1.step(n)
        s2.step(n)
        _compare(s1, s2, "rotated %d after %d" % (nx, s1.time))
    melt = W.cavity(nx=nx, ny=30, Ra=3e5, Da=5e-3, Ste=0.5, T_init=0.37)
    s1, s2 = _pair(melt, graph_steps=8)
    s1.step(201)
    s2.step(201)
    _compare(s1, s2, "rotated cavity %d" % nx)


def test_launch_steps_reports_where_two_steps_apply():
    """Two steps per launch by default; one where the option, a literal
    variant of the thermal model, R2 or another launch shape rules it out
    (dmrt_launch_steps)."""
    from paper_1503_08406_amd.dmrt import Solver
    case = W.cavity(nx=70, ny=37)
    for over, want in (({}, 2), (dict(steps_per_launch=1), 1), (dict(sigma_mode=1), 1),
                       (dict(latent_mode=1), 1), (dict(block_rows=8), 1),
                       (dict(cells_per_lane=2), 1)):
        s = Solver(case, **over)
        assert s.launch_steps == want, over
        s.close()
