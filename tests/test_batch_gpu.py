"""GPU tests of batched cavities (dmrt_batch_*): every cavity of a batch must
equal, bit for bit, a single lattice created with the same inputs (one step
per launch), whatever the launch shape (one or two steps per launch), graph
replay or tuning; small members are checked against
the FP64 oracle with the contract tolerances; the full 512-cavity workload
(10000 steps, in the launch configuration the benchmark times) is checked
on sampled cavities against single lattices and against stored oracle
values for its three smallest cavities."""
import os
import sys

import numpy as np
import pytest

from conftest import oracle_from_case
from parity_util import assert_fields_close
from paper_1503_08406_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small_batch():
    """Six cavities: ragged sizes (one and several 64-wide tiles, last column
    chunks wider and narrower than 32, a cavity narrower than 32, ragged y),
    C4-like parameters, one clear-fluid cavity (eps = 1) and one periodic in
    y; initial temperature just below melting so fronts and flow develop."""
    cavs, opts, _ = W.cavity_batch(n=6, seed=11, size_lo=20, size_hi=140)
    cavs[0].update(nx=64, ny=40)
    cavs[1].update(nx=130, ny=67)
    cavs[2].update(eps=1.0)
    cavs[3].update(nx=65, ny=9, H=64.0, Ra=2e4, bc_kind=[1, 1, 0, 0])
    cavs[4].update(nx=27, ny=50)  # narrower than half a tile
    opts["T_init"] = W.THETA_M_CAVITY - 0.05
    return cavs, opts


def _fields_equal(a, b, label):
    for k in ("T", "ux", "uy", "fl"):
        assert np.array_equal(a[k], b[k]), "%s %s differs (max %g)" % (
            label, k, np.abs(a[k] - b[k]).max())


@pytest.fixture(scope="module")
def small_reference():
    """Fields of each small-batch cavity from a single lattice, 300 steps of
    one step per launch."""
    from paper_1503_08406_amd.dmrt import Solver
    cavs, opts = _small_batch()
    out = []
    for i, c in enumerate(cavs):
        _say("single lattice", i, c["nx"], c["ny"])
        s = Solver(W.batch_member(c, opts), steps_per_launch=1)
        s.step(300)
        out.append(s.fields())
        s.close()
    return out


@pytest.mark.parametrize("rows,blocks,hint", [(4, 0, 0), (8, 0, 0), (4, 8, 0), (8, 1024, 0),
                                              (4, 0, 1), (4, 0, 2), (8, 0, 3), (0, 0, 0),
                                              (0, 0, 1), (0, 0, 2), (0, 0, 3)])
def test_batch_equals_single_lattices(small_reference, rows, blocks, hint):
    """Any launch shape (rows 0: two steps per launch, here also with an odd
    chunk that ends on a one-step launch) and any cache policy of the stores
    (store_hint)."""
    from paper_1503_08406_amd.dmrt import BatchSolver
    cavs, opts = _small_batch()
    _say("batch", rows, blocks, hint)
    b = BatchSolver(cavs, store_hint=hint, **opts)
    b.set_launch(rows, blocks)
    if rows == 0:
        assert b.launch()[0] == 0
        b.step(151)
        b.step(149)
    else:
        b.step(300)
    assert b.time == 300
    for i in range(len(cavs)):
        _fields_equal(b.fields(i), small_reference[i], "cavity %d" % i)
    liq, bad = b.check()
    assert (bad == 0).all()
    for i in range(len(cavs)):
        assert liq[i] == int((small_reference[i]["fl"] > 0).sum())
    b.close()


def test_batch_per_array_addressing(small_reference):
    """Two steps per launch with one buffer resource per array (addressing 1)
    instead of one per half of the state arena: the same bits."""
    from paper_1503_08406_amd.dmrt import BatchSolver
    cavs, opts = _small_batch()
    b = BatchSolver(cavs, addressing=1, **opts)
    b.set_launch(0, 0)
    b.step(151)
    b.step(149)
    for i in range(len(cavs)):
        _fields_equal(b.fields(i), small_reference[i], "cavity %d" % i)
    b.close()


def test_batch_graph_and_tune_keep_results(small_reference, tmp_path):
    """Graph replay (even chunks plus a plain remainder) and the tuner (which
    times candidates on a copy of the state) leave the results unchanged; the
    tuner's JSON cache returns the same choice."""
    from paper_1503_08406_amd.dmrt import BatchSolver
    cavs, opts = _small_batch()
    b = BatchSolver(cavs, graph_steps=16, **opts)
    b.step(50)
    cache = str(tmp_path / "tune.json")
    rows, blocks, ms = b.tune(trial_steps=3, cache=cache)
    _say("tuned", rows, blocks, ms)
    assert rows in (0, 4, 8) and blocks % 8 == 0 and ms > 0
    assert b.time == 50
    b.step(250)
    for i in range(len(cavs)):
        _fields_equal(b.fields(i), small_reference[i], "cavity %d" % i)
    b2 = BatchSolver(cavs, **opts)
    assert b2.tune(trial_steps=3, cache=cache)[:2] == (rows, blocks)
    assert b2.launch() == (rows, blocks)
    b.close()
    b2.close()


@pytest.mark.parametrize("graph_steps", [6, 16])
def test_batch_two_steps_per_launch_with_graphs(small_reference, graph_steps):
    """Graphs of an odd (3) and an even (8) number of two-step launches, then
    a plain odd remainder: the same bits as single lattices."""
    from paper_1503_08406_amd.dmrt import BatchSolver
    cavs, opts = _small_batch()
    b = BatchSolver(cavs, graph_steps=graph_steps, **opts)
    b.set_launch(0)
    b.step(297)
    b.step(3)
    assert b.time == 300
    for i in range(len(cavs)):
        _fields_equal(b.fields(i), small_reference[i], "cavity %d" % i)
    b.close()


def test_batch_one_step_per_launch_refuses_two_step_shape():
    from paper_1503_08406_amd.dmrt import BatchSolver, DmrtError
    cavs, opts = _small_batch()
    b = BatchSolver(cavs[:2], steps_per_launch=1, **opts)
    assert b.launch()[0] == 4
    with pytest.raises(DmrtError):
        b.set_launch(0)
    b.close()


def test_batch_matches_oracle():
    """Small members against the FP64 oracle after 400 steps."""
    from paper_1503_08406_amd.dmrt import BatchSolver
    cavs, opts = _small_batch()
    b = BatchSolver(cavs, **opts)
    b.step(400)
    for i in (0, 2, 3, 4, 5):
        _say("oracle", i)
        o = oracle_from_case(W.batch_member(cavs[i], opts))
        o.step(400)
        e = assert_fields_close(b.fields(i), o.fields(), label="cavity %d" % i)
        _say("cavity %d: relative u error %.3e (max |u| %.3e)" % (i, e["u"], e["umax"]))
    b.close()


def test_batch_rejects_bad_cavity():
    from paper_1503_08406_amd.dmrt import BatchSolver, DmrtError
    cavs, opts = _small_batch()
    cavs[4]["eps"] = 1.5
    with pytest.raises(DmrtError, match="cavity 4"):
        BatchSolver(cavs, **opts)
    cavs[4]["eps"] = 0.5
    b = BatchSolver(cavs, **opts)
    with pytest.raises(DmrtError):
        b.set_launch(6, 0)
    with pytest.raises(DmrtError):
        b.set_launch(4, 12)
    with pytest.raises(IndexError):
        b.fields(len(cavs))
    with pytest.raises(DmrtError):
        b.derived(-1)
    b.close()


def test_full_batch_workload():
    """The 512-cavity workload, 10000 steps, tuned launch with graph replay of
    64 steps (as benchmarked): every cavity finite; sampled cavities equal
    single lattices bit for bit; the three smallest match stored oracle
    values."""
    from paper_1503_08406_amd.dmrt import BatchSolver, Solver
    cavs, opts, steps = W.cavity_batch()
    _say("full batch: create")
    b = BatchSolver(cavs, graph_steps=64, **opts)
    _say("full batch: tune", b.tune(trial_steps=16))
    b.step(steps)
    b.sync()
    liq, bad = b.check()
    _say("full batch: liquid nodes", int(liq.sum()), "bad cavities", int((bad > 0).sum()))
    assert (bad == 0).all(), np.nonzero(bad)[0]
    assert (liq > 0).all()
    area = np.array([c["nx"] * c["ny"] for c in cavs])
    tau = np.array([b.derived(i)["tau_nu"] for i in range(len(cavs))])
    sample = sorted({int(np.argmin(area)), int(np.argmax(area)), int(np.argmin(tau)),
                     int(np.argmax(tau)), int(np.argmax([c["Ra"] for c in cavs])),
                     int(np.argmin([c["Ste"] for c in cavs])), 0, 255, 511})
    for i in sample:
        _say("full batch: single lattice", i)
        s = Solver(W.batch_member(cavs[i], opts), graph_steps=64, steps_per_launch=1)
        s.step(steps)
        _fields_equal(b.fields(i), s.fields(), "cavity %d" % i)
        s.close()
    gold = np.load(os.path.join(GOLDEN, "batch_512_smallest.npz"))
    assert int(gold["steps"]) == steps
    for k, i in enumerate(gold["index"]):
        fo = {n: gold["%s_%d" % (n, k)] for n in ("T", "ux", "uy", "fl")}
        e = assert_fields_close(b.fields(int(i)), fo, label="cavity %d" % i)
        _say("full batch: cavity %d against the oracle: relative u error %.3e (max |u| %.3e)"
             % (i, e["u"], e["umax"]))
    b.close()
