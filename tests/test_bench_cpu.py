"""Host-side checks of the benchmark driver that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The step runs on one GPU; asking for more exits with a message."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""



def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_lead_steps_cover_both_graph_parities():
    """The untimed steps right before a timed window hold one graph's worth
    of steps, two when a graph holds an odd number of launches (so that the
    window replays graphs captured for both buffer parities)."""
    b = _bench()
    assert b.lead_steps(20, 2) == 20    # 10 two-step launches: parity kept
    assert b.lead_steps(10, 2) == 20    # 5 launches: parity flips per graph
    assert b.lead_steps(64, 2) == 64
    assert b.lead_steps(64, 1) == 64
    assert b.lead_steps(0, 2) == 8      # plain launches: a few to warm up


def test_byte_model_per_launch():
    """A launch, of one step or of two, moves the bytes of one step's state
    read and write (the intermediate state of two steps stays on chip)."""
    b = _bench()
    assert b.BYTES_FLUID == 132 and b.BYTES_SOLID == 52
    assert b.BYTES_FLUID_BATCH == 120 and b.BYTES_SOLID_BATCH == 48
    assert "k_step2" in b.step_kernel(2) and "k_step " in b.step_kernel(1) + " "
