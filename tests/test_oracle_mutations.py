"""The oracle's pins are sharp enough to catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (a scratch
build in a temporary directory; the oracle itself is untouched), builds it
and runs a set of pins against that build in a child process.  The unchanged
copy must pass every pin; each mutated copy must fail the pins named for it.
The mistakes are the ones a reader of Sec. 4 (non-equilibrium extrapolation
at walls and at the moving solid-liquid interface, flow solved in the liquid
only) could plausibly make.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dmrt_oracle.c")

PINS = ["slab_flow", "pressure_level", "box_rest", "solid_channel"]

_RUNNER = r"""
import json, sys
sys.path[:0] = [%(root)r, %(tests)r]
import oracle
import test_oracle_pins as P
pins = {
    "slab_flow": lambda: P.check_slab_flow_follows_brinkman(),
    "pressure_level": lambda: P.check_flow_independent_of_pressure_level(oracle),
    "box_rest": lambda: P.test_closed_box_at_rest_keeps_any_density(oracle),
    "solid_channel": lambda: P.test_channel_bounded_by_solid_nodes(oracle),
}
out = {}
for name in %(pins)r:
    try:
        pins[name]()
        out[name] = "pass"
    except Exception as e:  # a mistake may also break a pin by NaN or a failed solve
        out[name] = "fail: %%s" %% (type(e).__name__,)
print(json.dumps(out))
"""

WALL_EQ = "orc_feq(s->rho[c], 0, 0, phi, feq_w);"
NODE_EQ = "orc_feq(s->rho[c], s->ux[c], s->uy[c], phi, feq_x);"
RESTART = "double rbar = cnt ? rsum / cnt : RHO0;"
LIQ_SRC = "s->chi[sc = (long)sy * nx + sx]"
NEE = """                } else {
                    s->fnew[c * Q9 + i] = feq_w[i] + s->fpost[c * Q9 + i] - feq_x[i];
                }"""
OPP = "static const int opp[Q9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};"

# name: (text, replacement, pins that must fail)
MUTATIONS = {
    "wall equilibrium at rho0 instead of the node's density":
        (WALL_EQ, "orc_feq(RHO0, 0, 0, phi, feq_w);", ["slab_flow", "pressure_level", "box_rest"]),
    "melted node restarts at rho0":
        (RESTART, "double rbar = RHO0; (void)rsum;", ["pressure_level"]),
    "pull from solid nodes without extrapolation":
        (LIQ_SRC, "((sc = (long)sy * nx + sx) >= 0)", ["pressure_level", "solid_channel"]),
    "half-way bounce-back at solid sources":
        (NEE, """                } else if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side)) {
                    %s
                    s->fnew[c * Q9 + i] = s->fpost[c * Q9 + opp[i]];
""" % OPP + NEE.lstrip(), ["solid_channel"]),
    "extrapolation from the solid node's populations":
        (NEE, """                } else if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side)) {
                    s->fnew[c * Q9 + i] = feq_w[i] + s->fpost[((long)sy * nx + sx) * Q9 + i] - feq_x[i];
""" + NEE.lstrip(), ["pressure_level", "solid_channel"]),
    "extrapolation without the node's velocity":
        (NODE_EQ, "orc_feq(s->rho[c], 0, 0, phi, feq_x);",
         ["slab_flow", "pressure_level", "solid_channel"]),
}


def _build_and_run(tmp_path, tag, text=None, repl=None):
    src = open(SRC).read()
    if text is not None:
        assert src.count(text) == 1, "mutation target not unique: %r" % text
        src = src.replace(text, repl)
    d = tmp_path / tag
    d.mkdir()
    (d / "o.c").write_text(src)
    hdr = os.path.join(ROOT, "oracle")
    lib = str(d / "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-I", hdr, "-o", lib, str(d / "o.c"),
                           "-lm"])
    env = dict(os.environ, DMRT_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    code = _RUNNER % dict(root=ROOT, tests=os.path.join(ROOT, "tests"), pins=PINS)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_unchanged_copy_passes_every_pin(tmp_path):
    res = _build_and_run(tmp_path, "control")
    assert all(v == "pass" for v in res.values()), res


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_its_pins(tmp_path, name):
    text, repl, must_fail = MUTATIONS[name]
    res = _build_and_run(tmp_path, "m", text, repl)
    print(name, res)
    for pin in must_fail:
        assert res[pin] != "pass", (name, pin, res)
