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
DERIV_PINS = ["tangent_fd", "tangent_fd_phase", "dot_product", "dot_product_phase",
              "run_gradient"]

_RUNNER = r"""
import json, sys
sys.path[:0] = [%(root)r, %(tests)r]
import oracle
import test_oracle_pins as P
import test_oracle_adjoint as D
pins = {
    "tangent_fd": lambda: D.test_tangent_of_one_step_matches_central_differences("mixed", True),
    "tangent_fd_phase": lambda: D.test_tangent_covers_melting_restart_and_freezing(),
    "dot_product": lambda: D.test_adjoint_of_one_step_is_the_transpose_of_the_tangent("mixed", True),
    "dot_product_phase": lambda: D.test_adjoint_is_the_transpose_across_melting_and_freezing(),
    "run_gradient": lambda: D.test_gradient_of_a_run_matches_central_differences("convection"),
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
LIQ_SRC = """s->chi[sc = (long)sy * nx + sx]) {
                    s->fnew[c * Q9 + i] = s->fpost[sc * Q9 + i];"""
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
        (LIQ_SRC, LIQ_SRC.replace("s->chi[sc = (long)sy * nx + sx]", "((sc = (long)sy * nx + sx) >= 0)"),
         ["pressure_level", "solid_channel"]),
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


# Mistakes in the oracle's discrete derivatives (tangent-linear model and
# its transpose): name: (text, replacement, pins that must fail).
DERIV_MUTATIONS = {
    "wrong sign of the (1 - eps)^2 factor in dK_e":
        ("- 2.0 * deps / (1.0 - w->eps) +", "+ 2.0 * deps / (1.0 - w->eps) +",
         ["tangent_fd", "dot_product"]),
    "moment adjoint relaxed with s instead of 1 - s":
        ("        bm[a] = (1.0 - sv[a]) * bmp[a];", "        bm[a] = sv[a] * bmp[a];",
         ["dot_product", "run_gradient"]),
    "adjoint of the g pull kept at the receiving node":
        ("                    bgp[((long)sy * nx + sx) * Q5 + i] += b;",
         "                    bgp[c * Q5 + i] += b;", ["dot_product", "run_gradient"]),
    "latent source tangent without the porosity of a":
        ("(dTs + a * dfl[c] + (fk - fn) * da) / (dTm + a)", "(dTs + a * dfl[c]) / (dTm + a)",
         ["tangent_fd", "dot_product"]),
    "restart adjoint not divided by the neighbour count":
        ("brho[nb[k]] += br / cnt;", "brho[nb[k]] += br;", ["dot_product_phase", "run_gradient"]),
    "enthalpy derivative also on the clamped branches":
        ("(fn > 0 && fn < 1) ? (dTs", "(fn >= 0 && fn <= 1) ? (dTs",
         ["tangent_fd", "tangent_fd_phase", "dot_product"]),
}


def _build_and_run(tmp_path, tag, text=None, repl=None, pins=None):
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
    code = _RUNNER % dict(root=ROOT, tests=os.path.join(ROOT, "tests"), pins=pins or PINS)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_unchanged_copy_passes_every_pin(tmp_path):
    res = _build_and_run(tmp_path, "control", pins=PINS + DERIV_PINS)
    assert all(v == "pass" for v in res.values()), res


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_its_pins(tmp_path, name):
    text, repl, must_fail = MUTATIONS[name]
    res = _build_and_run(tmp_path, "m", text, repl)
    print(name, res)
    for pin in must_fail:
        assert res[pin] != "pass", (name, pin, res)


@pytest.mark.parametrize("name", list(DERIV_MUTATIONS))
def test_planted_derivative_mistake_fails_its_pins(tmp_path, name):
    text, repl, must_fail = DERIV_MUTATIONS[name]
    res = _build_and_run(tmp_path, "d", text, repl, pins=DERIV_PINS)
    print(name, res)
    for pin in must_fail:
        assert res[pin] != "pass", (name, pin, res)
