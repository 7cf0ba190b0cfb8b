"""The oracle's own discrete derivatives of its step (tangent-linear model and
its transpose, the adjoint) and of whole runs, pinned independently of any
GPU code:

- the tangent of one step against central differences of the oracle's step
  (Secs. 3.1-3.2, Eqs. 17-42, with walls and moving interface of Sec. 4);
- the adjoint against the tangent by the dot-product identity
  <J v, w> = <v, J^T w>;
- the gradient of a run against central differences of whole oracle runs.

The enthalpy fixed point is iterated to its exact FP64 value here (tolerance
0), so that differences of runs measure the derivative and not the stopping
rule of the iteration.
"""
import numpy as np
import pytest

from conftest import oracle_from_case
from paper_1503_08406_amd import workloads as W

BCS = {
    "periodic": ([0, 0, 0, 0], [0, 0, 0, 0]),
    "box": ([1, 1, 2, 2], [0.9, 0.1, 0, 0]),
    "mixed": ([2, 1, 1, 2], [0, 0.05, 0.7, 0]),
}
EXACT = dict(fl_tol=0.0, fl_maxit=400)


def _case(nx, ny, bc, seed, Ergun=True):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.35, 0.65, (ny, nx))
    K = 2e-3 * 64 * 64 * np.exp(0.5 * rng.standard_normal((ny, nx)))
    Feps = None if Ergun else rng.uniform(0.3, 0.6, (ny, nx))
    kinds, tw = BCS[bc]
    return W.make_case("adj_rand", nx, ny, kinds, tw, Ra=2e5, Da=2e-3, Pr=1.0, Ste=0.8, eps=eps,
                       K=K, Feps=Feps, H=64, T_init=0.4, T_s=0.38, T_l=0.42, convective=1)


def _sim(case, eps=None, K=None):
    c = dict(case)
    if eps is not None:
        c["eps"] = eps
    if K is not None:
        c["K"] = K
    return oracle_from_case(c, nthreads=1, **EXACT)


def _state(case, seed):
    from oracle import lattice
    L = lattice()
    f, g, fl = W.random_state(case["nx"], case["ny"], seed, L["w9"], L["w5"])
    f = f.astype(np.float64)
    f[:, fl == 0] = 0.0  # solid cells carry no flow populations
    return f, g.astype(np.float64), fl.astype(np.float64)


def _direction(case, fl, seed):
    rng = np.random.default_rng(seed)
    ny, nx = fl.shape
    df = 1e-2 * rng.standard_normal((9, ny, nx)) * (fl > 0)
    dg = 1e-1 * rng.standard_normal((5, ny, nx))
    dfl = 0.1 * rng.standard_normal((ny, nx)) * (fl > 0)
    dlnK = rng.standard_normal((ny, nx))
    deps = 0.1 * rng.standard_normal((ny, nx))
    return df, dg, dfl, dlnK, deps


def _one_step(case, state, eps, K):
    o = _sim(case, eps, K)
    o.set_state(*state)
    o.step(1)
    return o.get_state()


@pytest.mark.parametrize("bc", list(BCS))
@pytest.mark.parametrize("ergun", [True, False])
def test_tangent_of_one_step_matches_central_differences(bc, ergun):
    case = _case(11, 7, bc, 3, Ergun=ergun)
    f, g, fl = _state(case, 5)
    o = _sim(case)
    o.set_state(f, g, fl)
    v = _direction(case, fl, 7)
    tl = o.step_tl(*v)
    eps0, K0 = case["eps"].astype(np.float64), case["K"].astype(np.float64)
    h = 1e-6
    plus = _one_step(case, (f + h * v[0], g + h * v[1], fl + h * v[2]), eps0 + h * v[4],
                     K0 * np.exp(h * v[3]))
    minus = _one_step(case, (f - h * v[0], g - h * v[1], fl - h * v[2]), eps0 - h * v[4],
                      K0 * np.exp(-h * v[3]))
    for name, a, p, m in zip(("f", "g", "fl"), tl, plus, minus):
        fd = (p - m) / (2 * h)
        err = np.abs(a - fd).max() / max(np.abs(fd).max(), 1e-300)
        assert np.abs(fd).max() > 0 and err < 1e-6, (name, err)
    # the state of the oracle is untouched
    f2, g2, fl2 = o.get_state()
    assert np.array_equal(f2, f) and np.array_equal(g2, g) and np.array_equal(fl2, fl)


@pytest.mark.parametrize("bc", list(BCS))
@pytest.mark.parametrize("ergun", [True, False])
def test_adjoint_of_one_step_is_the_transpose_of_the_tangent(bc, ergun):
    case = _case(11, 7, bc, 4, Ergun=ergun)
    f, g, fl = _state(case, 6)
    o = _sim(case)
    o.set_state(f, g, fl)
    v = _direction(case, fl, 8)
    rng = np.random.default_rng(9)
    w = (rng.standard_normal(f.shape), rng.standard_normal(g.shape),
         rng.standard_normal(fl.shape))
    Jv = o.step_tl(*v)
    JTw = o.step_ad(*w)
    lhs = sum(float(np.sum(a * b)) for a, b in zip(Jv, w))
    rhs = sum(float(np.sum(a * b)) for a, b in zip(v, JTw))
    scale = sum(float(np.sum(np.abs(a * b))) for a, b in zip(Jv, w))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


def _phase_change_state():
    """A random state with some solid nodes made hot enough to melt in the
    next step (they restart from their neighbours' density) and some liquid
    nodes cold enough to freeze."""
    case = _case(12, 9, "box", 11)
    f, g, fl = _state(case, 12)
    from oracle import lattice
    w5 = lattice()["w5"]
    for (y, x) in np.argwhere(fl == 0)[::3]:
        g[:, y, x] = w5 * 0.6   # well above the liquidus: melts in this step
    for (y, x) in np.argwhere(fl > 0)[::5]:
        g[:, y, x] = w5 * -0.6  # well below the solidus: freezes in this step
    return case, f, g, fl


def test_tangent_covers_melting_restart_and_freezing():
    """A step in which some nodes melt (restart from their neighbours'
    density) and others freeze: tangent against central differences."""
    case, f, g, fl = _phase_change_state()
    o = _sim(case)
    o.set_state(f, g, fl)
    o.step(1)
    fn = o.get_state()[2]
    o.set_state(f, g, fl)
    assert ((fn > 0) & (fl == 0)).any() and ((fn == 0) & (fl > 0)).any()
    v = _direction(case, fl, 13)
    tl = o.step_tl(*v)
    eps0, K0 = case["eps"].astype(np.float64), case["K"].astype(np.float64)
    h = 1e-6
    p = _one_step(case, (f + h * v[0], g + h * v[1], fl + h * v[2]), eps0 + h * v[4],
                  K0 * np.exp(h * v[3]))
    m = _one_step(case, (f - h * v[0], g - h * v[1], fl - h * v[2]), eps0 - h * v[4],
                  K0 * np.exp(-h * v[3]))
    for a, pp, mm in zip(tl, p, m):
        fd = (pp - mm) / (2 * h)
        assert np.abs(a - fd).max() < 1e-6 * np.abs(fd).max()


def test_adjoint_is_the_transpose_across_melting_and_freezing():
    """The dot-product identity on the step with restarts and freezing."""
    case, f, g, fl = _phase_change_state()
    o = _sim(case)
    o.set_state(f, g, fl)
    v = _direction(case, fl, 14)
    rng = np.random.default_rng(15)
    w = (rng.standard_normal(f.shape), rng.standard_normal(g.shape),
         rng.standard_normal(fl.shape))
    Jv = o.step_tl(*v)
    JTw = o.step_ad(*w)
    lhs = sum(float(np.sum(a * b)) for a, b in zip(Jv, w))
    rhs = sum(float(np.sum(a * b)) for a, b in zip(v, JTw))
    scale = sum(float(np.sum(np.abs(a * b))) for a, b in zip(Jv, w))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


def _run_fields(case, steps, eps, K):
    o = _sim(case, eps, K)
    o.step(steps)
    F = o.fields()
    return F["T"], F["fl"]


def _central(case, steps, wT, wf, plus, minus, h):
    """Central difference of sum(wT T + wf f_l), summed over the field
    differences (the loss itself is O(10); its rounding would swamp the
    small derivatives)."""
    Tp, fp = _run_fields(case, steps, *plus)
    Tm, fm = _run_fields(case, steps, *minus)
    return float(np.sum(wT * (Tp - Tm)) + np.sum(wf * (fp - fm))) / (2 * h)


@pytest.mark.parametrize("kind", ["convection", "conduction"])
def test_gradient_of_a_run_matches_central_differences(kind):
    """Gradients of sum(wT T + wf f_l) after a melting run (nodes melting while
    the liquid convects, or pure conduction) with respect to ln K and eps of
    single cells, against central differences of whole oracle runs."""
    nx, ny = 10, 8
    rng = np.random.default_rng(21)
    eps = rng.uniform(0.35, 0.6, (ny, nx))
    H = 32.0
    K = 5e-3 * H * H * np.exp(0.5 * rng.standard_normal((ny, nx)))
    if kind == "convection":
        case = W.make_case("adj_run", nx, ny, [1, 1, 2, 2], [1.0, 0, 0, 0], Ra=2e4, Da=5e-3,
                           Pr=1.0, Ste=1.0, eps=eps, K=K, H=H, T_init=0.375, T_s=0.38,
                           T_l=0.42, convective=1)
        steps = 60
    else:
        case = W.make_case("adj_run", nx, ny, [1, 2, 2, 2], [1.0, 0, 0, 0], Ra=0.0, Da=1e-2,
                           Pr=1.0, Ste=1.0, eps=eps, K=K, T_init=-0.06, T_s=-0.02, T_l=0.02,
                           alpha_l=0.05, convective=0)
        steps = 50
    wT = rng.standard_normal((ny, nx))
    wf = rng.standard_normal((ny, nx))
    o = _sim(case)
    gk, ge = o.adjoint_run(steps, wT, wf)
    assert o.time == 0
    o.step(steps)
    assert (o.fields()["fl"] > 0).sum() >= 8
    eps0, K0 = case["eps"].astype(np.float64), case["K"].astype(np.float64)
    cells = [tuple(int(v) for v in np.unravel_index(np.abs(ge).argmax(), ge.shape)),
             (ny // 2, 1), (1, 2), (ny - 2, 3)]
    if kind == "convection":
        cells.append(tuple(int(v) for v in np.unravel_index(np.abs(gk).argmax(), gk.shape)))
    # rounding of the field differences is ~1e-15: bound the error by the
    # contract relative to the largest gradient plus that noise over 2h
    for c in cells:
        h = 1e-6
        ep, em = eps0.copy(), eps0.copy()
        ep[c] += h
        em[c] -= h
        fe = _central(case, steps, wT, wf, (ep, K0), (em, K0), h)
        assert abs(ge[c] - fe) <= 1e-6 * np.abs(ge).max() + 1e-15 / h, (c, ge[c], fe)
        h = 1e-4
        kp, km = K0.copy(), K0.copy()
        kp[c] *= np.exp(h)
        km[c] *= np.exp(-h)
        fk = _central(case, steps, wT, wf, (eps0, kp), (eps0, km), h)
        assert abs(gk[c] - fk) <= 1e-6 * np.abs(gk).max() + 1e-15 / h, (c, gk[c], fk)
    if kind == "conduction":
        # the liquid stays at rest: K acts only through rounding-level flow
        assert np.abs(gk).max() <= 1e-12 * np.abs(ge).max()
    else:
        assert np.abs(gk).max() > 0


def test_derivatives_refuse_a_non_uniform_heat_capacity():
    case = _case(6, 5, "box", 1)
    case["opts"]["sigma_l"] = 1.2
    o = _sim(case)
    with pytest.raises(ValueError):
        o.adjoint_run(3)
