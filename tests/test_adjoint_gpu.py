"""GPU tests of the discrete adjoint (dmrt_record / dmrt_adjoint): gradients
of a functional of the final T and f_l fields with respect to per-cell
log K and porosity, against the FP64 oracle's own discrete adjoint and
central differences of the oracle on tiny grids (conduction melting;
convection melting with nodes melting during the run; a liquid cavity with
strong buoyancy freezing at the cold wall), and against a directional central
difference of the FP64 oracle on the full 512x512 inverse problem, with the
contract's relative error bound of 1e-3."""
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


@pytest.mark.parametrize("kind", ["conduction", "convection", "liquid"])
def test_adjoint_matches_oracle_adjoint(kind):
    """GPU gradients against the FP64 oracle's own discrete adjoint of the
    same run (oracle/dmrt_oracle.c, pinned on the CPU by central differences
    and the dot-product identity), element by element, at the contract's
    1e-3 relative to the largest component; and at the four cells of largest
    gradient against central differences of the oracle's run."""
    from paper_1503_08406_amd.dmrt import Solver
    case, steps, wT, wf = _case(kind)
    s = Solver(case, fl_tol=1e-7)
    s.record(steps)
    F = s.fields()
    assert (F["fl"] > 0).sum() >= 10 and ((F["fl"] > 0) & (F["fl"] < 1)).sum() > 0
    gk, ge = s.adjoint(wT, wf)
    _say(kind, "GPU gradients done; liquid", int((F["fl"] > 0).sum()))
    o = oracle_from_case(case, nthreads=1, fl_tol=1e-14)
    ok, oe = o.adjoint_run(steps, wT.astype(np.float64), wf.astype(np.float64))
    ek = np.abs(gk - ok).max() / max(np.abs(ok).max(), 1e-30)
    ee = np.abs(ge - oe).max() / max(np.abs(oe).max(), 1e-30)
    _say(kind, "max |dL/dlogK| %.3e err %.2e; max |dL/deps| %.3e err %.2e"
         % (np.abs(ok).max(), ek, np.abs(oe).max(), ee))
    assert ee <= FD_TOL
    if kind == "conduction":
        assert np.abs(gk).max() == 0.0  # no flow: permeability does not enter
    else:
        assert np.abs(ok).max() > 0 and ek <= FD_TOL
    eps0, K0 = case["eps"].astype(np.float64), case["K"].astype(np.float64)
    for idx in np.argsort(-np.abs(oe).ravel())[:4]:
        c = np.unravel_index(idx, oe.shape)
        h = 1e-6
        ep, em = eps0.copy(), eps0.copy()
        ep[c] += h
        em[c] -= h
        fd = (_oracle_functional(case, steps, wT, wf, ep, K0) -
              _oracle_functional(case, steps, wT, wf, em, K0)) / (2 * h)
        assert abs(ge[c] - fd) <= FD_TOL * np.abs(oe).max(), (c, ge[c], fd)
    # the state of the handle is unchanged by the adjoint
    F2 = s.fields()
    for k in F:
        assert np.array_equal(F[k], F2[k])


def test_record_modes_give_the_same_gradients_and_state():
    """Keeping every state of the run (no recomputation) and keeping sqrt(n)
    checkpoints (segments recomputed), each recorded (and recomputed) with one
    or two steps per launch (these with either addressing of the two-step
    kernel), give the same gradients bit for bit; the recorded run ends at
    the state dmrt_step reaches, and a second recording (graph replay)
    repeats the first."""
    from paper_1503_08406_amd.dmrt import Solver
    case, steps, wT, wf = _case("liquid")
    steps += 3  # not a square, odd
    ref = Solver(case, fl_tol=1e-7, steps_per_launch=1)
    ref.step(steps)
    Fr = ref.fields()
    out = []
    for mode, spl, addr in ((2, 2, 0), (1, 2, 0), (2, 1, 0), (1, 1, 0), (2, 2, 1), (1, 2, 1)):
        s = Solver(case, fl_tol=1e-7, record_mode=mode, steps_per_launch=spl, addressing=addr)
        assert s.launch_steps == spl
        for rep in range(2):
            s.reset()
            s.record(steps)
            F = s.fields()
            for k in F:
                assert np.array_equal(F[k], Fr[k]), (mode, spl, addr, rep, k)
            assert s.time == steps * (rep + 1)
            g = s.adjoint(wT, wf)
            if rep:
                assert all(np.array_equal(a, b) for a, b in zip(g, out[-1]))
            out.append(g)
        s.close()
    _say("record modes: max |dL/deps| %.3e" % float(np.abs(out[0][1]).max()))
    for other in out[2::2]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


def _loss(T, fl, Ts, fs):
    return 0.5 * (((T - Ts) ** 2).sum() + ((fl - fs) ** 2).sum())


def test_torch_function_and_directional_derivative():
    """The torch.autograd.Function gives the library's adjoint gradients, and
    a central difference of the GPU forward along a random direction matches
    the directional derivative."""
    import torch
    from paper_1503_08406_amd.dmrt import Solver, melting_run
    case, steps, _, _ = _case("liquid")
    s = Solver(case, fl_tol=1e-7)
    rng = np.random.default_rng(5)
    lk0 = torch.tensor(np.log(case["K"].astype(np.float64)), dtype=torch.float32, device="cuda")
    ep0 = torch.tensor(case["eps"], dtype=torch.float32, device="cuda")
    # target: the run with a perturbed permeability field
    with torch.no_grad():
        Ts, fs = melting_run(s, lk0 + 0.3 * torch.tensor(rng.standard_normal(lk0.shape),
                                                         dtype=torch.float32, device="cuda"), ep0, steps)
        Ts, fs = Ts.clone(), fs.clone()
    lk = lk0.clone().requires_grad_(True)
    ep = ep0.clone().requires_grad_(True)
    T, fl = melting_run(s, lk, ep, steps)
    L = _loss(T.double(), fl.double(), Ts.double(), fs.double())
    L.backward()
    gk, ge = s.adjoint((T - Ts).detach(), (fl - fs).detach())
    assert torch.equal(lk.grad, gk) and torch.equal(ep.grad, ge)
    vk = torch.tensor(rng.standard_normal(lk0.shape), dtype=torch.float32, device="cuda")
    ve = 0.02 * torch.tensor(rng.standard_normal(lk0.shape), dtype=torch.float32, device="cuda")
    dd = float((lk.grad * vk).sum() + (ep.grad * ve).sum())
    h = 1e-2
    with torch.no_grad():
        Lp = _loss(*[a.double() for a in melting_run(s, lk0 + h * vk, ep0 + h * ve, steps)],
                   Ts.double(), fs.double())
        Lm = _loss(*[a.double() for a in melting_run(s, lk0 - h * vk, ep0 - h * ve, steps)],
                   Ts.double(), fs.double())
    fd = float(Lp - Lm) / (2 * h)
    _say("directional derivative: adjoint %.6e, central difference %.6e" % (dd, fd))
    assert abs(dd - fd) <= 2e-2 * abs(fd)


def test_adjoint_full_size_inverse_problem():
    """The inverse-problem workload (512x512 cavity, Gaussian-random-field
    log K, seed 1; target run seed 2; 2000 steps) in the configuration the
    benchmark times: finite gradients, zero log K gradient away from the
    melted region (K enters only through the flow of liquid nodes), and the
    directional derivative along the gradient against a central difference
    of the FP64 oracle's runs, at the contract's 1e-3.

    The loss is the FP64 misfit L = 1/2 sum((f_l - f_l*)^2 + (T - T*)^2) of
    oracle runs, and its adjoint source (f_l - f_l*, T - T*) comes from those
    runs: the misfits are ~1e-5, so the FP32 forward's own rounding (~1e-7
    per field after 2000 steps) would change the source by percents.  The
    GPU's adjoint (its recorded FP32 run) is what is checked."""
    import os
    from paper_1503_08406_amd.dmrt import Solver
    case = W.adjoint_cavity()
    target = W.adjoint_cavity(seed=2)
    steps = case["steps"]
    nthr = min(16, len(os.sched_getaffinity(0)))
    tight = dict(fl_tol=1e-15, fl_maxit=400)
    _say("oracle: target run (seed 2) and the run of seed 1, 512^2 x %d steps, %d threads"
         % (steps, nthr))
    ot = oracle_from_case(target, nthreads=nthr, **tight)
    ot.step(steps)
    Ft = ot.fields()
    ot.close()
    o = oracle_from_case(case, nthreads=nthr, **tight)
    o.step(steps)
    Fo = o.fields()
    o.close()
    s = Solver(case, graph_steps=64)
    _say("GPU: record and adjoint")
    s.record(steps)
    Fg = s.fields()
    gk, ge = s.adjoint((Fo["T"] - Ft["T"]).astype(np.float32),
                       (Fo["fl"] - Ft["fl"]).astype(np.float32))
    assert np.isfinite(gk).all() and np.isfinite(ge).all()
    liquid = Fg["fl"] > 0
    near = liquid.copy()
    for _ in range(3):  # within 3 nodes of the final liquid region
        near = near | np.roll(near, 1, 0) | np.roll(near, -1, 0) | np.roll(near, 1, 1) | np.roll(near, -1, 1)
    L = 0.5 * (np.sum((Fo["T"] - Ft["T"]) ** 2) + np.sum((Fo["fl"] - Ft["fl"]) ** 2))
    gn = float(np.linalg.norm(gk.astype(np.float64)))
    _say("inverse problem: L %.6e, liquid %d, |g| %.6e" % (L, int(liquid.sum()), gn))
    assert liquid.sum() > 0 and np.all(gk[~near] == 0.0) and np.abs(gk[liquid]).max() > 0
    v = gk.astype(np.float64) / gn
    lk0 = np.log(case["K"].astype(np.float64))

    def fields_at(h):
        c = dict(case)
        c["K"] = np.exp(lk0 + h * v)
        oo = oracle_from_case(c, nthreads=nthr, **tight)
        oo.step(steps)
        F = oo.fields()
        oo.close()
        return F

    h = 1e-2  # changes no node's log K by more than h max|v|
    _say("oracle: runs at log K +- %g g/|g| (max |v| %.3f)" % (h, float(np.abs(v).max())))
    Fp, Fm = fields_at(h), fields_at(-h)
    dL = 0.0  # L(+h) - L(-h) summed from the field differences (no cancellation)
    for q, tq in (("T", Ft["T"]), ("fl", Ft["fl"])):
        dL += 0.5 * float(np.sum((Fp[q] - Fm[q]) * (Fp[q] + Fm[q] - 2 * tq)))
    fd = dL / (2 * h)
    err = abs(fd - gn) / gn
    _say("inverse problem: <g, v> = |g| %.6e, FP64 central difference %.6e, rel %.2e"
         % (gn, fd, err))
    assert err <= FD_TOL
    # the gradient the GPU gives for its own FP32 misfit, for the record
    gk32, _ = s.adjoint(Fg["T"] - Ft["T"].astype(np.float32), Fg["fl"] - Ft["fl"].astype(np.float32))
    _say("with the GPU's own FP32 misfit as the source: <g32, v> / |g| - 1 = %.2e"
         % (float(np.sum(gk32.astype(np.float64) * v)) / gn - 1))
    s.close()


def test_backward_refuses_a_replaced_recording():
    """Two differentiable runs on one solver before the first backward: the
    first backward raises (its recording was replaced), the second run's
    backward still gives the library's gradients."""
    import torch
    from paper_1503_08406_amd.dmrt import Solver, melting_run
    case, steps, wT, wf = _case("convection")
    s = Solver(case, fl_tol=1e-7)
    lk = torch.tensor(np.log(case["K"].astype(np.float64)), dtype=torch.float32,
                      device="cuda").requires_grad_(True)
    ep = torch.tensor(case["eps"], dtype=torch.float32, device="cuda").requires_grad_(True)
    wT_t = torch.tensor(wT, device="cuda")
    wf_t = torch.tensor(wf, device="cuda")
    T1, f1 = melting_run(s, lk, ep, steps)
    T2, f2 = melting_run(s, lk * 1.01, ep, steps)
    with pytest.raises(RuntimeError, match="recorded another run"):
        ((T1 * wT_t).sum() + (f1 * wf_t).sum()).backward()
    lk.grad = None
    ep.grad = None
    ((T2 * wT_t).sum() + (f2 * wf_t).sum()).backward()
    gk, ge = s.adjoint(wT, wf)
    assert np.array_equal(ep.grad.cpu().numpy(), ge)
    s.close()
