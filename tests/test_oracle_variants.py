"""Pins of the oracle's literal variants of the thermal model (ablations of
the readings): the heat-capacity ratio of Eq. (7), the effective
conductivity of Eq. (8), and the latent source of Eq. (30) placed at the
pre-stream site with a global iteration (R2).

As in the other pin files, the references are independent of the oracle's
code: the differential effective-medium equation that Eq. (8) integrates,
the decay rate of a Fourier mode of Eq. (3), the two-region Neumann
solution, an exact invariant, and the bookkeeping of a single melting node.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq
from scipy.special import erf, erfc

from conftest import front_rows, oracle_from_case
from paper_1503_08406_amd import workloads as W


def _dem(phi, kp, km):
    """Bruggeman's differential effective medium for spherical inclusions of
    conductivity km in a host of conductivity kp: adding inclusions up to the
    volume fraction 1 - phi, dk/dv = 3 k (km - k) / ((1 - v)(km + 2k))."""
    rhs = lambda v, k: 3 * k * (km - k) / ((1 - v) * (km + 2 * k))
    r = solve_ivp(rhs, (0.0, 1.0 - phi), [kp], rtol=1e-12, atol=1e-14)
    return float(r.y[0, -1])


@pytest.mark.parametrize("phi,fl,ks,km", [
    (0.5, 1.0, 2.0, 3.0), (0.4, 0.0, 2.0, 3.0), (0.3, 0.5, 0.5, 10.0),
    (0.1, 1.0, 1.0, 100.0),
    # matrix far less conductive than the PCM: three real roots of the cubic
    (0.9, 1.0, 1.0, 0.01), (0.9, 0.2, 3.0, 0.02), (0.99, 1.0, 1.0, 1e-3),
])
def test_ke_of_eq8_is_the_effective_medium_integral(oracle_mod, phi, fl, ks, km):
    """Eq. (8), for a random distribution of spherical inclusions, is the
    integral of the differential effective-medium equation; the oracle's
    root is that integral (also where the cubic has three real roots)."""
    kp = fl + (1 - fl) * ks
    assert abs(oracle_mod.ke(phi, fl, ks, km) / _dem(phi, kp, km) - 1) < 1e-10


def test_ke_limits(oracle_mod):
    """No matrix (phi = 1) gives the PCM's k_p; equal conductivities give
    that value; the dilute limit has Maxwell's slope 3 k_p (k_m - k_p) /
    (k_m + 2 k_p) in the matrix fraction."""
    for fl, ks, km in [(1.0, 1.0, 3.0), (0.0, 2.0, 0.1), (0.3, 0.5, 7.0)]:
        kp = fl + (1 - fl) * ks
        assert abs(oracle_mod.ke(1.0, fl, ks, km) - kp) < 1e-12 * kp
        assert abs(oracle_mod.ke(0.37, fl, ks, kp) - kp) < 1e-12 * kp
        d = 1e-5
        slope = (oracle_mod.ke(1.0 - d, fl, ks, km) - kp) / d
        maxwell = 3 * kp * (km - kp) / (km + 2 * kp)
        assert abs(slope / maxwell - 1) < 1e-4


def _mode_decay_rate(oracle_mod, T_s, T_l, fl0, **opts):
    """Decay rate per step of a cos(q x) temperature mode in a periodic
    1-D slab with porosity 0.4, far from the melting range."""
    nx, amp, steps = 128, 0.1, 400
    c = W.make_case("mode", nx, 1, [0] * 4, [0] * 4, Ra=0, Da=1e-2, Pr=1, Ste=1, eps=0.4,
                    T_init=0.0, T_s=T_s, T_l=T_l, alpha_l=0.03, convective=1, **opts)
    o = oracle_from_case(c)
    L = oracle_mod.lattice()
    q = 2 * math.pi / nx
    x = np.arange(nx)
    g = L["w5"][:, None, None] * (amp * np.cos(q * x))[None, None, :]
    o.set_state(np.zeros((9, 1, nx)), g, np.full((1, nx), fl0))
    o.step(50)
    a0 = (o.fields()["T"][0] * np.cos(q * x)).sum()
    o.step(steps)
    a1 = (o.fields()["T"][0] * np.cos(q * x)).sum()
    return -math.log(a1 / a0) / steps, q


@pytest.mark.parametrize("phase", ["solid", "liquid"])
def test_eq7_and_eq8_set_the_diffusion_of_each_phase(oracle_mod, phase):
    """Eq. (3) with sigma of Eq. (7) and alpha_e = alpha_l k_e / k_l of
    Eq. (8): a mode decays at alpha_e q^2 / sigma, with sigma = phi (f_l +
    (1 - f_l) c_ps/c_pl) + (1 - phi) (rho c_p)_m / (rho c_pl) and k_e the
    effective-medium value of the phase."""
    phi, cps, cm, ks, km = 0.4, 0.5, 2.0, 2.0, 3.0
    if phase == "solid":
        T_s, T_l, fl = 5.0, 6.0, 0.0
    else:
        T_s, T_l, fl = -6.0, -5.0, 1.0
    rate, q = _mode_decay_rate(oracle_mod, T_s, T_l, fl, sigma_mode=1, cps_ratio=cps,
                               cm_ratio=cm, ke_mode=1, ks_ratio=ks, km_ratio=km)
    sigma = phi * (fl + (1 - fl) * cps) + (1 - phi) * cm
    kp = fl + (1 - fl) * ks
    alpha_e = 0.03 * _dem(phi, kp, km)
    assert abs(rate / (alpha_e * q * q / sigma) - 1) < 5e-3


def _periodic_variant(nx, ny, seed, **kw):
    """Periodic box with random porosity and a random state crossing the
    melting range."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.3, 0.7, (ny, nx))
    c = W.make_case("variant_box", nx, ny, [0] * 4, [0] * 4, Ra=1e4, Da=1e-2, Pr=1.0,
                    Ste=0.7, eps=eps, T_s=0.38, T_l=0.42, **kw)
    return c


@pytest.mark.parametrize("latent_mode", [0, 1])
def test_enthalpy_invariant_with_cellwise_sigma(oracle_mod, latent_mode):
    """Eqs. (33), (38): collision and periodic streaming conserve sum T, and
    the latent source changes T of the cells it reaches by -phi/(sigma St)
    df_l in total, so sum(T + phi f_l / (sigma St)) is conserved when sigma
    of Eq. (7) varies from cell to cell (through phi) but not with f_l
    (c_ps = c_pl); with the source at the receiving node (R1) and at the
    pre-stream site (R2)."""
    nx, ny = 24, 20
    c = _periodic_variant(nx, ny, 7, sigma_mode=1, cps_ratio=1.0, cm_ratio=1.6,
                          latent_mode=latent_mode, fl_tol=1e-14)
    o = oracle_from_case(c)
    L = oracle_mod.lattice()
    f, g, fl = W.random_state(nx, ny, 8, L["w9"], L["w5"])
    o.set_state(f, g, fl)
    eps, St = c["eps"].astype(float), c["Ste"]
    sig = eps + (1 - eps) * 1.6
    F = o.fields()
    h0 = (F["T"] + eps * F["fl"] / (sig * St)).sum()
    fl0 = F["fl"].copy()
    o.step(200)
    F = o.fields()
    h1 = (F["T"] + eps * F["fl"] / (sig * St)).sum()
    assert abs(h1 - h0) < 1e-11 * abs(h0)
    assert np.abs(F["fl"] - fl0).max() > 0.1


def test_neumann_two_region_with_eq7_and_eq8():
    """Sec. 4.1 conduction melting with unequal phases: sigma from Eq. (7)
    (c_ps/c_pl = 0.6, matrix capacity 1.5) and k_e from Eq. (8) (k_s/k_l = 2,
    k_m/k_l = 3), porosity 0.5.

    The D2Q5 scheme (equilibrium of Eq. (34), tau_T from alpha_e / sigma,
    source of Eq. (38) divided by sigma) recovers T_t = (D T_x)_x -
    phi/(sigma St) (f_l)_t with D = alpha_e / sigma: Eq. (3) divided by
    sigma.  Each region diffuses with its D, and across the front the jump
    of D T_x balances phi/St x_m' times the mean of 1/sigma over the melting
    range, ln(sigma_l/sigma_s)/(sigma_l - sigma_s), where Eq. (3) itself
    would balance the jump of alpha_e T_x against phi/St x_m'.  The front
    and profiles follow the two-region Neumann solution of the former; the
    latter's front lies 1.2 lattice units further here."""
    phi, St, t = 0.5, 1.0, 10000
    cps, cm, ks, km, a0 = 0.6, 1.5, 2.0, 3.0, 0.02
    o = oracle_from_case(W.conduction_slab(), sigma_mode=1, cps_ratio=cps, cm_ratio=cm,
                         ke_mode=1, ks_ratio=ks, km_ratio=km)
    o.step(t)
    F = o.fields()
    sl, ss = phi + (1 - phi) * cm, phi * cps + (1 - phi) * cm
    Dl, Ds = a0 * _dem(phi, 1.0, km) / sl, a0 * _dem(phi, ks, km) / ss
    r = Dl / Ds
    lam = math.log(sl / ss) / (sl - ss)

    def g(e):
        return (Dl * math.exp(-e * e) / (erf(e) * math.sqrt(math.pi * Dl))
                - Ds * math.exp(-e * e * r) / (erfc(e * math.sqrt(r)) * math.sqrt(math.pi * Ds))
                - phi / St * lam * e * math.sqrt(Dl))

    eta = brentq(g, 1e-6, 5)
    xm = 2 * eta * math.sqrt(Dl * t)
    assert np.all(np.abs(front_rows(F["fl"]) - xm) < 0.5), (front_rows(F["fl"])[0], xm)
    x = np.arange(256) + 1.0
    Tan = np.where(x <= xm, 1 - erf(x / (2 * math.sqrt(Dl * t))) / erf(eta),
                   -1 + erfc(x / (2 * math.sqrt(Ds * t))) / erfc(eta * math.sqrt(r)))
    assert np.abs(F["T"][0] - Tan).max() < 0.02


def test_r2_conduction_melting_matches_neumann():
    """The literal placement of Eq. (30) (R2) solves the same problem: the
    Sec. 4.1 front and profiles of the one-region Neumann solution."""
    o = oracle_from_case(W.conduction_slab(), latent_mode=1)
    o.step(5000)
    F = o.fields()
    eta, a, t = 0.417942, 0.02, 5000
    xm = 2 * eta * math.sqrt(a * t)
    assert np.all(np.abs(front_rows(F["fl"]) - xm) < 0.5)
    x = np.arange(256) + 1.0
    s = 2 * math.sqrt(a * t)
    Tan = np.where(x <= xm, 1 - erf(x / s) / erf(eta), -1 + erfc(x / s) / erfc(eta))
    assert np.abs(F["T"][0] - Tan).max() < 0.01


def test_r2_source_reaches_the_neighbours(oracle_mod):
    """Eq. (30) with the source N^-1 S~ added before streaming: when a single
    node melts, its neighbours receive the component w~_i S0 of the
    direction pointing at them and the node keeps w~_0 S0, with
    N^-1 (1, 0, 0, varpi, 0) = (w~_0, w~_1, ..., w~_4); placed after
    streaming (R1) the node keeps all of S0."""
    n, phi, St = 9, 0.5, 1.0
    L = oracle_mod.lattice()
    T0 = np.full((n, n), -0.5)
    T0[4, 4] = 0.3
    g = L["w5"][:, None, None] * T0[None]
    out = {}
    for mode in (0, 1):
        c = W.make_case("one_node", n, n, [0] * 4, [0] * 4, Ra=0, Da=1e-2, Pr=1, Ste=St,
                        eps=phi, T_s=-0.02, T_l=0.02, alpha_l=0.05, convective=0,
                        latent_mode=mode, fl_tol=1e-14)
        o = oracle_from_case(c)
        o.set_state(np.zeros((9, n, n)), g, np.zeros((n, n)))
        o.step(1)
        out[mode] = o.fields()
    r1, r2 = out[0], out[1]
    f1, f2 = r1["fl"][4, 4], r2["fl"][4, 4]
    assert 0 < f2 < 1 and 0 < f1 < 1
    assert np.count_nonzero(r1["fl"]) == 1 and np.count_nonzero(r2["fl"]) == 1
    Ninv = np.linalg.inv(L["N"])
    wt = Ninv @ np.array([1.0, 0, 0, -2.0, 0])  # varpi = -2 (Sec. 4)
    S2 = -phi / St * f2
    Tstar = r1["T"][4, 4] + phi / St * f1  # before the R1 source
    assert abs(r2["T"][4, 4] - (Tstar + wt[0] * S2)) < 1e-14
    ex, ey = L["e5"][:, 0], L["e5"][:, 1]
    for i in range(1, 5):
        y, x = 4 + ey[i], 4 + ex[i]
        assert abs(r2["T"][y, x] - r1["T"][y, x] - wt[i] * S2) < 1e-14
    d = r2["T"] - r1["T"]
    d[4, 4] = 0
    for i in range(1, 5):
        d[4 + ey[i], 4 + ex[i]] = 0
    assert np.abs(d).max() < 1e-15


def test_variants_at_unit_ratios_reduce_to_the_default(oracle_mod):
    """Eq. (7) with c_ps = c_pl and (rho c_p)_m = rho c_pl gives sigma = 1,
    and Eq. (8) with k_s = k_m = k_l gives k_e = k_l: a convection-melting
    run agrees with the default model to rounding."""
    c = W.cavity(nx=24, ny=24, Ra=1e4, Da=1e-2, seed=3)
    a = oracle_from_case(c)
    b = oracle_from_case(c, sigma_mode=1, cps_ratio=1.0, cm_ratio=1.0, ke_mode=1,
                         ks_ratio=1.0, km_ratio=1.0)
    a.step(300)
    b.step(300)
    A, B = a.fields(), b.fields()
    assert A["fl"].max() > 0
    for k in ("T", "fl", "ux", "uy"):
        np.testing.assert_allclose(B[k], A[k], atol=1e-9, rtol=0)


def test_enthalpy_fixed_point_with_unequal_heat_capacities(oracle_mod):
    """Eqs. (38), (40)-(42) with c_ps != c_pl (the Eq. (7) variant): En =
    c_p T + f_l L_a with the mixture c_p = f_l c_pl + (1 - f_l) c_ps and
    En_s = c_ps T_s, En_l = c_pl T_l + L_a.  With sigma uniform, T = B - a f
    (B = T* + a f^k, a = phi/(sigma St)) and the mushy branch of Eq. (41)
    make f the root in (0, 1) of a quadratic; outside it f is 0 when B <= T_s
    and 1 when B - a >= T_l.  Unlike c_ps = c_pl, the plain iteration is not
    a contraction everywhere (En depends on the origin of T): the check
    covers the draws whose mushy root is attracting, slope of the map below
    0.9 in magnitude, and requires that most draws are."""
    rng = np.random.default_rng(77)
    checked = 0
    for _ in range(400):
        eps, St, sig = rng.uniform(0.1, 1.0), 10 ** rng.uniform(-1, 0.6), rng.uniform(0.8, 2.0)
        cps = rng.uniform(0.5, 1.5)
        Ts = rng.uniform(-0.5, 0.5)
        Tl = Ts + rng.uniform(0.01, 0.2)
        Tstar, flk = rng.uniform(Ts - 0.6, Tl + 0.6), rng.choice([0.0, 1.0, rng.uniform()])
        a = eps / (sig * St)
        B = Tstar + a * flk
        Es, El = cps * Ts, Tl + 1 / St
        if B <= Ts:
            fr = 0.0
        elif B - a >= Tl:
            fr = 1.0
        else:
            # f (En_l - En_s) = (cps + (1 - cps) f)(B - a f) + f / St - cps T_s
            A2 = (1 - cps) * a
            A1 = (El - Es) + cps * a - (1 - cps) * B - 1 / St
            A0 = cps * Ts - cps * B
            roots = np.roots([A2, A1, A0]) if abs(A2) > 1e-14 else np.array([-A0 / A1])
            roots = [r.real for r in np.atleast_1d(roots)
                     if abs(r.imag) < 1e-12 and -1e-12 <= r.real <= 1 + 1e-12]
            assert len(roots) == 1, roots
            fr = min(max(roots[0], 0.0), 1.0)
            slope = ((1 - cps) * (B - a * fr) - (cps + (1 - cps) * fr) * a + 1 / St) / (El - Es)
            if abs(slope) >= 0.9:
                continue
        fl, T, it = oracle_mod.enthalpy(Tstar, flk, eps, St, sig, sig, Ts, Tl, 1e-14, 2000,
                                        cps=cps)
        assert it < 2000
        assert abs(fl - fr) < 1e-10, (Tstar, flk, eps, St, cps, fl, fr)
        assert abs(T - (B - a * fl)) < 1e-12
        checked += 1
    assert checked > 300
