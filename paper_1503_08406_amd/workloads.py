"""Seeded synthetic workloads for the double-MRT phase-change solver.

This module only builds inputs (grid, boundary spec, dimensionless groups,
per-cell porosity and permeability fields).  It holds none of the method's
arithmetic and is shared by the HIP path, the oracle-based tests and the
benchmark.  Every floating-point field is rounded to float32 here, so both
sides of a parity test receive identical numbers.

Side order for boundaries: x-, x+, y-, y+.  Kinds: 0 periodic, 1 wall at a
fixed temperature, 2 adiabatic wall.  All walls are no-slip.

Workloads (the paper's three validation problems restated at new sizes):
  conduction_slab   Sec. 4.1 -- 256x4, periodic y, hot left wall
  corner            Sec. 4.2 -- 256x256, cold left and bottom walls
  cavity            Sec. 4.3 -- 1024x1024 convection melting, seeded
                    log-normal permeability perturbation (sigma 0.1)
  cavity_batch      many Sec. 4.3 cavities of seeded uneven sizes and
                    parameters, uniform porous fields per cavity
  adjoint_cavity    512x512 Sec. 4.3 cavity whose log-permeability is a
                    seeded Gaussian random field (inverse-problem setting)
"""
import math

import numpy as np

PERIODIC, WALL_T, WALL_ADIABATIC = 0, 1, 2


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def make_case(name, nx, ny, bc_kind, T_wall, Ra, Da, Pr, Ste, eps, K=None, Feps=None,
              steps=0, H=0.0, **opts):
    """A workload: a plain dict consumed by both the library binding and the
    oracle helpers.  eps / K / Feps are float32 [ny, nx] arrays (K / Feps may be
    None: the solver then uses Da*H^2 and the Ergun relation)."""
    shape = (ny, nx)
    eps = _f32(np.broadcast_to(eps, shape))
    K = None if K is None else _f32(np.broadcast_to(K, shape))
    Feps = None if Feps is None else _f32(np.broadcast_to(Feps, shape))
    return dict(name=name, nx=int(nx), ny=int(ny), H=float(H), bc_kind=list(bc_kind),
                T_wall=[float(t) for t in T_wall], Ra=float(Ra), Da=float(Da),
                Pr=float(Pr), Ste=float(Ste), eps=eps, K=K, Feps=Feps, steps=int(steps),
                opts=dict(opts))


def conduction_slab(nx=256, ny=4, steps=5000, porosity=0.5, Ste=1.0, alpha=0.02):
    """Conduction melting of a semi-infinite porous slab (Sec. 4.1): left wall
    at theta = 1, initial theta = -1 (solid), melting at theta_m = 0 with the
    mushy range +-0.02, periodic in y, no gravity (flow at rest)."""
    return make_case("conduction_slab", nx, ny, [WALL_T, WALL_ADIABATIC, PERIODIC, PERIODIC],
                     [1.0, 0.0, 0.0, 0.0], Ra=0.0, Da=1e-4, Pr=1.0, Ste=Ste,
                     eps=porosity, steps=steps, T_init=-1.0, T_s=-0.02, T_l=0.02,
                     alpha_l=alpha, convective=0)


def corner(n=256, steps=20000, porosity=0.4, Ste=0.5, alpha=0.02):
    """Solidification in a semi-infinite corner (Sec. 4.2): left and bottom
    walls at theta = -1, the far sides adiabatic, initial liquid theta = 0.3,
    theta_m = 0, no convection."""
    return make_case("corner", n, n, [WALL_T, WALL_ADIABATIC, WALL_T, WALL_ADIABATIC],
                     [-1.0, 0.0, -1.0, 0.0], Ra=0.0, Da=1e-4, Pr=1.0, Ste=Ste,
                     eps=porosity, steps=steps, T_init=0.3, T_s=-0.02, T_l=0.02,
                     alpha_l=alpha, convective=0)


THETA_M_CAVITY = 9.78 / 25.0  # (T_m - T_c)/(T_h - T_c) of Sec. 4.3


def cavity(nx=1024, ny=1024, steps=100000, Ra=1e6, Da=1e-4, Pr=1.0, Ste=1.0,
           porosity=0.4, k_sigma=0.1, seed=3, T_init=0.0):
    """Convection melting in a porous square cavity (Sec. 4.3): hot left wall
    theta = 1, cold right wall theta = 0, adiabatic top and bottom, initially
    solid at theta = 0, theta_m = 9.78/25 with a +-0.02 mushy range.  The
    permeability is Da*H^2 times a seeded log-normal factor exp(k_sigma*xi),
    xi ~ N(0, 1) iid per cell (H = ny)."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((ny, nx))
    K = Da * float(ny) ** 2 * np.exp(k_sigma * xi)
    return make_case("cavity", nx, ny, [WALL_T, WALL_T, WALL_ADIABATIC, WALL_ADIABATIC],
                     [1.0, 0.0, 0.0, 0.0], Ra=Ra, Da=Da, Pr=Pr, Ste=Ste, eps=porosity,
                     K=K, steps=steps, T_init=T_init, T_s=THETA_M_CAVITY - 0.02,
                     T_l=THETA_M_CAVITY + 0.02, convective=1)


def gallium_cavity(n=200, steps=0):
    """The Sec. 4.3 problem as the paper sets it up (gallium melting in a
    cavity packed with glass beads): n x n lattice, H = n, Ra = 8.409e5,
    Da = 1.37e-5, porosity 0.385, J = 1, Pr = 0.0208, lambda = 0.2719,
    alpha_l/alpha_s = 1, St = 0.1241, sigma 0.8604 (liquid) and 0.8352
    (solid), Ma = 0.1; hot wall 45, cold wall and initial state 20, melting
    at 29.78, scaled to theta = (T - 20)/25 (T_0 = 20: theta_0 = 0), with a
    +-0.02 mushy range in theta; uniform K = Da H^2."""
    return make_case("gallium_cavity", n, n, [WALL_T, WALL_T, WALL_ADIABATIC, WALL_ADIABATIC],
                     [1.0, 0.0, 0.0, 0.0], Ra=8.409e5, Da=1.37e-5, Pr=0.0208, Ste=0.1241,
                     eps=0.385, steps=steps, H=float(n), T_init=0.0,
                     T_s=THETA_M_CAVITY - 0.02, T_l=THETA_M_CAVITY + 0.02, T0=0.0,
                     convective=1, Ma=0.1, J=1.0, sigma_s=0.8352, sigma_l=0.8604,
                     **{"lambda": 0.2719})


CAVITY_BATCH_OPTS = dict(T_init=0.0, T_s=THETA_M_CAVITY - 0.02, T_l=THETA_M_CAVITY + 0.02,
                         convective=1)


def cavity_batch(n=512, seed=4, size_lo=64, size_hi=512, steps=10000):
    """Independent Sec. 4.3 cavities (hot left wall, cold right wall,
    adiabatic top and bottom, initially solid at theta = 0) with seeded
    uneven sizes and parameters: nx, ny iid integers in [size_lo, size_hi],
    Ra = 10^U(4, 6), Da = 10^U(-5, -2), porosity U(0.3, 0.9) (rounded to
    float32), Ste U(0.1, 2), Pr = 1, H = ny; each cavity has uniform porous
    fields (K = Da H^2, F_eps from the Ergun relation).  Returns (cavities,
    shared options, steps)."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(size_lo, size_hi + 1, n)
    ny = rng.integers(size_lo, size_hi + 1, n)
    Ra = 10.0 ** rng.uniform(4.0, 6.0, n)
    Da = 10.0 ** rng.uniform(-5.0, -2.0, n)
    eps = rng.uniform(0.3, 0.9, n).astype(np.float32).astype(np.float64)
    Ste = rng.uniform(0.1, 2.0, n)
    cavs = [dict(nx=int(nx[i]), ny=int(ny[i]), H=0.0,
                 bc_kind=[WALL_T, WALL_T, WALL_ADIABATIC, WALL_ADIABATIC],
                 T_wall=[1.0, 0.0, 0.0, 0.0], eps=float(eps[i]), Ra=float(Ra[i]),
                 Da=float(Da[i]), Pr=1.0, Ste=float(Ste[i])) for i in range(n)]
    return cavs, dict(CAVITY_BATCH_OPTS), int(steps)


def batch_member(cav, opts, steps=0):
    """One cavity of a batch as a single-lattice workload (uniform porosity
    array, K and F_eps left to the solver's defaults)."""
    return make_case("batch_member", cav["nx"], cav["ny"], cav["bc_kind"], cav["T_wall"],
                     Ra=cav["Ra"], Da=cav["Da"], Pr=cav["Pr"], Ste=cav["Ste"], eps=cav["eps"],
                     steps=steps, H=cav.get("H", 0.0), **opts)


def gaussian_field(nx, ny, corr, seed):
    """Seeded Gaussian random field of unit standard deviation with the
    covariance exp(-r^2 / (2 corr^2)): white noise convolved (periodically,
    by FFT) with a Gaussian of width corr / sqrt(2), then normalised."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((ny, nx))
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    k2 = kx[None, :] ** 2 + ky[:, None] ** 2
    f = np.real(np.fft.ifft2(np.fft.fft2(xi) * np.exp(-k2 * corr * corr / 4.0)))
    return (f - f.mean()) / f.std()


def adjoint_cavity(n=512, steps=2000, seed=1, Ra=1e5, Da=1e-3, Ste=1.0, porosity=0.4,
                   corr=32.0, sigma=0.5):
    """Sec. 4.3 cavity (hot left wall, cold right wall, adiabatic top and
    bottom, initially solid at theta = 0, theta_m = 9.78/25 +- 0.02) whose
    permeability is K = Da H^2 exp(sigma xi), xi a Gaussian random field of
    correlation length corr (H = n); porosity uniform.  The parameters of
    the inverse problem use seed 1, its target run seed 2."""
    xi = gaussian_field(n, n, corr, seed)
    K = Da * float(n) ** 2 * np.exp(sigma * xi)
    return make_case("adjoint_cavity", n, n, [WALL_T, WALL_T, WALL_ADIABATIC, WALL_ADIABATIC],
                     [1.0, 0.0, 0.0, 0.0], Ra=Ra, Da=Da, Pr=1.0, Ste=Ste, eps=porosity, K=K,
                     steps=steps, T_init=0.0, T_s=THETA_M_CAVITY - 0.02,
                     T_l=THETA_M_CAVITY + 0.02, convective=1)


def periodic_box(nx, ny, T, fl_phase="liquid", Ra=1e5, Da=1e-2, Pr=1.0, Ste=1.0,
                 porosity=0.6, seed=0, **opts):
    """Fully periodic box for conservation checks; T is the uniform initial
    temperature (the caller may overwrite the state afterwards)."""
    return make_case("periodic_box", nx, ny, [PERIODIC] * 4, [0.0] * 4, Ra=Ra, Da=Da,
                     Pr=Pr, Ste=Ste, eps=porosity, T_init=T, **opts)


def random_state(nx, ny, seed, w9, w5, dT=0.3, T_mean=0.4, du=0.02):
    """A seeded random pre-collision state for step-by-step parity checks:
    f = w9 (1 + noise), g = w5 T (1 + noise) with T a smooth random field, and
    f_l a clipped smooth random field holding solid (0), mushy and liquid (1)
    cells.  The caller supplies the rest weights w9, w5.  Returns float32
    planar arrays f[9, ny, nx], g[5, ny, nx], fl[ny, nx]."""
    rng = np.random.default_rng(seed)
    w9 = np.asarray(w9, dtype=np.float64)
    w5 = np.asarray(w5, dtype=np.float64)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    T = T_mean + dT * np.sin(2 * math.pi * X / max(nx, 2) + rng.uniform(0, 6.3)) * \
        np.cos(2 * math.pi * Y / max(ny, 2) + rng.uniform(0, 6.3))
    T = T + 0.02 * rng.standard_normal((ny, nx))
    s = (T - T_mean) / dT
    fl = np.clip(0.5 + 1.5 * s + 0.05 * rng.standard_normal((ny, nx)), 0.0, 1.0)
    f = w9[:, None, None] * (1.0 + du * rng.standard_normal((9, ny, nx)))
    g = w5[:, None, None] * T[None] * (1.0 + 0.05 * rng.standard_normal((5, ny, nx)))
    return _f32(f), _f32(g), _f32(fl)
