"""ctypes binding of the FP64 oracle (oracle/dmrt_oracle.c).

Test infrastructure only.  Field arrays crossing this interface are planar
float64: f[9, ny, nx], g[5, ny, nx], scalars [ny, nx].
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dmrt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_dmrt.so")
# DMRT_ORACLE_LIB loads another build of the oracle instead (the mutation
# tests load copies with one planted mistake); nothing is built then.
_LIB_OVERRIDE = os.environ.get("DMRT_ORACLE_LIB")

PERIODIC, WALL_T, WALL_ADIABATIC = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (OpenMP).  Always recompiles when force."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("H", C.c_double),
                ("bc_kind", C.c_int * 4), ("T_wall", C.c_double * 4),
                ("Ra", C.c_double), ("Da", C.c_double), ("Pr", C.c_double),
                ("Ste", C.c_double), ("Ma", C.c_double), ("J", C.c_double),
                ("lambda_", C.c_double), ("alpha_ratio", C.c_double),
                ("sigma_s", C.c_double), ("sigma_l", C.c_double),
                ("T_s", C.c_double), ("T_l", C.c_double), ("T0", C.c_double),
                ("T_init", C.c_double), ("alpha_l", C.c_double),
                ("varpi", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double),
                ("s_q", C.c_double), ("zeta_e", C.c_double), ("zeta_nu", C.c_double),
                ("ergun_c", C.c_double), ("fl_tol", C.c_double),
                ("fl_maxit", C.c_int), ("convective", C.c_int), ("nthreads", C.c_int),
                ("sigma_mode", C.c_int), ("cps_ratio", C.c_double), ("cm_ratio", C.c_double),
                ("ke_mode", C.c_int), ("ks_ratio", C.c_double), ("km_ratio", C.c_double),
                ("latent_mode", C.c_int)]


class Derived(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("H", "tau_nu", "nu_l", "nu_e", "alpha_l", "alpha_s", "gbeta",
                 "K_default", "cs2", "csT2", "tau_T_liquid", "tau_T_solid")]


_lib = None
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is None:
        if not _LIB_OVERRIDE and not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB_OVERRIDE or _LIB)
        lib.orc_default_params.argtypes = [C.POINTER(Params)]
        lib.orc_derive.argtypes = [C.POINTER(Params), C.POINTER(Derived)]
        lib.orc_derive.restype = C.c_int
        lib.orc_lattice.argtypes = [C.c_double, _IP, _IP, _DP, _DP, _DP, _IP, _IP, _DP, _DP, _DP]
        lib.orc_feq.argtypes = [C.c_double] * 4 + [_DP]
        lib.orc_meq.argtypes = [C.c_double] * 4 + [_DP]
        lib.orc_force_moments.argtypes = [C.c_double] * 5 + [_DP]
        lib.orc_geq.argtypes = [C.c_double] * 5 + [_DP]
        lib.orc_neq.argtypes = [C.c_double] * 5 + [C.c_int, _DP]
        lib.orc_collide_f.argtypes = [_DP] + [C.c_double] * 6 + [_DP, _DP]
        lib.orc_closure.argtypes = [C.c_double] * 8 + [_DP, _DP]
        lib.orc_enthalpy.argtypes = [C.c_double] * 10 + [C.c_int, _DP, _DP]
        lib.orc_ke.argtypes = [C.c_double] * 4
        lib.orc_ke.restype = C.c_double
        lib.orc_enthalpy.restype = C.c_int
        lib.orc_create.argtypes = [C.POINTER(Params), _DP, _DP, _DP]
        lib.orc_create.restype = C.c_void_p
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_set_state.argtypes = [C.c_void_p, _DP, _DP, _DP]
        lib.orc_get_state.argtypes = [C.c_void_p, _DP, _DP, _DP]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_time.argtypes = [C.c_void_p]
        lib.orc_time.restype = C.c_long
        lib.orc_fields.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP]
        lib.orc_post_collision.argtypes = [C.c_void_p, _DP, _DP]
        lib.orc_iter_stats.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.POINTER(C.c_long)]
        lib.orc_step_tl.argtypes = [C.c_void_p] + [_DP] * 8
        lib.orc_step_tl.restype = C.c_int
        lib.orc_step_ad.argtypes = [C.c_void_p] + [_DP] * 8
        lib.orc_step_ad.restype = C.c_int
        lib.orc_adjoint_run.argtypes = [C.c_void_p, C.c_long, _DP, _DP, _DP, _DP]
        lib.orc_adjoint_run.restype = C.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(_DP)


def default_params():
    p = Params()
    _load().orc_default_params(C.byref(p))
    return p


def make_params(nx, ny, **kw):
    """Params with the paper defaults, overridden by keyword arguments.
    bc_kind / T_wall take 4-sequences ordered x-, x+, y-, y+."""
    p = default_params()
    p.nx, p.ny = int(nx), int(ny)
    for k, v in kw.items():
        if k == "lambda":
            k = "lambda_"
        if k in ("bc_kind", "T_wall"):
            arr = getattr(p, k)
            for i in range(4):
                arr[i] = v[i]
        else:
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
    return p


def derive(p):
    d = Derived()
    rc = _load().orc_derive(C.byref(p), C.byref(d))
    if rc != 0:
        raise ValueError("orc_derive failed (%d)" % rc)
    return {n: getattr(d, n) for n, _ in Derived._fields_}


def lattice(varpi=-2.0):
    ex9 = (C.c_int * 9)(); ey9 = (C.c_int * 9)(); w9 = np.zeros(9)
    M = np.zeros(81); Minv = np.zeros(81)
    ex5 = (C.c_int * 5)(); ey5 = (C.c_int * 5)(); w5 = np.zeros(5)
    N = np.zeros(25); Ninv = np.zeros(25)
    _load().orc_lattice(varpi, ex9, ey9, _dp(w9), _dp(M), _dp(Minv), ex5, ey5, _dp(w5),
                        _dp(N), _dp(Ninv))
    return dict(e9=np.array([list(ex9), list(ey9)]).T, w9=w9, M=M.reshape(9, 9),
                Minv=Minv.reshape(9, 9), e5=np.array([list(ex5), list(ey5)]).T, w5=w5,
                N=N.reshape(5, 5), Ninv=Ninv.reshape(5, 5))


def feq(rho, ux, uy, phi):
    out = np.zeros(9); _load().orc_feq(rho, ux, uy, phi, _dp(out)); return out


def meq(rho, ux, uy, phi):
    out = np.zeros(9); _load().orc_meq(rho, ux, uy, phi, _dp(out)); return out


def force_moments(ux, uy, Fx, Fy, phi):
    out = np.zeros(9); _load().orc_force_moments(ux, uy, Fx, Fy, phi, _dp(out)); return out


def geq(T, ux, uy, sigma, varpi=-2.0):
    out = np.zeros(5); _load().orc_geq(T, ux, uy, sigma, varpi, _dp(out)); return out


def neq(T, ux, uy, sigma, varpi=-2.0, convective=1):
    out = np.zeros(5); _load().orc_neq(T, ux, uy, sigma, varpi, convective, _dp(out)); return out


def collide_f(f, rho, ux, uy, Fx, Fy, phi, s):
    f = np.ascontiguousarray(f, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros(9)
    _load().orc_collide_f(_dp(f), rho, ux, uy, Fx, Fy, phi, _dp(s), _dp(out))
    return out


def closure(jx, jy, phi, nu_l, Ke, Ce, Gx, Gy):
    u = np.zeros(2); F = np.zeros(2)
    _load().orc_closure(jx, jy, phi, nu_l, Ke, Ce, Gx, Gy, _dp(u), _dp(F))
    return u, F


def enthalpy(Tstar, fl_old, eps, Ste, sigma_s=1.0, sigma_l=1.0, T_s=-0.02, T_l=0.02,
             tol=1e-12, maxit=200, cps=1.0):
    fl = C.c_double(); T = C.c_double()
    it = _load().orc_enthalpy(Tstar, fl_old, eps, Ste, sigma_s, sigma_l, cps, T_s, T_l, tol,
                              maxit, C.byref(fl), C.byref(T))
    return fl.value, T.value, it


def ke(phi, fl, ks_ratio, km_ratio):
    """k_e / k_l from Eq. (8)."""
    return _load().orc_ke(phi, fl, ks_ratio, km_ratio)


class OracleSim:
    """Whole-lattice FP64 simulation.  eps is required; K / Feps may be None."""

    def __init__(self, params, eps, K=None, Feps=None):
        lib = _load()
        self.p = params
        self.nx, self.ny = params.nx, params.ny
        shape = (self.ny, self.nx)
        self._eps = np.ascontiguousarray(np.broadcast_to(eps, shape), dtype=np.float64)
        self._K = None if K is None else np.ascontiguousarray(np.broadcast_to(K, shape), dtype=np.float64)
        self._F = None if Feps is None else np.ascontiguousarray(np.broadcast_to(Feps, shape), dtype=np.float64)
        h = lib.orc_create(C.byref(params), _dp(self._eps),
                           _dp(self._K) if self._K is not None else None,
                           _dp(self._F) if self._F is not None else None)
        if not h:
            raise ValueError("orc_create rejected the parameters")
        self._h = C.c_void_p(h)
        self.derived = derive(params)

    def close(self):
        if getattr(self, "_h", None):
            _load().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self):
        return _load().orc_time(self._h)

    def step(self, n=1):
        _load().orc_step(self._h, int(n))

    def set_state(self, f, g, fl):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(5, self.ny, self.nx)
        fl = np.ascontiguousarray(fl, dtype=np.float64).reshape(self.ny, self.nx)
        _load().orc_set_state(self._h, _dp(f), _dp(g), _dp(fl))

    def get_state(self):
        f = np.zeros((9, self.ny, self.nx)); g = np.zeros((5, self.ny, self.nx))
        fl = np.zeros((self.ny, self.nx))
        _load().orc_get_state(self._h, _dp(f), _dp(g), _dp(fl))
        return f, g, fl

    def fields(self):
        shape = (self.ny, self.nx)
        T, ux, uy, fl, rho = (np.zeros(shape) for _ in range(5))
        _load().orc_fields(self._h, _dp(T), _dp(ux), _dp(uy), _dp(fl), _dp(rho))
        return dict(T=T, ux=ux, uy=uy, fl=fl, rho=rho)

    def post_collision(self):
        fp = np.zeros((9, self.ny, self.nx)); gp = np.zeros((5, self.ny, self.nx))
        _load().orc_post_collision(self._h, _dp(fp), _dp(gp))
        return fp, gp

    def _arr(self, a, q=0):
        if a is None:
            return None
        shape = (q, self.ny, self.nx) if q else (self.ny, self.nx)
        return np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)

    def step_tl(self, df, dg, dfl, dlnK=None, deps=None):
        """Tangent of one step at the current state (planar arrays); returns
        (dfn, dgn, dfln).  The state is not changed."""
        a = [self._arr(df, 9), self._arr(dg, 5), self._arr(dfl), self._arr(dlnK), self._arr(deps)]
        outs = [np.zeros((9, self.ny, self.nx)), np.zeros((5, self.ny, self.nx)),
                np.zeros((self.ny, self.nx))]
        rc = _load().orc_step_tl(self._h, *[None if x is None else _dp(x) for x in a],
                                 *[_dp(x) for x in outs])
        if rc != 0:
            raise ValueError("orc_step_tl refused the model (%d)" % rc)
        return tuple(outs)

    def step_ad(self, bfn, bgn, bfln):
        """Transpose of step_tl: (bf, bg, bfl, blnK, beps)."""
        a = [self._arr(bfn, 9), self._arr(bgn, 5), self._arr(bfln)]
        outs = [np.zeros((9, self.ny, self.nx)), np.zeros((5, self.ny, self.nx))] + \
               [np.zeros((self.ny, self.nx)) for _ in range(3)]
        rc = _load().orc_step_ad(self._h, *[_dp(x) for x in a], *[_dp(x) for x in outs])
        if rc != 0:
            raise ValueError("orc_step_ad refused the model (%d)" % rc)
        return tuple(outs)

    def adjoint_run(self, n, dL_dT=None, dL_dfl=None):
        """Gradients (dL/dln K, dL/deps) of a loss of T and f_l after n steps
        from the current state; the state is not changed."""
        a = [self._arr(dL_dT), self._arr(dL_dfl)]
        gk, ge = np.zeros((self.ny, self.nx)), np.zeros((self.ny, self.nx))
        rc = _load().orc_adjoint_run(self._h, int(n), *[None if x is None else _dp(x) for x in a],
                                     _dp(gk), _dp(ge))
        if rc != 0:
            raise ValueError("orc_adjoint_run failed (%d)" % rc)
        return gk, ge

    def iter_stats(self):
        mx = C.c_long(); sm = C.c_long()
        _load().orc_iter_stats(self._h, C.byref(mx), C.byref(sm))
        return mx.value, sm.value
