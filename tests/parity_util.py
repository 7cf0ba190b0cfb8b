"""Helpers shared by the GPU parity tests: build the HIP solver and the FP64
oracle on the same workload and compare them with the tolerances of the
parity contract (T: relative L-inf 1e-4; u: relative L-inf 1e-3;
f_l: L-inf 1e-3; front: 0.5 lattice units)."""
import numpy as np

from conftest import front_rows, oracle_from_case

TOL_T, TOL_U, TOL_FL, TOL_FRONT = 1e-4, 1e-3, 1e-3, 0.5


def pair(case, gpu_over=None, **over):
    """(HIP solver, oracle) on the same workload; gpu_over holds options only
    the HIP side takes (launch options, its FP32 enthalpy tolerance)."""
    from paper_1503_08406_amd.dmrt import Solver
    g = dict(over)
    g.update(gpu_over or {})
    return Solver(case, **g), oracle_from_case(case, **over)


def field_errors(fg, fo):
    """Errors of GPU fields fg against oracle fields fo (dicts)."""
    Tmax = max(np.abs(fo["T"]).max(), 1e-30)
    umax = max(np.abs(fo["ux"]).max(), np.abs(fo["uy"]).max(), 1e-30)
    du = max(np.abs(fg["ux"] - fo["ux"]).max(), np.abs(fg["uy"] - fo["uy"]).max())
    return dict(T=np.abs(fg["T"] - fo["T"]).max() / Tmax,
                u=du / umax, u_abs=du, umax=umax,
                fl=np.abs(fg["fl"] - fo["fl"]).max(),
                front=np.abs(front_rows(fg["fl"]) - front_rows(fo["fl"])).max())


def assert_fields_close(fg, fo, tol_T=TOL_T, tol_u=TOL_U, tol_fl=TOL_FL, tol_front=TOL_FRONT,
                        u_floor=0.0, label=""):
    e = field_errors(fg, fo)
    msg = "%s %s" % (label, {k: float("%.3g" % v) for k, v in e.items()})
    assert e["T"] <= tol_T, msg
    assert e["u"] <= tol_u or e["u_abs"] <= u_floor, msg
    assert e["fl"] <= tol_fl, msg
    assert e["front"] <= tol_front, msg
    return e


def oracle_diag(case, Fo):
    """The reductions dmrt_diag reports, formed from oracle fields: sum of rho
    over liquid nodes (Eq. 24), sum of sigma T + phi f_l / St (Eqs. 3, 40),
    sum of f_l, sum of T (Eq. 33), max |u| (Eq. 26), the liquid count (Sec. 4)
    and the mean and max of the row fronts."""
    opts = case["opts"]
    ss, sl = opts.get("sigma_s", 1.0), opts.get("sigma_l", 1.0)
    fl, T = Fo["fl"], Fo["T"]
    eps = case["eps"].astype(np.float64)
    liq = fl > 0
    fr = front_rows(fl)
    return dict(mass=float(Fo["rho"][liq].sum()),
                enthalpy=float(((ss + fl * (sl - ss)) * T + eps * fl / case["Ste"]).sum()),
                liquid=float(fl.sum()), T_sum=float(T.sum()),
                u_max=float(np.sqrt(Fo["ux"] ** 2 + Fo["uy"] ** 2).max()),
                active=int(liq.sum()), front_mean=float(fr.mean()), front_max=float(fr.max()),
                T_abs=float(np.abs(T).sum()))


def assert_diag_close(dg, do, label=""):
    """dmrt_diag against oracle_diag: sums to relative 1e-6 (T against the sum
    of |T|), max |u| to relative 1e-3, the liquid count exactly, fronts to
    0.5 lattice units."""
    rel = lambda a, b, s: abs(a - b) / max(abs(s), 1e-300)
    e = dict(mass=rel(dg["mass"], do["mass"], do["mass"]),
             enthalpy=rel(dg["enthalpy"], do["enthalpy"], do["enthalpy"]),
             liquid=rel(dg["liquid"], do["liquid"], do["liquid"]),
             T_sum=rel(dg["T_sum"], do["T_sum"], do["T_abs"]),
             u_max=rel(dg["u_max"], do["u_max"], do["u_max"]))
    msg = "%s %s active %d/%d front %.4f/%.4f" % (
        label, {k: float("%.3g" % v) for k, v in e.items()}, dg["active"], do["active"],
        dg["front_mean"], do["front_mean"])
    for k in ("mass", "enthalpy", "liquid", "T_sum"):
        assert e[k] <= 1e-6, msg
    assert e["u_max"] <= 1e-3, msg
    assert dg["active"] == do["active"], msg
    assert abs(dg["front_mean"] - do["front_mean"]) <= 0.5, msg
    assert abs(dg["front_max"] - do["front_max"]) <= 0.5, msg
    assert dg["nonfinite"] == 0, msg
    return e
