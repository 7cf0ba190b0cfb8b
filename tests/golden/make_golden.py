#!/usr/bin/env python3
"""Write the oracle-generated expected values used by the full-size GPU
parity tests.  Calls only the FP64 oracle (oracle/) on the seeded workloads;
nothing here comes from the HIP path.

  corner_256_20000.npz   Sec. 4.2 setting at 256x256 (porosity 0.4, Ste 0.5),
                         20000 steps: T and f_l on sampled rows, the row fronts.
  cavity_1024_2000.npz   Sec. 4.3 setting at 1024x1024 (Ra 1e6, Da 1e-4, seed 3),
                         2000 steps: T, u, f_l on the melted strip next to the
                         hot wall and on sampled rows.
  cavity_1024_2000_diag.npz  the same run's whole-lattice reductions (the
                         quantities dmrt_diag reports: sums of rho over liquid
                         nodes, of sigma T + phi f_l / St, f_l and T, max |u|,
                         the liquid count and the row fronts).
  cavity_1024_long.npz   the same workload over its full 100000 steps, with
                         snapshots after 20000, 50000 and 100000 steps.
  batch_512_smallest.npz the three smallest cavities of the 512-cavity batch
                         (seed 4), each over the batch's 10000 steps: T, u,
                         f_l in full.
  gallium_200.npz        the Sec. 4.3 problem as the paper sets it up (200x200,
                         gallium in glass beads): T, u, f_l in full at Fourier
                         numbers 0.457 and 1.829 (209368 and 837931 steps).

Usage: python tests/golden/make_golden.py [corner|cavity|cavity_diag|cavity_long|batch|gallium ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1503_08406_amd import workloads as W  # noqa: E402

CORNER_ROWS = [0, 1, 2, 8, 32, 64, 100, 128, 160, 200, 240, 254, 255]
CAVITY_ROWS = [0, 1, 2, 100, 511, 512, 900, 1021, 1022, 1023]
CAVITY_STRIP = 48


def make_oracle(case, threads=None):
    opts = dict(case["opts"])
    n = threads or min(16, len(os.sched_getaffinity(0)))
    p = oracle.make_params(case["nx"], case["ny"], H=case["H"], bc_kind=case["bc_kind"],
                           T_wall=case["T_wall"], Ra=case["Ra"], Da=case["Da"], Pr=case["Pr"],
                           Ste=case["Ste"], nthreads=n, **opts)
    K = None if case["K"] is None else case["K"].astype(np.float64)
    return oracle.OracleSim(p, case["eps"].astype(np.float64), K, None)


def run(case, steps):
    opts = dict(case["opts"])
    p = oracle.make_params(case["nx"], case["ny"], H=case["H"], bc_kind=case["bc_kind"],
                           T_wall=case["T_wall"], Ra=case["Ra"], Da=case["Da"], Pr=case["Pr"],
                           Ste=case["Ste"], nthreads=min(16, len(os.sched_getaffinity(0))), **opts)
    K = None if case["K"] is None else case["K"].astype(np.float64)
    o = oracle.OracleSim(p, case["eps"].astype(np.float64), K, None)
    t = time.time()
    o.step(steps)
    print("%s: %d steps in %.1f s" % (case["name"], steps, time.time() - t), flush=True)
    return o.fields()


def front_rows(fl):
    out = np.zeros(fl.shape[0])
    for r in range(fl.shape[0]):
        row = fl[r]
        s0 = row[0] >= 0.5
        idx = np.nonzero((row >= 0.5) != s0)[0]
        if idx.size:
            i = idx[0]
            out[r] = (i - 1) + (row[i - 1] - 0.5) / (row[i - 1] - row[i]) + 1.0
    return out


def corner():
    F = run(W.corner(n=256, steps=20000), 20000)
    np.savez_compressed(os.path.join(HERE, "corner_256_20000.npz"), steps=20000,
                        rows=np.array(CORNER_ROWS), T=F["T"][CORNER_ROWS], fl=F["fl"][CORNER_ROWS],
                        front=front_rows(F["fl"]), T_max=np.abs(F["T"]).max())


def cavity():
    F = run(W.cavity(nx=1024, ny=1024, steps=2000), 2000)
    s = slice(0, CAVITY_STRIP)
    np.savez_compressed(os.path.join(HERE, "cavity_1024_2000.npz"), steps=2000,
                        rows=np.array(CAVITY_ROWS), strip=CAVITY_STRIP,
                        T_strip=F["T"][:, s].astype(np.float32),
                        ux_strip=F["ux"][:, s].astype(np.float32),
                        uy_strip=F["uy"][:, s].astype(np.float32),
                        fl_strip=F["fl"][:, s].astype(np.float32),
                        T_rows=F["T"][CAVITY_ROWS].astype(np.float32),
                        T_max=np.abs(F["T"]).max(),
                        u_max=max(np.abs(F["ux"]).max(), np.abs(F["uy"]).max()),
                        front=front_rows(F["fl"]))


def cavity_diag():
    case = W.cavity(nx=1024, ny=1024, steps=2000)
    F = run(case, 2000)
    liq = F["fl"] > 0
    fr = front_rows(F["fl"])
    eps, St = case["eps"].astype(np.float64), case["Ste"]
    np.savez_compressed(os.path.join(HERE, "cavity_1024_2000_diag.npz"), steps=2000,
                        mass=F["rho"][liq].sum(),
                        enthalpy=(F["T"] + eps * F["fl"] / St).sum(),  # sigma = 1
                        liquid=F["fl"].sum(), T_sum=F["T"].sum(), T_abs=np.abs(F["T"]).sum(),
                        u_max=np.sqrt(F["ux"] ** 2 + F["uy"] ** 2).max(), active=liq.sum(),
                        front_mean=fr.mean(), front_max=fr.max())


LONG_SNAPS = (20000, 50000, 100000)
LONG_STRIP = 192


def cavity_long():
    o = make_oracle(W.cavity(nx=1024, ny=1024, steps=100000),
                    threads=int(os.environ.get("ORACLE_THREADS", "0")) or None)
    out = dict(snaps=np.array(LONG_SNAPS), rows=np.array(CAVITY_ROWS), strip=LONG_STRIP)
    t = time.time()
    for n in LONG_SNAPS:
        o.step(n - o.time)
        F = o.fields()
        s = slice(0, LONG_STRIP)
        for k in ("T", "ux", "uy", "fl"):
            out["%s_strip_%d" % (k, n)] = F[k][:, s].astype(np.float32)
        out["T_rows_%d" % n] = F["T"][CAVITY_ROWS].astype(np.float32)
        out["T_max_%d" % n] = np.abs(F["T"]).max()
        out["u_max_%d" % n] = max(np.abs(F["ux"]).max(), np.abs(F["uy"]).max())
        out["front_%d" % n] = front_rows(F["fl"])
        out["liquid_beyond_strip_%d" % n] = float(F["fl"][:, LONG_STRIP:].max())
        print("cavity_long: step %d (%.0f s)" % (n, time.time() - t), flush=True)
        np.savez_compressed(os.path.join(HERE, "cavity_1024_long.npz"), **out)


def batch():
    cavs, opts, steps = W.cavity_batch()
    area = [c["nx"] * c["ny"] for c in cavs]
    index = sorted(range(len(cavs)), key=lambda i: (area[i], i))[:3]
    out = dict(steps=steps, index=np.array(index))
    for k, i in enumerate(index):
        F = run(W.batch_member(cavs[i], opts), steps)
        for n in ("T", "ux", "uy", "fl"):
            out["%s_%d" % (n, k)] = F[n]
    np.savez_compressed(os.path.join(HERE, "batch_512_smallest.npz"), **out)


GALLIUM_FO = (0.457, 1.829)


def gallium():
    case = W.gallium_cavity()
    o = make_oracle(case, threads=int(os.environ.get("ORACLE_THREADS", "0")) or None)
    alpha_l = o.derived["alpha_l"]  # Sec. 4.3 mapping, through the oracle
    steps = [int(round(fo * case["H"] ** 2 / alpha_l)) for fo in GALLIUM_FO]
    out = dict(fo=np.array(GALLIUM_FO), steps=np.array(steps))
    t = time.time()
    for k, n in enumerate(steps):
        o.step(n - o.time)
        F = o.fields()
        for q in ("T", "ux", "uy", "fl"):
            out["%s_%d" % (q, k)] = F[q].astype(np.float32)
        out["front_%d" % k] = front_rows(F["fl"])
        print("gallium: step %d (%.0f s)" % (n, time.time() - t), flush=True)
        np.savez_compressed(os.path.join(HERE, "gallium_200.npz"), **out)


if __name__ == "__main__":
    oracle.build(force=False)
    which = sys.argv[1:] or ["corner", "cavity"]
    for w in which:
        globals()[w]()
