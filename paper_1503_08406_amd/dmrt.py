"""Python binding of the HIP double-MRT solver (libdmrt.so, C ABI in
include/dmrt.h).  Argument marshalling only: every step of the method runs in
the library's kernels.  PyTorch supplies the HIP stream (and, when asked,
device tensors for outputs).  There is no CPU fallback: if the library is
missing, importing the binding raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DMRT_LIB_PATH selects another build of the same library (for timing two
# builds against each other); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("DMRT_LIB_PATH") or os.path.join(_HERE, "libdmrt.so")

DMRT_OK, DMRT_EINVAL, DMRT_ENOMEM, DMRT_EDEVICE, DMRT_ENONFINITE, DMRT_ESIZE = 0, -1, -2, -3, -4, -5
PERIODIC, WALL_T, WALL_ADIABATIC = 0, 1, 2


class DmrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dmrt error %d: %s" % (code, msg))
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("H", C.c_double)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int32 * 4), ("T_wall", C.c_double * 4)]


class Opts(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("Ma", "J", "lambda_", "alpha_ratio", "sigma_s", "sigma_l", "T_s", "T_l", "T0",
                 "T_init", "alpha_l", "varpi", "s_e", "s_eps", "s_q", "zeta_e", "zeta_nu",
                 "ergun_c", "fl_tol")] + \
              [("fl_maxit", C.c_int32), ("convective", C.c_int32), ("check_every", C.c_int32),
               ("graph_steps", C.c_int32), ("block_rows", C.c_int32), ("cells_per_lane", C.c_int32),
               ("stream", C.c_void_p),
               ("sigma_mode", C.c_int32), ("ke_mode", C.c_int32), ("latent_mode", C.c_int32),
               ("store_hint", C.c_int32), ("cps_ratio", C.c_double), ("cm_ratio", C.c_double),
               ("ks_ratio", C.c_double), ("km_ratio", C.c_double), ("record_mode", C.c_int32),
               ("steps_per_launch", C.c_int32), ("addressing", C.c_int32)]


class Cavity(C.Structure):
    _fields_ = [("grid", Grid), ("bc", BC), ("eps", C.c_double), ("Ra", C.c_double),
                ("Da", C.c_double), ("Pr", C.c_double), ("Ste", C.c_double)]


class Derived(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("H", "tau_nu", "nu_l", "nu_e", "alpha_l", "alpha_s", "gbeta", "K_default",
                 "tau_T_liquid", "tau_T_solid", "csT2")]


class Diag(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("mass", "enthalpy", "liquid", "T_sum", "u_max", "front_mean", "front_max")] + \
              [("active", C.c_int64), ("nonfinite", C.c_int64), ("step", C.c_int64)]


def _hip_runtimes():
    """Distinct HIP runtime files mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            return sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln})
    except OSError:
        return []


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdmrt.so not built at %s (run __graft_entry__.build())" % LIB_PATH)
    # PyTorch's HIP runtime must be loaded first: the library then binds to it
    # (same soname) instead of mapping a second runtime into the process.
    import torch  # noqa: F401
    import torch.cuda  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are mapped into the process: %s" % rts)
    P, FP, VP = C.c_void_p, C.POINTER(C.c_float), C.c_void_p
    sig = {
        "dmrt_opts_default": (None, [C.POINTER(Opts)]),
        "dmrt_derive": (C.c_int, [C.POINTER(Grid), C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.POINTER(Opts), C.POINTER(Derived)]),
        "dmrt_create": (C.c_int, [C.POINTER(Grid), VP, VP, VP, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.POINTER(BC), C.POINTER(Opts), C.POINTER(P)]),
        "dmrt_step": (C.c_int, [P, C.c_int64]),
        "dmrt_fields": (C.c_int, [P, VP, VP, VP, VP]),
        "dmrt_set_state": (C.c_int, [P, VP, VP, VP]),
        "dmrt_get_populations": (C.c_int, [P, VP, VP]),
        "dmrt_diag": (C.c_int, [P, C.POINTER(Diag)]),
        "dmrt_diag_noalloc": (C.c_int, [P, C.POINTER(Diag)]),
        "dmrt_get_derived": (C.c_int, [P, C.POINTER(Derived)]),
        "dmrt_step_counted": (C.c_int, [P, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "dmrt_state_bytes": (C.c_int64, [P]),
        "dmrt_launch_steps": (C.c_int32, [P]),
        "dmrt_save": (C.c_int, [P, VP, C.c_size_t]),
        "dmrt_load": (C.c_int, [P, VP, C.c_size_t]),
        "dmrt_set_porous": (C.c_int, [P, VP, VP, VP]),
        "dmrt_record": (C.c_int, [P, C.c_int64]),
        "dmrt_adjoint": (C.c_int, [P, VP, VP, VP, VP]),
        "dmrt_time": (C.c_int64, [P]),
        "dmrt_sync": (C.c_int, [P]),
        "dmrt_destroy": (None, [P]),
        "dmrt_last_error": (C.c_char_p, []),
        "dmrt_batch_create": (C.c_int, [C.c_int32, C.POINTER(Cavity), C.POINTER(Opts), C.POINTER(P)]),
        "dmrt_batch_step": (C.c_int, [P, C.c_int64]),
        "dmrt_batch_fields": (C.c_int, [P, C.c_int32, VP, VP, VP, VP]),
        "dmrt_batch_check": (C.c_int, [P, VP, VP]),
        "dmrt_batch_set_launch": (C.c_int, [P, C.c_int32, C.c_int32]),
        "dmrt_batch_get_launch": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "dmrt_batch_tune": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double)]),
        "dmrt_batch_get_derived": (C.c_int, [P, C.c_int32, C.POINTER(Derived)]),
        "dmrt_batch_cells": (C.c_int64, [P]),
        "dmrt_batch_time": (C.c_int64, [P]),
        "dmrt_batch_sync": (C.c_int, [P]),
        "dmrt_batch_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc):
    if rc != DMRT_OK:
        raise DmrtError(rc, _lib.dmrt_last_error().decode())
    return rc


def default_opts():
    o = Opts()
    _lib.dmrt_opts_default(C.byref(o))
    return o


def make_opts(**kw):
    o = default_opts()
    for k, v in kw.items():
        if k == "lambda":
            k = "lambda_"
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def derive(nx, ny, Ra, Da, Pr, Ste, H=0.0, **opts):
    g = Grid(nx, ny, H)
    d = Derived()
    _check(_lib.dmrt_derive(C.byref(g), Ra, Da, Pr, Ste, C.byref(make_opts(**opts)), C.byref(d)))
    return {n: getattr(d, n) for n, _ in Derived._fields_}


def _ptr(a):
    """Pointer of a float32 host array (numpy) or device tensor (torch)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if str(a.dtype) != "torch.float32" or not a.is_contiguous():
            raise TypeError("expected a contiguous float32 tensor, got %s" % (a.dtype,))
        return C.c_void_p(a.data_ptr())
    if a.dtype != np.float32 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous float32 array, got %s" % (a.dtype,))
    return a.ctypes.data_as(C.c_void_p)


class Solver:
    """One lattice on one GPU.  `case` is a workload dict of
    paper_1503_08406_amd.workloads; keyword arguments override its options."""

    def __init__(self, case, stream=None, **over):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the dmrt solver needs a ROCm GPU")
        self.torch = torch
        self.nx, self.ny = case["nx"], case["ny"]
        self.stream = stream if stream is not None else torch.cuda.Stream()
        opts = dict(case["opts"])
        opts.update(over)
        o = make_opts(**opts)
        o.stream = C.c_void_p(self.stream.cuda_stream)
        g = Grid(self.nx, self.ny, case["H"])
        bc = BC()
        for k in range(4):
            bc.kind[k] = case["bc_kind"][k]
            bc.T_wall[k] = case["T_wall"][k]
        self._keep = [np.ascontiguousarray(case["eps"], dtype=np.float32)]
        K = case["K"]
        F = case["Feps"]
        self._keep += [None if K is None else np.ascontiguousarray(K, dtype=np.float32),
                       None if F is None else np.ascontiguousarray(F, dtype=np.float32)]
        h = C.c_void_p()
        _check(_lib.dmrt_create(C.byref(g), _ptr(self._keep[0]), _ptr(self._keep[1]),
                                _ptr(self._keep[2]), case["Ra"], case["Da"], case["Pr"],
                                case["Ste"], C.byref(bc), C.byref(o), C.byref(h)))
        self._h = h
        d = Derived()
        _check(_lib.dmrt_get_derived(self._h, C.byref(d)))
        self.derived = {n: getattr(d, n) for n, _ in Derived._fields_}
        # changes whenever the library's recorded run is replaced or
        # discarded (record, set_porous), so that a backward pass can tell
        # whether the recording is still the one its forward pass made
        self.record_id = 0

    @property
    def handle(self):
        return self._h

    @property
    def launch_steps(self):
        """Time steps one launch of the step kernel advances (1 or 2)."""
        n = _lib.dmrt_launch_steps(self._h)
        if n < 0:
            _check(n)
        return n

    def close(self):
        if getattr(self, "_h", None):
            _lib.dmrt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self):
        return _lib.dmrt_time(self._h)

    def step(self, n=1):
        _check(_lib.dmrt_step(self._h, int(n)))

    def step_counted(self, n):
        mx = C.c_int32()
        mean = C.c_double()
        _check(_lib.dmrt_step_counted(self._h, int(n), C.byref(mx), C.byref(mean)))
        return mx.value, mean.value

    def sync(self):
        _check(_lib.dmrt_sync(self._h))

    def fields(self):
        shape = (self.ny, self.nx)
        out = {k: np.zeros(shape, np.float32) for k in ("T", "ux", "uy", "fl")}
        _check(_lib.dmrt_fields(self._h, _ptr(out["T"]), _ptr(out["ux"]), _ptr(out["uy"]),
                                _ptr(out["fl"])))
        return out

    def fields_device(self):
        """Fields written straight into device tensors."""
        t = self.torch
        out = {k: t.empty((self.ny, self.nx), dtype=t.float32, device="cuda")
               for k in ("T", "ux", "uy", "fl")}
        t.cuda.current_stream().synchronize()
        _check(_lib.dmrt_fields(self._h, _ptr(out["T"]), _ptr(out["ux"]), _ptr(out["uy"]),
                                _ptr(out["fl"])))
        return out

    def set_state(self, f=None, g=None, fl=None):
        conv = lambda a, q: None if a is None else np.ascontiguousarray(
            np.asarray(a, dtype=np.float32).reshape((q, self.ny, self.nx) if q else (self.ny, self.nx)))
        f, g, fl = conv(f, 9), conv(g, 5), conv(fl, 0)
        _check(_lib.dmrt_set_state(self._h, _ptr(f), _ptr(g), _ptr(fl)))

    def populations(self):
        fp = np.zeros((9, self.ny, self.nx), np.float32)
        gp = np.zeros((5, self.ny, self.nx), np.float32)
        _check(_lib.dmrt_get_populations(self._h, _ptr(fp), _ptr(gp)))
        return fp, gp

    def diag(self):
        d = Diag()
        _check(_lib.dmrt_diag(self._h, C.byref(d)))
        return {n: getattr(d, n) for n, _ in Diag._fields_}

    def diag_noalloc(self):
        """dmrt_diag_noalloc: the same reductions without any device
        allocation (the library's fixed scratch array)."""
        d = Diag()
        _check(_lib.dmrt_diag_noalloc(self._h, C.byref(d)))
        return {n: getattr(d, n) for n, _ in Diag._fields_}

    def save(self):
        n = _lib.dmrt_state_bytes(self._h)
        if n < 0:
            _check(int(n))
        buf = np.zeros(n, np.uint8)
        _check(_lib.dmrt_save(self._h, buf.ctypes.data_as(C.c_void_p), buf.nbytes))
        return buf

    def set_porous(self, eps, K=None, Feps=None):
        """Replace the porous fields (float32 [ny, nx]; K / Feps None: the
        defaults of dmrt_create)."""
        shape = (self.ny, self.nx)
        conv = lambda a: None if a is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(a, dtype=np.float32), shape))
        e, k, f = conv(eps), conv(K), conv(Feps)
        self.record_id += 1  # the library discards a recorded run here
        _check(_lib.dmrt_set_porous(self._h, _ptr(e), _ptr(k), _ptr(f)))

    def reset(self):
        """Back to the initial state (uniform T_init at rest)."""
        _check(_lib.dmrt_set_state(self._h, None, None, None))

    def record(self, n):
        """Advance n steps keeping what dmrt_adjoint needs."""
        self.record_id += 1
        _check(_lib.dmrt_record(self._h, int(n)))

    def adjoint(self, dL_dT=None, dL_dfl=None):
        """Gradients (dL/dlog K, dL/deps), float32 [ny, nx], of a loss of the
        fields at the end of the recorded run with the given adjoints.  With
        torch tensors the result is torch tensors on their device."""
        shape = (self.ny, self.nx)
        t = self.torch
        if isinstance(dL_dT, t.Tensor) or isinstance(dL_dfl, t.Tensor):
            ref = dL_dT if isinstance(dL_dT, t.Tensor) else dL_dfl
            conv = lambda a: None if a is None else a.detach().to(t.float32).reshape(shape).contiguous()
            gT, gf = conv(dL_dT), conv(dL_dfl)
            gk = t.empty(shape, dtype=t.float32, device=ref.device)
            ge = t.empty(shape, dtype=t.float32, device=ref.device)
            if ref.is_cuda:
                t.cuda.current_stream().synchronize()
        else:
            conv = lambda a: None if a is None else np.ascontiguousarray(
                np.asarray(a, dtype=np.float32).reshape(shape))
            gT, gf = conv(dL_dT), conv(dL_dfl)
            gk = np.zeros(shape, np.float32)
            ge = np.zeros(shape, np.float32)
        _check(_lib.dmrt_adjoint(self._h, _ptr(gT), _ptr(gf), _ptr(gk), _ptr(ge)))
        return gk, ge

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(_lib.dmrt_load(self._h, buf.ctypes.data_as(C.c_void_p), buf.nbytes))


class BatchSolver:
    """Many independent cavities advanced together, one or two steps per
    launch (steps_per_launch, default 2).
    `cavities` is a list of dicts with nx, ny, bc_kind, T_wall, eps (a
    scalar), Ra, Da, Pr, Ste and optionally H; keyword arguments are solver
    options shared by all cavities."""

    def __init__(self, cavities, stream=None, **opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the dmrt solver needs a ROCm GPU")
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        o = make_opts(**opts)
        o.stream = C.c_void_p(self.stream.cuda_stream)
        n = len(cavities)
        arr = (Cavity * n)()
        for i, c in enumerate(cavities):
            a = arr[i]
            a.grid = Grid(int(c["nx"]), int(c["ny"]), float(c.get("H", 0.0)))
            for k in range(4):
                a.bc.kind[k] = int(c["bc_kind"][k])
                a.bc.T_wall[k] = float(c["T_wall"][k])
            a.eps, a.Ra, a.Da, a.Pr, a.Ste = (float(c[k]) for k in ("eps", "Ra", "Da", "Pr", "Ste"))
        self.shapes = [(int(c["ny"]), int(c["nx"])) for c in cavities]
        h = C.c_void_p()
        _check(_lib.dmrt_batch_create(n, arr, C.byref(o), C.byref(h)))
        self._h = h
        self.ncav = n

    def close(self):
        if getattr(self, "_h", None):
            _lib.dmrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self):
        return _lib.dmrt_batch_time(self._h)

    @property
    def cells(self):
        return _lib.dmrt_batch_cells(self._h)

    def step(self, n=1):
        _check(_lib.dmrt_batch_step(self._h, int(n)))

    def sync(self):
        _check(_lib.dmrt_batch_sync(self._h))

    def fields(self, i):
        if not 0 <= i < self.ncav:
            raise IndexError("cavity %d out of range" % i)
        out = {k: np.zeros(self.shapes[i], np.float32) for k in ("T", "ux", "uy", "fl")}
        _check(_lib.dmrt_batch_fields(self._h, int(i), _ptr(out["T"]), _ptr(out["ux"]),
                                      _ptr(out["uy"]), _ptr(out["fl"])))
        return out

    def check(self):
        """Per-cavity (liquid node count, non-finite value count)."""
        liq = np.zeros(self.ncav, np.int64)
        bad = np.zeros(self.ncav, np.int64)
        _check(_lib.dmrt_batch_check(self._h, liq.ctypes.data_as(C.c_void_p),
                                     bad.ctypes.data_as(C.c_void_p)))
        return liq, bad

    def derived(self, i):
        d = Derived()
        _check(_lib.dmrt_batch_get_derived(self._h, int(i), C.byref(d)))
        return {n: getattr(d, n) for n, _ in Derived._fields_}

    def set_launch(self, rows, blocks=0):
        _check(_lib.dmrt_batch_set_launch(self._h, int(rows), int(blocks)))

    def launch(self):
        r, b = C.c_int32(), C.c_int32()
        _check(_lib.dmrt_batch_get_launch(self._h, C.byref(r), C.byref(b)))
        return r.value, b.value

    def tune(self, trial_steps=10, cache=None):
        """Pick the fastest launch shape by timing trial steps on a copy of
        the state (the library's tuner; results are unchanged).  With `cache`
        (a JSON file path) the choice is stored under a key made of the device
        name and the cavity sizes, and later batches of the same sizes reuse
        it without timing.  Returns (rows, blocks, ms_per_step or None)."""
        import hashlib
        import json
        key = None
        if cache:
            dev = self.torch.cuda.get_device_name(self.torch.cuda.current_device())
            sizes = hashlib.sha1(repr(self.shapes).encode()).hexdigest()[:16]
            key = "%s|%d|%s" % (dev, self.ncav, sizes)
            try:
                with open(cache) as fh:
                    hit = json.load(fh).get(key)
            except (OSError, ValueError):
                hit = None
            if hit:
                self.set_launch(hit["rows"], hit["blocks"])
                return hit["rows"], hit["blocks"], None
        r, b, ms = C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.dmrt_batch_tune(self._h, int(trial_steps), C.byref(r), C.byref(b), C.byref(ms)))
        if key:
            try:
                with open(cache) as fh:
                    db = json.load(fh)
            except (OSError, ValueError):
                db = {}
            db[key] = {"rows": r.value, "blocks": b.value, "ms_per_step": ms.value}
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(db, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return r.value, b.value, ms.value


def melting_run(solver, logK, eps, steps):
    """Differentiable run: (T, f_l) after `steps` steps from the initial state
    of `solver` with per-cell log-permeability logK and porosity eps (torch
    tensors [ny, nx]); gradients flow back to logK and eps through the
    library's discrete adjoint (checkpointed recomputation).

    The solver keeps one recorded run: a backward pass raises if the solver
    recorded another run (or had its porous fields replaced) after the
    forward pass it belongs to, instead of returning that run's gradient."""
    import torch

    class _MeltingRun(torch.autograd.Function):
        @staticmethod
        def forward(ctx, lk, ep):
            K = torch.exp(lk.detach().double()).float().cpu().numpy()
            solver.set_porous(ep.detach().float().cpu().numpy(), K)
            solver.reset()
            solver.record(steps)
            ctx.record_id = solver.record_id
            F = solver.fields_device()
            return F["T"].to(lk.device), F["fl"].to(lk.device)

        @staticmethod
        def backward(ctx, dT, dfl):
            if solver.record_id != ctx.record_id:
                raise RuntimeError(
                    "melting_run: the solver recorded another run after this one's forward "
                    "pass; call backward before the next melting_run on the same solver, or "
                    "use one solver per differentiated run")
            dev = dT.device if dT is not None else dfl.device
            z = torch.zeros((solver.ny, solver.nx), dtype=torch.float32, device="cuda")
            gT = z if dT is None else dT.to("cuda")
            gF = z if dfl is None else dfl.to("cuda")
            gk, ge = solver.adjoint(gT, gF)
            return gk.to(dev), ge.to(dev)

    return _MeltingRun.apply(logK, eps)
