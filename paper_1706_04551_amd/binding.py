"""ctypes binding of libnhswe.so (include/nhswe.h): argument marshalling only.

Every step of the time stepper runs in the library's HIP kernels; this module
converts numpy arrays to host pointers and back.  It raises if the library has
not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libnhswe.so")

NH_FP64, NH_FP32 = 0, 1
STATUS = {0: "NH_OK", -1: "NH_EINVAL", -2: "NH_ENOMEM", -3: "NH_EDEVICE",
          -4: "NH_ENOCONV", -5: "NH_ENONFINITE", -6: "NH_ENEGDEPTH",
          -8: "NH_ESTATE"}

_DP = C.POINTER(C.c_double)


class NhGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double),
                ("dy", C.c_double)]


class NhParams(C.Structure):
    _fields_ = [("g", C.c_double), ("cfl", C.c_double),
                ("delta", C.c_double), ("dry_eps", C.c_double),
                ("precision", C.c_int32), ("nh_on", C.c_int32),
                ("breaking_on", C.c_int32), ("b1", C.c_double),
                ("b2", C.c_double), ("solve_max_iter", C.c_int32),
                ("check_every", C.c_int32), ("solve_tol", C.c_double),
                ("omega_schedule", _DP), ("n_omega", C.c_int32),
                ("fixed_dt", C.c_int32), ("dt", C.c_double),
                ("manning", C.c_double), ("open_sides", C.c_int32),
                ("periodic", C.c_int32), ("w_advection", C.c_int32),
                ("solve_path", C.c_int32), ("solve_norm", C.c_int32),
                ("wait_polls", C.c_int32)]


class NhDeviceViews(C.Structure):
    _fields_ = [("H", C.c_void_p), ("h", C.c_void_p), ("hu", C.c_void_p),
                ("hv", C.c_void_p), ("w", C.c_void_p)]


class NhStats(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_next", C.c_double),
                ("dt_last", C.c_double), ("step", C.c_int64),
                ("sweeps", C.c_int32 * 2), ("measure", C.c_double),
                ("sweeps_total", C.c_int64), ("solves_total", C.c_int64),
                ("clamped_mass", C.c_double), ("last_status", C.c_int32),
                ("mass", C.c_double), ("nondominant", C.c_int64),
                ("adjoint_sweeps", C.c_int64)]


class NhProfile(C.Structure):
    _fields_ = [("fv_ms", C.c_double), ("assemble_ms", C.c_double),
                ("solve_ms", C.c_double), ("correct_ms", C.c_double),
                ("fv_launches", C.c_int64), ("assemble_launches", C.c_int64),
                ("solve_launches", C.c_int64),
                ("correct_launches", C.c_int64),
                ("sweep_kernel_ms", C.c_double),
                ("sweep_kernel_launches", C.c_int64),
                ("sweep_kernel_sweeps", C.c_int64),
                ("sweep_kernel_corner_sweeps", C.c_double),
                ("solve_kernel_ms", C.c_double),
                ("solve_kernel_launches", C.c_int64),
                ("solve_kernel_sweeps", C.c_int64)]


_lib = None


def lib():
    """Load libnhswe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        # torch first: it brings its own HIP runtime, and the library must
        # bind to that same runtime (one set of devices, streams and device
        # pointers in the process); loaded the other way round, torch finds
        # the runtime already loaded and sees no device
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.nh_create.argtypes = [C.POINTER(NhGrid), C.POINTER(NhParams), vp,
                                C.POINTER(vp)]
        L.nh_set_bathymetry.argtypes = [vp, _DP]
        L.nh_set_relaxation.argtypes = [vp] + [_DP] * 6
        L.nh_set_state.argtypes = [vp, _DP, _DP, _DP, _DP, _DP]
        L.nh_step.argtypes = [vp, _DP]
        L.nh_run.argtypes = [vp, C.c_int64]
        L.nh_read_state.argtypes = [vp, _DP, _DP, _DP, _DP, _DP]
        L.nh_bind_device_buffers.argtypes = [vp, C.POINTER(NhDeviceViews)]
        L.nh_get_stats.argtypes = [vp, C.POINTER(NhStats)]
        L.nh_profile.argtypes = [vp, C.c_int32]
        L.nh_get_profile.argtypes = [vp, C.POINTER(NhProfile)]
        L.nh_destroy.argtypes = [vp]
        L.nh_destroy.restype = None
        i32 = C.c_int32
        L.nh_adjoint_run.argtypes = [vp, C.c_int64, i32, C.POINTER(i32), _DP,
                                     i32, C.c_double, _DP, _DP, _DP, _DP, _DP]
        L.nh_ensemble_create.argtypes = [i32, C.POINTER(NhGrid),
                                         C.POINTER(NhParams), vp,
                                         C.POINTER(vp)]
        L.nh_ensemble_set_bathymetry.argtypes = [vp, i32, _DP]
        L.nh_ensemble_set_state.argtypes = [vp, i32, _DP, _DP, _DP, _DP, _DP]
        L.nh_ensemble_set_tile.argtypes = [vp, i32, i32, i32]
        L.nh_ensemble_get_tile.argtypes = [vp, i32, C.POINTER(i32),
                                           C.POINTER(i32)]
        L.nh_ensemble_tune.argtypes = [vp, i32]
        L.nh_ensemble_run.argtypes = [vp, C.c_int64]
        L.nh_ensemble_run_graph.argtypes = [vp, C.c_int64]
        L.nh_ensemble_read_state.argtypes = [vp, i32, _DP, _DP, _DP, _DP,
                                             _DP]
        L.nh_ensemble_get_stats.argtypes = [vp, i32, C.POINTER(NhStats)]
        L.nh_ensemble_profile.argtypes = [vp, i32]
        L.nh_ensemble_get_profile.argtypes = [vp, C.POINTER(NhProfile)]
        L.nh_ensemble_destroy.argtypes = [vp]
        L.nh_ensemble_destroy.restype = None
        L.nh_run_noalloc.argtypes = [C.POINTER(NhGrid), C.POINTER(NhParams),
                                     vp, vp, vp, vp, vp, vp, vp, C.c_int64,
                                     C.POINTER(NhStats)]
        L.nh_last_error.restype = C.c_char_p
        L.nh_version.restype = C.c_char_p
        for f in ("nh_create", "nh_set_bathymetry", "nh_set_relaxation",
                  "nh_set_state", "nh_step",
                  "nh_run", "nh_read_state", "nh_bind_device_buffers", "nh_get_stats", "nh_profile",
                  "nh_get_profile", "nh_adjoint_run", "nh_ensemble_create",
                  "nh_ensemble_set_bathymetry", "nh_ensemble_set_state",
                  "nh_ensemble_set_tile", "nh_ensemble_get_tile",
                  "nh_ensemble_tune", "nh_ensemble_run",
                  "nh_ensemble_run_graph",
                  "nh_ensemble_read_state", "nh_ensemble_get_stats",
                  "nh_ensemble_profile", "nh_ensemble_get_profile",
                  "nh_run_noalloc"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class NhError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().nh_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")
        self.status = status


def _check(st, where):
    if st != 0:
        raise NhError(st, where)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_DP)


def _f64(a, shape):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def _params(*, g=9.81, cfl=0.9, delta=1e-5, dry_eps=1e-10, precision="f64",
            nh_on=1, breaking_on=0, b1=0.15, b2=0.5, solve_max_iter=200000,
            check_every=1, solve_tol=1e-10, omega=None, fixed_dt=0,
            dt_fixed=0.0, manning=0.0, open_sides=0, periodic=0,
            w_advection=0, solve_path=0, solve_norm=0, wait_polls=0):
    """nh_params and the relaxation schedule array it points to (the caller
    keeps the array alive until the create call returns)."""
    om = None if omega is None else np.ascontiguousarray(
        np.asarray(omega, dtype=np.float64).ravel())
    prec = {"f64": NH_FP64, "f32": NH_FP32}[precision]
    par = NhParams(g, cfl, delta, dry_eps, prec, nh_on, breaking_on, b1, b2,
                   solve_max_iter, check_every, solve_tol, _ptr(om),
                   0 if om is None else len(om), fixed_dt, dt_fixed,
                   manning, open_sides, periodic, w_advection, solve_path,
                   solve_norm, wait_polls)
    return par, om


def _stats_dict(s: "NhStats") -> dict:
    return dict(t=s.t, dt=s.dt_next, dt_last=s.dt_last, step=s.step,
                sweeps1=s.sweeps[0], sweeps2=s.sweeps[1], measure=s.measure,
                sweeps_total=s.sweeps_total, solves=s.solves_total,
                clamped=s.clamped_mass, status=s.last_status, mass=s.mass,
                nondominant=s.nondominant, adjoint_sweeps=s.adjoint_sweeps)


class Solver:
    """One grid on one HIP stream (see include/nhswe.h)."""

    def __init__(self, nx, ny, dx, dy, *, stream=None, **params):
        self.nx, self.ny = int(nx), int(ny)
        self.is1d = self.ny == 1
        self.cshape = (self.nx + 1,) if self.is1d else (self.ny + 1,
                                                         self.nx + 1)
        grid = NhGrid(self.nx, self.ny, float(dx), float(dy))
        par, self._omega = _params(**params)
        self.precision = params.get("precision", "f64")
        self._bound = {}
        h = C.c_void_p()
        st = lib().nh_create(C.byref(grid), C.byref(par),
                             C.c_void_p(stream) if stream else None,
                             C.byref(h))
        _check(st, "nh_create")
        self._h = h

    @classmethod
    def from_case(cls, case, **over):
        kw = case.param_dict()
        kw.pop("nx"), kw.pop("ny"), kw.pop("dx"), kw.pop("dy")
        kw["precision"] = case.precision
        kw.update(over)
        s = cls(case.nx, case.ny, case.dx, case.dy, **kw)
        s.set_bathymetry(case.H)
        s.set_state(case.h, case.hu, case.hv)
        return s

    def close(self):
        if getattr(self, "_h", None):
            lib().nh_destroy(self._h)   # synchronises the solver's stream
            self._h = None
        self._bound = {}                # then the borrowed tensors may go

    __del__ = close

    @property
    def shape(self):
        return (self.ny, self.nx)

    def bind(self, H=None, h=None, hu=None, hv=None, w=None):
        """Borrow device tensors for the bathymetry and the state
        (nh_bind_device_buffers): contiguous, on the solver's device, of the
        solver's precision (float64, or float32 in FP32 bulk), with the cell
        count (H, h, hu, hv) or the corner count (w).  Bound h, hu (and hv in
        2D) become the state; the solver then steps them in place on its
        stream (create it on torch's current stream to keep torch's work on
        the tensors in order).  In FP32 bulk the h tensor holds
        s = h - max(H, 0) (the surface elevation over water, the depth on
        land), the depth storage of such grids.  The tensors stay referenced
        here."""
        import torch
        dtype = torch.float64 if self.precision == "f64" else torch.float32
        ncell, ncorn = self.nx * self.ny, int(np.prod(self.cshape))
        views, keep = NhDeviceViews(), {}
        for name, t, n in (("H", H, ncell), ("h", h, ncell), ("hu", hu, ncell),
                           ("hv", hv, ncell), ("w", w, ncorn)):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or not t.is_cuda:
                raise TypeError(f"{name}: a device tensor is required")
            if t.dtype != dtype:
                raise TypeError(f"{name}: dtype {t.dtype}, the solver uses "
                                f"{dtype}")
            if not t.is_contiguous() or t.numel() != n:
                raise ValueError(f"{name}: a contiguous tensor of {n} "
                                 "elements is required")
            setattr(views, name, t.data_ptr())
            keep[name] = t
        _check(lib().nh_bind_device_buffers(self._h, C.byref(views)),
               "nh_bind_device_buffers")
        self._bound.update(keep)

    def set_bathymetry(self, H):
        H = _f64(H, self.shape)
        _check(lib().nh_set_bathymetry(self._h, _ptr(H)), "nh_set_bathymetry")

    def set_relaxation(self, widths, h=None, hu=None, hv=None, w=None,
                       p=None):
        """Generation/absorption zones: widths (west, east, south, north)
        in metres; targets default to still water (the absorbing zone)."""
        wd = _f64(widths, (4,))
        t = [_f64(a, self.shape) for a in (h, hu, hv)] + \
            [_f64(a, self.cshape) for a in (w, p)]
        _check(lib().nh_set_relaxation(self._h, _ptr(wd),
                                       *[_ptr(a) for a in t]),
               "nh_set_relaxation")

    def set_state(self, h, hu, hv=None, w=None, p=None):
        h, hu = _f64(h, self.shape), _f64(hu, self.shape)
        hv = _f64(hv, self.shape)
        w, p = _f64(w, self.cshape), _f64(p, self.cshape)
        _check(lib().nh_set_state(self._h, _ptr(h), _ptr(hu), _ptr(hv),
                                  _ptr(w), _ptr(p)), "nh_set_state")

    def step(self) -> float:
        dt = C.c_double(0.0)
        _check(lib().nh_step(self._h, C.byref(dt)), "nh_step")
        return dt.value

    def run(self, n: int):
        _check(lib().nh_run(self._h, int(n)), "nh_run")

    def run_status(self, n: int) -> int:
        return lib().nh_run(self._h, int(n))

    def state(self):
        out = {k: np.zeros(self.shape) for k in ("h", "hu", "hv")}
        out["w"] = np.zeros(self.cshape)
        out["p"] = np.zeros(self.cshape)
        _check(lib().nh_read_state(self._h, _ptr(out["h"]), _ptr(out["hu"]),
                                   _ptr(out["hv"]), _ptr(out["w"]),
                                   _ptr(out["p"])), "nh_read_state")
        return out

    def stats(self) -> dict:
        s = NhStats()
        _check(lib().nh_get_stats(self._h, C.byref(s)), "nh_get_stats")
        return _stats_dict(s)

    def profile(self, on=True):
        """nh_profile: False/0 off, True/1 every phase, n >= 2 only the sweep
        batch of one relaxation cycle in n (low overhead)."""
        _check(lib().nh_profile(self._h, int(on)), "nh_profile")

    def adjoint(self, nsteps: int, gauges, target, ckpt_every: int = 100,
                adj_tol: float = 1e-8) -> dict:
        """Misfit J of nsteps steps from the current state against
        target[nsteps][ngauges] at the gauge cells (flat indices), and its
        gradients (nh_adjoint_run): dh0, dhu0, dhv0 w.r.t. the initial state,
        dH w.r.t. the bathymetry at fixed initial state."""
        g = np.ascontiguousarray(np.asarray(gauges, dtype=np.int32).ravel())
        t = np.ascontiguousarray(np.asarray(target, dtype=np.float64))
        if t.shape != (int(nsteps), g.size):
            raise ValueError("target must be [nsteps, ngauges]")
        J = C.c_double(0.0)
        out = {k: np.zeros(self.shape) for k in ("dh0", "dhu0", "dhv0", "dH")}
        _check(lib().nh_adjoint_run(
            self._h, int(nsteps), int(g.size),
            g.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(t), int(ckpt_every),
            float(adj_tol), C.byref(J), _ptr(out["dh0"]), _ptr(out["dhu0"]),
            _ptr(out["dhv0"]), _ptr(out["dH"])), "nh_adjoint_run")
        out["J"] = J.value
        return out

    def get_profile(self) -> dict:
        p = NhProfile()
        _check(lib().nh_get_profile(self._h, C.byref(p)), "nh_get_profile")
        return {k: getattr(p, k) for k, _ in NhProfile._fields_}


class Ensemble:
    """Independent 2D grids advanced together (nh_ensemble_* in
    include/nhswe.h).  Member k has the layout of a Solver on its grid."""

    def __init__(self, grids, params, stream=None):
        """grids: list of (nx, ny, dx, dy); params: list of keyword dicts of
        Solver (one per member)."""
        n = len(grids)
        if n != len(params) or n == 0:
            raise ValueError("need one parameter dict per grid")
        G = (NhGrid * n)()
        P = (NhParams * n)()
        keep = []
        self.shapes, self.cshapes = [], []
        for k, ((nx, ny, dx, dy), kw) in enumerate(zip(grids, params)):
            G[k] = NhGrid(int(nx), int(ny), float(dx), float(dy))
            par, om = _params(**kw)
            P[k] = par
            keep.append(om)
            self.shapes.append((int(ny), int(nx)))
            self.cshapes.append((int(ny) + 1, int(nx) + 1))
        h = C.c_void_p()
        st = lib().nh_ensemble_create(n, G, P,
                                      C.c_void_p(stream) if stream else None,
                                      C.byref(h))
        _check(st, "nh_ensemble_create")
        self._h = h
        self.n = n

    @classmethod
    def from_cases(cls, cases, stream=None, **over):
        grids, params = [], []
        for c in cases:
            kw = c.param_dict()
            grids.append((kw.pop("nx"), kw.pop("ny"), kw.pop("dx"),
                          kw.pop("dy")))
            kw["precision"] = c.precision
            kw.update(over)
            params.append(kw)
        e = cls(grids, params, stream=stream)
        for k, c in enumerate(cases):
            e.set_bathymetry(k, c.H)
            e.set_state(k, c.h, c.hu, c.hv)
        return e

    def close(self):
        if getattr(self, "_h", None):
            lib().nh_ensemble_destroy(self._h)
            self._h = None

    __del__ = close

    def set_bathymetry(self, k, H):
        H = _f64(H, self.shapes[k])
        _check(lib().nh_ensemble_set_bathymetry(self._h, k, _ptr(H)),
               "nh_ensemble_set_bathymetry")

    def set_state(self, k, h, hu, hv=None, w=None, p=None):
        sh, cs = self.shapes[k], self.cshapes[k]
        h, hu, hv = _f64(h, sh), _f64(hu, sh), _f64(hv, sh)
        w, p = _f64(w, cs), _f64(p, cs)
        _check(lib().nh_ensemble_set_state(self._h, k, _ptr(h), _ptr(hu),
                                           _ptr(hv), _ptr(w), _ptr(p)),
               "nh_ensemble_set_state")

    def set_tile(self, k, bx, by):
        _check(lib().nh_ensemble_set_tile(self._h, k, bx, by),
               "nh_ensemble_set_tile")

    def tile(self, k):
        bx, by = C.c_int32(), C.c_int32()
        _check(lib().nh_ensemble_get_tile(self._h, k, C.byref(bx),
                                          C.byref(by)), "nh_ensemble_get_tile")
        return bx.value, by.value

    def tune(self, reps: int = 3):
        _check(lib().nh_ensemble_tune(self._h, reps), "nh_ensemble_tune")

    def run(self, n: int):
        _check(lib().nh_ensemble_run(self._h, int(n)), "nh_ensemble_run")

    def run_status(self, n: int) -> int:
        return lib().nh_ensemble_run(self._h, int(n))

    def run_graph(self, n: int):
        """n steps replayed from a graph of one step (solve_path 2)."""
        _check(lib().nh_ensemble_run_graph(self._h, int(n)),
               "nh_ensemble_run_graph")

    def state(self, k):
        sh, cs = self.shapes[k], self.cshapes[k]
        out = {q: np.zeros(sh) for q in ("h", "hu", "hv")}
        out["w"] = np.zeros(cs)
        out["p"] = np.zeros(cs)
        _check(lib().nh_ensemble_read_state(
            self._h, k, _ptr(out["h"]), _ptr(out["hu"]), _ptr(out["hv"]),
            _ptr(out["w"]), _ptr(out["p"])), "nh_ensemble_read_state")
        return out

    def stats(self, k) -> dict:
        s = NhStats()
        _check(lib().nh_ensemble_get_stats(self._h, k, C.byref(s)),
               "nh_ensemble_get_stats")
        return _stats_dict(s)

    def profile(self, on=True):
        """As Solver.profile, summed over the members."""
        _check(lib().nh_ensemble_profile(self._h, int(on)),
               "nh_ensemble_profile")

    def get_profile(self) -> dict:
        p = NhProfile()
        _check(lib().nh_ensemble_get_profile(self._h, C.byref(p)),
               "nh_ensemble_get_profile")
        return {k: getattr(p, k) for k, _ in NhProfile._fields_}


def run_noalloc(nx, ny, dx, dy, H, h, hu, hv, w, p, nsteps, *, stream=None,
                **params) -> dict:
    """nh_run_noalloc: nsteps steps of caller-owned device tensors in place,
    with no device allocation by the library (include/nhswe.h).  H, h, hu,
    hv (cells) and w (corners) in the precision's type (float64, or float32
    in FP32 bulk, where h holds s = h - max(H, 0)), p (corners) float64; hv may be
    None in 1D.  Returns the run's statistics."""
    import torch
    prec = params.get("precision", "f64")
    dtype = torch.float64 if prec == "f64" else torch.float32
    ncell = int(nx) * int(ny)
    ncorn = (int(nx) + 1) * (1 if int(ny) == 1 else int(ny) + 1)
    ptrs = []
    for name, t, n, dt in (("H", H, ncell, dtype), ("h", h, ncell, dtype),
                           ("hu", hu, ncell, dtype), ("hv", hv, ncell, dtype),
                           ("w", w, ncorn, dtype),
                           ("p", p, ncorn, torch.float64)):
        if t is None and name == "hv" and int(ny) == 1:
            ptrs.append(None)
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name}: a device tensor is required")
        if t.dtype != dt or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: a contiguous {dt} tensor of {n} "
                             "elements is required")
        ptrs.append(t.data_ptr())
    grid = NhGrid(int(nx), int(ny), float(dx), float(dy))
    par, _om = _params(**params)
    st = NhStats()
    _check(lib().nh_run_noalloc(C.byref(grid), C.byref(par),
                                C.c_void_p(stream) if stream else None,
                                *ptrs, int(nsteps), C.byref(st)),
           "nh_run_noalloc")
    return _stats_dict(st)
