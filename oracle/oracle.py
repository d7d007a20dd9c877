"""ctypes wrapper of the FP64 CPU oracle (oracle/nh_oracle.c).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module.  It does not import the GPU package and
the GPU package does not import it.

Arrays: cells are (ny, nx) float64 (1D mode: ny == 1, arrays (1, nx) or (nx,)),
corners are (ny+1, nx+1) in 2D and (nx+1,) in 1D.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_DP = C.POINTER(C.c_double)


class OraParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double),
        ("g", C.c_double), ("cfl", C.c_double),
        ("delta", C.c_double), ("dry_eps", C.c_double),
        ("nh_on", C.c_int32), ("breaking_on", C.c_int32),
        ("b1", C.c_double), ("b2", C.c_double),
        ("solve_max_iter", C.c_int32), ("check_every", C.c_int32),
        ("solve_tol", C.c_double),
        ("fixed_dt", C.c_int32), ("dt_fixed", C.c_double),
        ("manning", C.c_double), ("open_sides", C.c_int32),
        ("periodic", C.c_int32), ("w_advection", C.c_int32),
        ("solve_norm", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(os.path.dirname(LIB_PATH), "nh_oracle.c")
        if (not os.path.exists(LIB_PATH) or
                os.path.getmtime(LIB_PATH) < os.path.getmtime(src)):
            # missing or older than its source: compile it first
            from . import build_oracle
            build_oracle.build()
        _lib = C.CDLL(LIB_PATH)
        L = _lib
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [C.POINTER(OraParams), _DP, C.c_int32]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_set_bathymetry.argtypes = [C.c_void_p, _DP]
        L.ora_set_state.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP]
        L.ora_get_state.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP]
        L.ora_step.argtypes = [C.c_void_p]
        L.ora_set_relaxation.argtypes = [C.c_void_p] + [_DP] * 6
        L.ora_run.argtypes = [C.c_void_p, C.c_int64]
        L.ora_get_stats.argtypes = [C.c_void_p, _DP]
        L.ora_cfl_dt.restype = C.c_double
        L.ora_cfl_dt.argtypes = [C.c_void_p, _DP, _DP, _DP]
        L.ora_fv_stage.argtypes = [C.c_void_p, _DP, _DP, _DP, C.c_double,
                                   _DP, _DP, _DP, _DP]
        L.ora_breaking.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, C.c_double]
        L.ora_assemble.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, C.c_double,
                                   _DP, _DP, _DP, _DP, _DP, _DP]
        L.ora_constraint.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP,
                                     C.c_double, _DP]
        L.ora_solve.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP, _DP, _DP,
                                C.POINTER(C.c_int32), _DP]
        L.ora_dense_solve.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP,
                                      _DP, _DP]
        L.ora_correct.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP,
                                  C.c_double, _DP, _DP, _DP]
        L.ora_pvm_fluct.argtypes = [_DP, _DP, C.c_double, C.c_double, _DP, _DP]
        L.ora_desing_velocity.restype = C.c_double
        L.ora_desing_velocity.argtypes = [C.c_double, C.c_double, C.c_double]
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


@dataclass
class Params:
    """Parameters of the scheme (same meaning as the GPU library's)."""
    nx: int
    ny: int
    dx: float
    dy: float
    g: float = 9.81
    cfl: float = 0.9
    delta: float = 1e-5
    dry_eps: float = 1e-10
    nh_on: int = 1
    breaking_on: int = 0
    b1: float = 0.15
    b2: float = 0.5
    solve_max_iter: int = 200000
    check_every: int = 1
    solve_tol: float = 1e-12
    fixed_dt: int = 0
    dt_fixed: float = 0.0
    manning: float = 0.0
    open_sides: int = 0
    periodic: int = 0
    w_advection: int = 0
    solve_norm: int = 0
    omega: np.ndarray = field(default_factory=lambda: np.ones(1))

    def c_struct(self) -> OraParams:
        return OraParams(self.nx, self.ny, self.dx, self.dy, self.g, self.cfl,
                         self.delta, self.dry_eps, self.nh_on, self.breaking_on,
                         self.b1, self.b2, self.solve_max_iter,
                         self.check_every, self.solve_tol, self.fixed_dt,
                         self.dt_fixed, self.manning, self.open_sides,
                         self.periodic, self.w_advection, self.solve_norm)


class Oracle:
    """The FP64 CPU oracle: state, time stepping and component operators."""

    def __init__(self, params: Params):
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        self.is1d = params.ny == 1
        st = params.c_struct()
        self._omega = _f64(params.omega).ravel().copy()
        self._h = lib().ora_create(C.byref(st), _p(self._omega),
                                   len(self._omega))
        if not self._h:
            raise ValueError("oracle: invalid parameters")
        self.cshape = (params.nx + 1,) if self.is1d else (params.ny + 1,
                                                           params.nx + 1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_destroy(h)
            self._h = None

    # ---- shapes
    @property
    def shape(self):
        return (self.ny, self.nx)

    def _cells(self, a):
        return _f64(a, self.shape) if a is not None else None

    def _corn(self, a):
        return _f64(a, self.cshape) if a is not None else None

    # ---- state
    def set_bathymetry(self, H):
        self._H = self._cells(H)
        lib().ora_set_bathymetry(self._h, _p(self._H))

    def set_state(self, h, hu, hv=None, w=None, p=None):
        h, hu = self._cells(h), self._cells(hu)
        hv = self._cells(hv if hv is not None else np.zeros(self.shape))
        w, p = self._corn(w), self._corn(p)
        st = lib().ora_set_state(self._h, _p(h), _p(hu), _p(hv), _p(w), _p(p))
        if st != 0:
            raise ValueError(f"oracle set_state status {st}")

    def set_relaxation(self, widths, h=None, hu=None, hv=None, w=None,
                       p=None):
        """Generation/absorption zones (Section 4.4): widths = (west, east,
        south, north) in metres; targets default to still water."""
        wd = _f64(np.asarray(widths, dtype=np.float64).ravel(), (4,))
        self._relax = [wd] + [self._cells(a) for a in (h, hu, hv)] + \
            [self._corn(a) for a in (w, p)]
        st = lib().ora_set_relaxation(self._h, *[_p(a) for a in self._relax])
        if st != 0:
            raise ValueError(f"oracle set_relaxation status {st}")

    def step(self) -> int:
        return lib().ora_step(self._h)

    def run(self, n: int) -> int:
        return lib().ora_run(self._h, n)

    def state(self):
        out = {k: np.zeros(self.shape) for k in ("h", "hu", "hv")}
        out["w"] = np.zeros(self.cshape)
        out["p"] = np.zeros(self.cshape)
        lib().ora_get_state(self._h, _p(out["h"]), _p(out["hu"]),
                            _p(out["hv"]), _p(out["w"]), _p(out["p"]))
        return out

    def stats(self):
        s = np.zeros(12)
        lib().ora_get_stats(self._h, _p(s))
        return dict(t=s[0], dt=s[1], step=int(s[2]), sweeps1=int(s[3]),
                    sweeps2=int(s[4]), measure=s[5], clamped=s[6],
                    sweeps_total=int(s[7]), solves=int(s[8]), dt_last=s[9],
                    status=int(s[10]), nondominant=int(s[11]))

    # ---- components
    def cfl_dt(self, h, hu, hv=None):
        h, hu = self._cells(h), self._cells(hu)
        hv = self._cells(hv if hv is not None else np.zeros(self.shape))
        return lib().ora_cfl_dt(self._h, _p(h), _p(hu), _p(hv))

    def fv_stage(self, h, hu, hv, dt):
        h, hu = self._cells(h), self._cells(hu)
        hv = self._cells(hv if hv is not None else np.zeros(self.shape))
        oh, o1, o2 = (np.zeros(self.shape) for _ in range(3))
        cl = C.c_double(0.0)
        lib().ora_fv_stage(self._h, _p(h), _p(hu), _p(hv), dt, _p(oh),
                           _p(o1), _p(o2), C.byref(cl))
        return oh, o1, o2, cl.value

    def breaking(self, h, hu, hv, w, dt):
        h = self._cells(h)
        hu = self._cells(hu).copy()
        hv = self._cells(hv if hv is not None else np.zeros(self.shape)).copy()
        w = self._corn(w).copy()
        lib().ora_breaking(self._h, _p(h), _p(hu), _p(hv), _p(w), dt)
        return hu, hv, w

    def assemble(self, h, hu, hv, w, dt):
        h, hu = self._cells(h), self._cells(hu)
        hv = self._cells(hv if hv is not None else np.zeros(self.shape))
        w = self._corn(w)
        outs = [np.zeros(self.cshape) for _ in range(6)]
        lib().ora_assemble(self._h, _p(h), _p(hu), _p(hv), _p(w), dt,
                           *[_p(a) for a in outs])
        return dict(zip(("diag", "cE", "cW", "cN", "cS", "rhs"), outs))

    def constraint(self, h, hu, hv, w, p, dt):
        h, hu = self._cells(h), self._cells(hu)
        hv = self._cells(hv if hv is not None else np.zeros(self.shape))
        w, p = self._corn(w), self._corn(p)
        out = np.zeros(self.cshape)
        lib().ora_constraint(self._h, _p(h), _p(hu), _p(hv), _p(w), _p(p), dt,
                             _p(out))
        return out

    def solve(self, coef, p0=None):
        p = np.zeros(self.cshape) if p0 is None else self._corn(p0).copy()
        sw = C.c_int32(0)
        meas = C.c_double(0.0)
        args = [self._corn(coef[k]) for k in ("diag", "cE", "cW", "cN", "cS",
                                               "rhs")]
        st = lib().ora_solve(self._h, *[_p(a) for a in args], _p(p),
                             C.byref(sw), C.byref(meas))
        return p, st, sw.value, meas.value

    def dense_solve(self, coef):
        p = np.zeros(self.cshape)
        args = [self._corn(coef[k]) for k in ("diag", "cE", "cW", "cN", "cS",
                                               "rhs")]
        st = lib().ora_dense_solve(self._h, *[_p(a) for a in args], _p(p))
        if st != 0:
            raise RuntimeError(f"dense solve status {st}")
        return p

    def correct(self, h, hu, hv, w, p, dt):
        h, hu = self._cells(h), self._cells(hu)
        hv = self._cells(hv if hv is not None else np.zeros(self.shape))
        w, p = self._corn(w), self._corn(p)
        o1, o2 = np.zeros(self.shape), np.zeros(self.shape)
        ow = np.zeros(self.cshape)
        lib().ora_correct(self._h, _p(h), _p(hu), _p(hv), _p(w), _p(p), dt,
                          _p(o1), _p(o2), _p(ow))
        return o1, o2, ow


def pvm_fluct(left, right, g=9.81, dry_eps=1e-10):
    """Edge fluctuation D-, D+ of eq. (18); left/right = (h, qn, qt, un, ut,
    eta, H)."""
    L = _f64(left).ravel()
    R = _f64(right).ravel()
    Dm, Dp = np.zeros(3), np.zeros(3)
    lib().ora_pvm_fluct(_p(L), _p(R), g, dry_eps, _p(Dm), _p(Dp))
    return Dm, Dp


def desing_velocity(h, q, delta=1e-5):
    return lib().ora_desing_velocity(h, q, delta)
