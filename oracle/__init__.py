"""FP64 CPU oracle for the Euler-step hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may use it; the product path never does.  It shares no
code with the HIP path.

`euler_oracle.c` holds the arithmetic (plain serial FP64 loops);
this module is a ctypes wrapper over numpy arrays.  State arrays are numpy
float64 arrays of shape (d+2, *reversed(n)) — i.e. (d+2, nz, ny, nx) in 3D,
x fastest — holding rho, m_0..m_{d-1}, E.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "euler_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_COUNT_SRC = os.path.join(_HERE, "flopcount.cpp")
_COUNT_PATH = os.path.join(_HERE, "liboracle_count.so")

PERIODIC = 0
OUTFLOW = 1
ANALYTIC = 2

# problems of the convergence tests (analytic boundaries)
ENTROPY_WAVE = 1
SOUND_WAVE = 2
SHOCK_TUBE = 3

OK = 0
BAD_ARG = -1
NONFINITE = -4


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math) and its operation counter."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    if force or not os.path.exists(_OMP_PATH):
        # the same source with its loops over cells run by OpenMP (bitwise the serial results)
        tmp = _OMP_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OMP_PATH)
    if force or not os.path.exists(_COUNT_PATH):
        tmp = _COUNT_PATH + ".tmp"
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-fpermissive", "-w",
                               "-ffp-contract=off", "-o", tmp, _COUNT_SRC])
        os.replace(tmp, _COUNT_PATH)
    return _LIB_PATH


class _Mesh(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("order", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double * 3),
                ("gamma", ctypes.c_double), ("bc", ctypes.c_int32 * 3),
                ("pad2_", ctypes.c_int32)]


class _Analytic(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("angle", ctypes.c_double), ("amplitude", ctypes.c_double)]


@dataclass
class Analytic:
    """A convergence-test problem on the unit square: kind, rotation angle of
    the initial condition about the centre (radians), sound-wave amplitude."""
    kind: int
    angle: float = 0.0
    amplitude: float = 1e-5

    def c(self) -> _Analytic:
        a = _Analytic()
        a.kind, a.angle, a.amplitude = int(self.kind), float(self.angle), float(self.amplitude)
        return a


_libs = {}
_parallel = False


def use_openmp(on: bool = True) -> None:
    """Route the calls below to the OpenMP build (all host cores; results are
    bitwise those of the serial build) or back to the serial one."""
    global _parallel
    _parallel = bool(on)


def num_threads() -> int:
    """Threads the current build's loops use (1 for the serial build)."""
    return int(_load().orc_num_threads())


def _load():
    key = "omp" if _parallel else "serial"
    if key not in _libs:
        path = _OMP_PATH if _parallel else _LIB_PATH
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        mp = ctypes.POINTER(_Mesh)
        lib.orc_stage.argtypes = [mp, dp, dp, ctypes.c_double, dp]
        lib.orc_step.argtypes = [mp, dp, ctypes.c_double, dp]
        lib.orc_cfl_qmax.argtypes = [mp, dp, dp]
        lib.orc_cfl_dt.argtypes = [mp, dp, ctypes.c_double, dp]
        lib.orc_totals.argtypes = [mp, dp, dp]
        lib.orc_advance.argtypes = [mp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                    dp, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_hllc.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        lib.orc_minmod.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_minmod.restype = ctypes.c_double
        lib.orc_interpolate.argtypes = [ctypes.c_double] * 3 + [dp, dp]
        lib.orc_prim_of_cons.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.orc_cons_of_prim.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        ap = ctypes.POINTER(_Analytic)
        lib.orc_stage_t.argtypes = [mp, ap, ctypes.c_double, dp, dp, ctypes.c_double, dp]
        lib.orc_step_t.argtypes = [mp, ap, ctypes.c_double, dp, ctypes.c_double, dp]
        lib.orc_advance_t.argtypes = [mp, ap, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                      dp, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_exact_prims.argtypes = [mp, ap, dp, ctypes.c_double, dp]
        lib.orc_exact_state.argtypes = [mp, ap, ctypes.c_double, dp]
        lib.orc_riemann_star.argtypes = [ctypes.c_double, dp, dp, dp, dp]
        lib.orc_riemann_sample.argtypes = [ctypes.c_double, dp, dp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, dp]
        lib.orc_riemann_sample.restype = None
        for fn in ("orc_stage", "orc_step", "orc_cfl_qmax", "orc_cfl_dt", "orc_totals",
                   "orc_advance", "orc_stage_t", "orc_step_t", "orc_advance_t", "orc_exact_prims", "orc_exact_state",
                   "orc_riemann_star"):
            getattr(lib, fn).restype = ctypes.c_int
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = ctypes.c_int
        _libs[key] = lib
    return _libs[key]


@dataclass
class Mesh:
    """Uniform mesh on [0,1]^d (or the given spacings), n = (nx, ny, nz)."""
    ndim: int
    n: tuple
    gamma: float
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    dx: tuple | None = None
    order: int = 2      # reconstruction: 2 minbee piecewise linear, 1 piecewise constant
    _c: _Mesh = field(init=False, repr=False)

    def __post_init__(self):
        n = tuple(int(v) for v in self.n) + (1,) * (3 - len(self.n))
        self.n = n
        if self.dx is None:
            self.dx = tuple(1.0 / n[a] if a < self.ndim else 1.0 for a in range(3))
        else:
            self.dx = tuple(float(v) for v in self.dx) + (1.0,) * (3 - len(self.dx))
        bc = tuple(int(b) for b in self.bc) + (PERIODIC,) * (3 - len(self.bc))
        self.bc = bc
        c = _Mesh()
        c.ndim = self.ndim
        c.order = int(self.order)
        for a in range(3):
            c.n[a] = n[a]
            c.dx[a] = self.dx[a]
            c.bc[a] = bc[a]
        c.gamma = float(self.gamma)
        self._c = c

    @property
    def nf(self) -> int:
        return self.ndim + 2

    @property
    def shape(self) -> tuple:
        return (self.nf,) + tuple(reversed(self.n[: self.ndim]))

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_state(mesh: Mesh, U) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.size != mesh.nf * mesh.ncells:
        raise OracleError(f"state has {U.size} values, mesh needs {mesh.nf * mesh.ncells}")
    return U.reshape(mesh.shape)


def _check(rc: int, what: str):
    if rc == NONFINITE:
        raise FloatingPointError(f"{what}: non-physical or non-finite state")
    if rc != OK:
        raise OracleError(f"{what}: status {rc}")


def _an(analytic):
    return ctypes.byref(analytic.c()) if analytic is not None else None


def stage(mesh: Mesh, U_in, U_base, cdt: float, t: float = 0.0, analytic: Analytic | None = None) -> np.ndarray:
    """One stage; t (the time U_in stands for) only matters for analytic boundaries."""
    lib = _load()
    a, b = _as_state(mesh, U_in), _as_state(mesh, U_base)
    out = np.empty_like(a)
    _check(lib.orc_stage_t(ctypes.byref(mesh._c), _an(analytic), float(t), _ptr(a), _ptr(b), float(cdt),
                           _ptr(out)), "stage")
    return out


def step(mesh: Mesh, U0, dt: float, t: float = 0.0, analytic: Analytic | None = None) -> np.ndarray:
    """One midpoint-RK2 step with the given dt (FP64) from time t."""
    lib = _load()
    a = _as_state(mesh, U0)
    out = np.empty_like(a)
    _check(lib.orc_step_t(ctypes.byref(mesh._c), _an(analytic), float(t), _ptr(a), float(dt), _ptr(out)),
           "step")
    return out


def cfl_qmax(mesh: Mesh, U) -> float:
    lib = _load()
    a = _as_state(mesh, U)
    q = ctypes.c_double()
    _check(lib.orc_cfl_qmax(ctypes.byref(mesh._c), _ptr(a), ctypes.byref(q)), "cfl")
    return q.value


def cfl_dt(mesh: Mesh, U, cfl: float) -> float:
    lib = _load()
    a = _as_state(mesh, U)
    dt = ctypes.c_double()
    _check(lib.orc_cfl_dt(ctypes.byref(mesh._c), _ptr(a), float(cfl), ctypes.byref(dt)), "cfl")
    return dt.value


def totals(mesh: Mesh, U) -> np.ndarray:
    lib = _load()
    a = _as_state(mesh, U)
    out = np.zeros(mesh.nf)
    _check(lib.orc_totals(ctypes.byref(mesh._c), _ptr(a), _ptr(out)), "totals")
    return out


def advance(mesh: Mesh, U0, cfl: float, t_end: float, max_steps: int = 1 << 40, t0: float = 0.0,
            analytic: Analytic | None = None, on_failure: str = "raise"):
    """Advance a copy of U0 to t_end; returns (U, t, steps).  When the state
    turns non-physical the advance stops after the step that produced it;
    on_failure="raise" raises FloatingPointError, on_failure="return" returns
    (U, t, steps, False) holding that step's output, time and count (and
    (U, t, steps, True) on success)."""
    lib = _load()
    U = _as_state(mesh, U0).copy()
    t = ctypes.c_double(t0)
    steps = ctypes.c_int64()
    rc = lib.orc_advance_t(ctypes.byref(mesh._c), _an(analytic), _ptr(U), float(cfl), float(t_end),
                           int(max_steps), ctypes.byref(t), ctypes.byref(steps))
    if on_failure == "return" and rc in (OK, NONFINITE):
        return U, t.value, steps.value, rc == OK
    _check(rc, "advance")
    return U, t.value, steps.value


# ---- exact solutions of the convergence-test problems ---------------------------------

def exact_prims(mesh: Mesh, analytic: Analytic, x, t: float) -> np.ndarray:
    """Primitive state (rho, v_a, p) of the problem at point x and time t."""
    x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    v = np.zeros(mesh.nf)
    _check(_load().orc_exact_prims(ctypes.byref(mesh._c), ctypes.byref(analytic.c()), _ptr(x), float(t),
                                   _ptr(v)), "exact")
    return v


def exact_state(mesh: Mesh, analytic: Analytic, t: float) -> np.ndarray:
    """Conserved state of the problem at every cell centre, in the oracle's layout."""
    U = np.zeros(mesh.shape)
    _check(_load().orc_exact_state(ctypes.byref(mesh._c), ctypes.byref(analytic.c()), float(t), _ptr(U)),
           "exact")
    return U


def riemann_star(gamma: float, left, right) -> tuple[float, float]:
    """(p*, u*) of the exact Riemann problem; states are (rho, u, p)."""
    L = np.ascontiguousarray(left, dtype=np.float64)
    R = np.ascontiguousarray(right, dtype=np.float64)
    ps, us = ctypes.c_double(), ctypes.c_double()
    _check(_load().orc_riemann_star(float(gamma), _ptr(L), _ptr(R), ctypes.byref(ps), ctypes.byref(us)),
           "riemann")
    return ps.value, us.value


def riemann_sample(gamma: float, left, right, xi: float) -> np.ndarray:
    L = np.ascontiguousarray(left, dtype=np.float64)
    R = np.ascontiguousarray(right, dtype=np.float64)
    ps, us = riemann_star(gamma, L, R)
    out = np.zeros(3)
    _load().orc_riemann_sample(float(gamma), _ptr(L), _ptr(R), ps, us, float(xi), _ptr(out))
    return out


# ---- single-cell pieces, exposed for the unit pins -----------------------------------

def minmod(a: float, b: float) -> float:
    return _load().orc_minmod(float(a), float(b))


def interpolate(y0: float, y1: float, y2: float) -> tuple[float, float]:
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _load().orc_interpolate(float(y0), float(y1), float(y2), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def hllc(ndim: int, gamma: float, axis: int, vl, vr) -> np.ndarray:
    lib = _load()
    vl = np.ascontiguousarray(vl, dtype=np.float64)
    vr = np.ascontiguousarray(vr, dtype=np.float64)
    f = np.zeros(ndim + 2)
    lib.orc_hllc(int(ndim), float(gamma), int(axis), _ptr(vl), _ptr(vr), _ptr(f))
    return f


def prim_of_cons(ndim: int, gamma: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.zeros(ndim + 2)
    _load().orc_prim_of_cons(int(ndim), float(gamma), _ptr(u), _ptr(v))
    return v


def cons_of_prim(ndim: int, gamma: float, v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    u = np.zeros(ndim + 2)
    _load().orc_cons_of_prim(int(ndim), float(gamma), _ptr(v), _ptr(u))
    return u


# ---- operation counts of the method (defines algorithmic work per cell-update) --------

_count_lib = None


def _load_count():
    global _count_lib
    if _count_lib is None:
        if not os.path.exists(_COUNT_PATH) or os.path.getmtime(_COUNT_PATH) < max(
                os.path.getmtime(_COUNT_SRC), os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(_COUNT_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        mp = ctypes.POINTER(_Mesh)
        lp = ctypes.POINTER(ctypes.c_longlong)
        lib.orc_count_step.argtypes = [mp, dp, ctypes.c_double, dp, lp]
        lib.orc_count_cfl.argtypes = [mp, dp, ctypes.c_double, dp, lp]
        lib.orc_count_step.restype = ctypes.c_int
        lib.orc_count_cfl.restype = ctypes.c_int
        _count_lib = lib
    return _count_lib


def count_ops(mesh: Mesh, U, dt: float, cfl: float = 0.5) -> dict:
    """Floating-point operations of one step plus its CFL reduction, per cell-update:
    add (incl. subtract), mul, div, sqrt, cmp (compare, min, max, abs)."""
    lib = _load_count()
    a = _as_state(mesh, U)
    out = np.empty_like(a)
    c1 = (ctypes.c_longlong * 5)()
    c2 = (ctypes.c_longlong * 5)()
    _check(lib.orc_count_step(ctypes.byref(mesh._c), _ptr(a), float(dt), _ptr(out), c1), "count step")
    d = ctypes.c_double()
    _check(lib.orc_count_cfl(ctypes.byref(mesh._c), _ptr(a), float(cfl), ctypes.byref(d), c2), "count cfl")
    names = ("add", "mul", "div", "sqrt", "cmp")
    n = float(mesh.ncells)
    return {k: (c1[i] + c2[i]) / n for i, k in enumerate(names)}
