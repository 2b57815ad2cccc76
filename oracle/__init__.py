"""FP64 CPU oracle for the direct N-body hot path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never calls
it.  The arithmetic lives in ``nbody_oracle.c`` (plain C, binary64); this
module only marshals numpy arrays through ctypes.

Every vector field is a float64 array of shape (3, n); times are int64 ticks
of 2^-20 time units.  Functions and the passages they follow:

* :func:`force` -- Eq. 1 (Section 2) with Plummer softening (Section 3.3),
  jerk and potential (Section 3), self removed by index (Section 3.1).
* :func:`force_vjp` -- the adjoint of :func:`force` (derived from it).
* :func:`predict`, :func:`correct`, :func:`aarseth_dt`, :func:`quantise_dt`,
  :func:`select_active`, :func:`hermite_run` -- the fourth-order Hermite
  scheme with block time steps (Section 3 and 3.1).
* :func:`force_acc` -- the force-only evaluation (acceleration and
  potential, no jerk) that Section 4 uses for its treecode runs.
* :func:`nearest` -- the nearest neighbour of each i (Section 3.3).
* :func:`leapfrog` -- a kick-drift-kick run on :func:`force_acc`.
* :func:`energy` -- Eq. 2 (Section 4) energy bookkeeping.
* :func:`hermite_shared_forward`, :func:`hermite_shared_adjoint` -- shared
  step runs and their gradient with respect to x0, v0, m.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TICKS_PER_UNIT = 1 << 20


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over i)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("eta", C.c_double),
                ("eta_s", C.c_double), ("lmin", C.c_int), ("lmax", C.c_int),
                ("shared_log2", C.c_int)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = C.CDLL(build())
            P = C.c_void_p
            I64, D, I = C.c_int64, C.c_double, C.c_int
            lib.oracle_force.argtypes = [I64, P, P, P, I64, P, P, P, D, D, P, P, P, I]
            lib.oracle_force.restype = I
            lib.oracle_force_vjp.argtypes = [I64, P, P, P, I64, P, P, P, D, D, P, P, P,
                                             P, P, P, P, P, I]
            lib.oracle_force_vjp.restype = I
            lib.oracle_predict_one.argtypes = [P, P, P, P, D, P, P]
            lib.oracle_predict_one.restype = None
            lib.oracle_correct_one.argtypes = [P, P, P, P, P, P, D, P, P, P, P]
            lib.oracle_correct_one.restype = None
            lib.oracle_aarseth_dt.argtypes = [P, P, P, P, D, D]
            lib.oracle_aarseth_dt.restype = D
            lib.oracle_quantise_dt.argtypes = [D, I64, I64, I, I]
            lib.oracle_quantise_dt.restype = I64
            lib.oracle_select_active.argtypes = [I64, P, P, P, P]
            lib.oracle_select_active.restype = I64
            lib.oracle_hermite_run.argtypes = [I64, P, P, P, P, P, P, P, C.POINTER(_Opts), I,
                                               I64, I64, P, I]
            lib.oracle_hermite_run.restype = I64
            lib.oracle_energy.argtypes = [I64, P, P, P, D, D, P, P, I]
            lib.oracle_energy.restype = I
            lib.oracle_hermite_shared_forward.argtypes = [I64, P, P, P, D, D, D, I64, P, P, I]
            lib.oracle_hermite_shared_forward.restype = I
            lib.oracle_hermite_shared_adjoint.argtypes = [I64, P, P, P, D, D, D, I64, P, P,
                                                          P, P, P, I]
            lib.oracle_hermite_shared_adjoint.restype = I
            lib.oracle_nearest.argtypes = [I64, P, P, I64, P, P, P, I]
            lib.oracle_nearest.restype = I
            lib.oracle_leapfrog.argtypes = [I64, P, P, P, D, D, D, I64, P, P, I, I]
            lib.oracle_leapfrog.restype = I
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = I
            _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return _load().oracle_num_threads()


def force(xi, vi, xj, vj, mj, eps, G=1.0, iself=None, nthreads=0):
    """Acceleration, jerk, potential of i from j.  Returns (acc, jerk, pot)
    with shapes (3, ni), (3, ni), (ni,).  ``iself[i]`` is the j index of i
    (excluded), or -1; None excludes nothing."""
    lib = _load()
    xi = _f64(xi); ni = xi.shape[1]
    vi = _f64(vi, (3, ni))
    xj = _f64(xj); nj = xj.shape[1]
    vj = _f64(vj, (3, nj)); mj = _f64(mj, (nj,))
    s = None if iself is None else np.ascontiguousarray(iself, dtype=np.int64)
    acc = np.empty((3, ni)); jerk = np.empty((3, ni)); pot = np.empty(ni)
    rc = lib.oracle_force(ni, _p(xi), _p(vi), _p(s), nj, _p(xj), _p(vj), _p(mj),
                          float(G), float(eps), _p(acc), _p(jerk), _p(pot), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_force: bad arguments")
    return acc, jerk, pot


def force_vjp(xi, vi, xj, vj, mj, eps, ga, gj=None, gp=None, G=1.0, iself=None,
              nthreads=0):
    """Cotangents (gxi, gvi, gxj, gvj, gmj) for output cotangents (ga, gj, gp)."""
    lib = _load()
    xi = _f64(xi); ni = xi.shape[1]
    vi = _f64(vi, (3, ni))
    xj = _f64(xj); nj = xj.shape[1]
    vj = _f64(vj, (3, nj)); mj = _f64(mj, (nj,))
    ga = _f64(ga, (3, ni))
    gj = None if gj is None else _f64(gj, (3, ni))
    gp = None if gp is None else _f64(gp, (ni,))
    s = None if iself is None else np.ascontiguousarray(iself, dtype=np.int64)
    gxi = np.empty((3, ni)); gvi = np.empty((3, ni))
    gxj = np.empty((3, nj)); gvj = np.empty((3, nj)); gmj = np.empty(nj)
    rc = lib.oracle_force_vjp(ni, _p(xi), _p(vi), _p(s), nj, _p(xj), _p(vj), _p(mj),
                              float(G), float(eps), _p(ga), _p(gj), _p(gp),
                              _p(gxi), _p(gvi), _p(gxj), _p(gvj), _p(gmj), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_force_vjp: bad arguments")
    return gxi, gvi, gxj, gvj, gmj


def predict(x, v, a, j, D):
    """Hermite predictor of one particle (3-vectors) over D time units."""
    lib = _load()
    x, v, a, j = (_f64(q, (3,)) for q in (x, v, a, j))
    xp = np.empty(3); vp = np.empty(3)
    lib.oracle_predict_one(_p(x), _p(v), _p(a), _p(j), float(D), _p(xp), _p(vp))
    return xp, vp


def correct(xp, vp, a0, j0, a1, j1, D):
    """Hermite corrector of one particle: returns (x1, v1, a2, a3)."""
    lib = _load()
    xp, vp, a0, j0, a1, j1 = (_f64(q, (3,)) for q in (xp, vp, a0, j0, a1, j1))
    x1 = np.empty(3); v1 = np.empty(3); a2 = np.empty(3); a3 = np.empty(3)
    lib.oracle_correct_one(_p(xp), _p(vp), _p(a0), _p(j0), _p(a1), _p(j1), float(D),
                           _p(x1), _p(v1), _p(a2), _p(a3))
    return x1, v1, a2, a3


def aarseth_dt(a1, j1, a2, a3, D, eta):
    lib = _load()
    a1, j1, a2, a3 = (_f64(q, (3,)) for q in (a1, j1, a2, a3))
    return lib.oracle_aarseth_dt(_p(a1), _p(j1), _p(a2), _p(a3), float(D), float(eta))


def quantise_dt(crit, dt_old, t_new, lmin=-20, lmax=-3):
    return _load().oracle_quantise_dt(float(crit), int(dt_old), int(t_new), int(lmin), int(lmax))


def select_active(t, dt):
    """(indices int32, t_next) of the next block."""
    lib = _load()
    t = np.ascontiguousarray(t, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.int64)
    n = t.shape[0]
    idx = np.empty(max(n, 1), dtype=np.int32)
    tn = C.c_int64(0)
    c = lib.oracle_select_active(n, _p(t), _p(dt), _p(idx), C.byref(tn))
    return idx[:c].copy(), int(tn.value)


class HermiteState:
    """Particle state for :func:`hermite_run` (arrays are updated in place)."""

    def __init__(self, pos, vel, mass):
        self.x = _f64(pos).copy()
        n = self.x.shape[1]
        self.v = _f64(vel, (3, n)).copy()
        self.m = _f64(mass, (n,)).copy()
        self.a = np.zeros((3, n)); self.j = np.zeros((3, n))
        self.t = np.zeros(n, dtype=np.int64); self.dt = np.zeros(n, dtype=np.int64)
        self.steps = 0
        self.sum_active = 0

    @property
    def n(self):
        return self.m.shape[0]


def hermite_run(state: HermiteState, t_end_ticks, *, G=1.0, eps=0.0, eta=0.02, eta_s=0.01,
                lmin=-20, lmax=-3, shared_log2=0, init=False, max_steps=1 << 62,
                nthreads=0):
    """Advance ``state`` by block (or shared) Hermite steps to t_end (ticks).
    Returns the number of block steps taken in this call."""
    lib = _load()
    o = _Opts(float(G), float(eps), float(eta), float(eta_s), int(lmin), int(lmax),
              int(shared_log2))
    sa = C.c_int64(0)
    st = lib.oracle_hermite_run(state.n, _p(state.x), _p(state.v), _p(state.a), _p(state.j),
                                _p(state.m), _p(state.t), _p(state.dt), C.byref(o),
                                1 if init else 0, int(t_end_ticks), int(max_steps),
                                C.byref(sa), int(nthreads))
    if st < 0:
        raise MemoryError("oracle_hermite_run: allocation failed")
    state.steps += st
    state.sum_active += sa.value
    return st


def energy(x, v, m, eps, G=1.0, nthreads=0):
    """(E_kin, E_pot) with the softened, self-excluded potential."""
    lib = _load()
    x = _f64(x); n = x.shape[1]
    v = _f64(v, (3, n)); m = _f64(m, (n,))
    ek = C.c_double(0); ep = C.c_double(0)
    rc = lib.oracle_energy(n, _p(x), _p(v), _p(m), float(G), float(eps), C.byref(ek),
                           C.byref(ep), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_energy")
    return ek.value, ep.value


def hermite_shared_forward(x0, v0, m, eps, D, nsteps, G=1.0, nthreads=0):
    """Shared-step Hermite run from (x0, v0); returns (x, v) at the end."""
    lib = _load()
    x = _f64(x0).copy(); n = x.shape[1]
    v = _f64(v0, (3, n)).copy(); m = _f64(m, (n,))
    rc = lib.oracle_hermite_shared_forward(n, _p(x), _p(v), _p(m), float(G), float(eps),
                                           float(D), int(nsteps), None, None, int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_hermite_shared_forward")
    return x, v


def hermite_shared_adjoint(x0, v0, m, eps, D, nsteps, gx_end, gv_end=None, G=1.0,
                           nthreads=0):
    """Gradient of L = <gx_end, x(T)> + <gv_end, v(T)> w.r.t. (x0, v0, m)."""
    lib = _load()
    x0 = _f64(x0); n = x0.shape[1]
    v0 = _f64(v0, (3, n)); m = _f64(m, (n,))
    gx_end = _f64(gx_end, (3, n))
    gv_end = None if gv_end is None else _f64(gv_end, (3, n))
    gx0 = np.empty((3, n)); gv0 = np.empty((3, n)); gm = np.empty(n)
    rc = lib.oracle_hermite_shared_adjoint(n, _p(x0), _p(v0), _p(m), float(G), float(eps),
                                           float(D), int(nsteps), _p(gx_end), _p(gv_end),
                                           _p(gx0), _p(gv0), _p(gm), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_hermite_shared_adjoint")
    return gx0, gv0, gm


def force_acc(xi, xj, mj, eps, G=1.0, iself=None, nthreads=0):
    """Acceleration and potential only (the force-only evaluation).  The
    jerk needs velocities; these two do not, so zero velocities are passed
    and the jerk is dropped.  Returns (acc (3, ni), pot (ni,))."""
    xi = _f64(xi)
    xj = _f64(xj)
    acc, _, pot = force(xi, np.zeros_like(xi), xj, np.zeros_like(xj), mj, eps, G=G, iself=iself,
                        nthreads=nthreads)
    return acc, pot


def nearest(xi, xj, iself=None, nthreads=0):
    """Nearest j of every i by unsoftened distance, self excluded by index,
    lowest j on ties.  Returns (nn int64 (ni,), r2 (ni,)); -1 / +inf when
    there is no candidate."""
    lib = _load()
    xi = _f64(xi); ni = xi.shape[1]
    xj = _f64(xj); nj = xj.shape[1]
    s = None if iself is None else np.ascontiguousarray(iself, dtype=np.int64)
    nn = np.empty(ni, dtype=np.int64); r2 = np.empty(ni)
    rc = lib.oracle_nearest(ni, _p(xi), _p(s), nj, _p(xj), _p(nn), _p(r2), nthreads)
    if rc:
        raise ValueError(f"oracle_nearest failed ({rc})")
    return nn, r2


def leapfrog(x0, v0, m, eps, dt, nsteps, G=1.0, acc=None, nthreads=0):
    """Kick-drift-kick run of ``nsteps`` steps of ``dt``; ``acc`` is a(x0)
    if known.  Returns (x, v, acc, pot) at the end."""
    lib = _load()
    x = _f64(x0).copy(); n = x.shape[1]
    v = _f64(v0, (3, n)).copy(); m = _f64(m, (n,))
    have = acc is not None
    a = _f64(acc, (3, n)).copy() if have else np.zeros((3, n))
    pot = np.empty(n)
    rc = lib.oracle_leapfrog(n, _p(x), _p(v), _p(m), float(G), float(eps), float(dt), int(nsteps),
                             _p(a), _p(pot), 1 if have else 0, nthreads)
    if rc:
        raise ValueError(f"oracle_leapfrog failed ({rc})")
    return x, v, a, pot
