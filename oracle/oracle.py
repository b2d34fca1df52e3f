"""ctypes binding of the C++ oracle (``chem_oracle.cpp``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Functions take the
mechanism dictionary of ``paper_2105_12070_amd.inputs`` and numpy arrays; the
pressure is in Pa.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chem_oracle.cpp")
_LIB = os.path.join(_HERE, "libchem_oracle.so")

STATUS = {0: "OK", 1: "TOO_MANY_STEPS", 2: "STEP_UNDERFLOW", 3: "SINGULAR", 4: "NONFINITE"}
METHOD = {"ros4": 0, "rodas3": 1, "euler": 2, "seulex": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with g++: -O3 for x86-64-v3 (AVX2 + FMA, every EPYC
    and recent Xeon), OpenMP, no fast-math and no floating-point contraction,
    so that every operation rounds as written in the source."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-std=c++17", "-fopenmp", "-fPIC",
               "-shared", "-fno-fast-math", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Mech(C.Structure):
    _fields_ = [("K", C.c_int32), ("R", C.c_int32),
                ("W", C.c_void_p), ("nasa7", C.c_void_p), ("rtype", C.c_void_p),
                ("reac", C.c_void_p), ("prod", C.c_void_p), ("lnA", C.c_void_p),
                ("b", C.c_void_p), ("theta", C.c_void_p), ("eff", C.c_void_p),
                ("troe", C.c_void_p), ("low", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("max_steps", C.c_int32), ("fac_safe", C.c_double),
                ("fac_min", C.c_double), ("fac_max", C.c_double), ("h_min", C.c_double),
                ("jac_mode", C.c_int32), ("lu_pivot", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = C.CDLL(_LIB)
        _lib.oracle_gas_constant.restype = C.c_double
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


class Mech:
    """Keeps contiguous copies of the mechanism arrays alive for the C struct."""

    def __init__(self, mech: dict, lnA=None, b=None, theta=None):
        self.K = int(mech["n_species"])
        self.R = int(mech["n_reactions"])
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self.arrs = dict(W=f64(mech["W"]), nasa7=f64(mech["nasa7"]), rtype=i32(mech["rtype"]),
                         reac=i32(mech["reac"]), prod=i32(mech["prod"]),
                         lnA=f64(mech["lnA"] if lnA is None else lnA),
                         b=f64(mech["b"] if b is None else b),
                         theta=f64(mech["theta"] if theta is None else theta),
                         eff=f64(mech["eff"]), troe=f64(mech["troe"]), low=f64(mech["low"]))
        a = self.arrs
        self.s = _Mech(self.K, self.R, *(a[k].ctypes.data for k in
                                         ("W", "nasa7", "rtype", "reac", "prod", "lnA", "b", "theta",
                                          "eff", "troe", "low")))

    @property
    def N(self):
        return self.K + 1


def _as_mech(m):
    return m if isinstance(m, Mech) else Mech(m)


def opts(method="ros4", max_steps=100000, fac_safe=0.9, fac_min=0.2, fac_max=6.0, h_min=1e-20, jac_mode=0,
         lu_pivot=0):
    """jac_mode 0 analytic / 1 finite differences; lu_pivot 0 partial pivoting / 1 none."""
    return _Opts(METHOD.get(method, method), max_steps, fac_safe, fac_min, fac_max, h_min, jac_mode, lu_pivot)


def gas_constant():
    return lib().oracle_gas_constant()


def rhs(mech, p, y):
    m = _as_mech(mech)
    y = np.ascontiguousarray(y, np.float64)
    f = np.zeros(m.N)
    lib().oracle_rhs(C.byref(m.s), C.c_double(p), _p(y), _p(f))
    return f


def jac(mech, p, y, mode="analytic"):
    m = _as_mech(mech)
    y = np.ascontiguousarray(y, np.float64)
    J = np.zeros((m.N, m.N))
    lib().oracle_jac(C.byref(m.s), C.c_double(p), _p(y), _p(J), {"analytic": 0, "ad": 1, "fd": 2}[mode])
    return J


def rates(mech, p, y):
    m = _as_mech(mech)
    y = np.ascontiguousarray(y, np.float64)
    q, k, Kc = np.zeros(m.R), np.zeros(m.R), np.zeros(m.R)
    lib().oracle_rates(C.byref(m.s), C.c_double(p), _p(y), _p(q), _p(k), _p(Kc))
    return q, k, Kc


def thermo(mech, T):
    m = _as_mech(mech)
    cpR, hRT, sR = np.zeros(m.K), np.zeros(m.K), np.zeros(m.K)
    lib().oracle_thermo(C.byref(m.s), C.c_double(T), _p(cpR), _p(hRT), _p(sR))
    return cpR, hRT, sR


def lu_factor(A, pivot=True):
    A = np.array(A, dtype=np.float64, order="C")
    n = A.shape[0]
    piv = np.zeros(n, np.int32)
    f = lib().oracle_lu_factor if pivot else lib().oracle_lu_factor_nopivot
    info = f(n, _p(A), _p(piv))
    return A, piv, info


def lu_solve(LU, piv, b, trans=False):
    b = np.array(b, dtype=np.float64)
    lib().oracle_lu_solve(LU.shape[0], _p(np.ascontiguousarray(LU)), _p(piv), _p(b), int(trans))
    return b


def integrate(mech, state, h, p, dt, rtol, atol, method="ros4", max_steps=100000, nthreads=0, **kw):
    """Integrate SoA state [N, ncells] in place-copy; returns (state, h, steps, rejects, status)."""
    m = _as_mech(mech)
    st = np.array(state, dtype=np.float64, order="C")
    N, nc = st.shape
    hh = np.array(h, dtype=np.float64) if h is not None else np.zeros(nc)
    steps, rej, status = np.zeros(nc, np.int32), np.zeros(nc, np.int32), np.zeros(nc, np.int32)
    o = opts(method, max_steps, **kw)
    lib().oracle_integrate(C.byref(m.s), C.c_int64(nc), C.c_int64(nc), _p(st), _p(hh), C.c_double(p),
                           C.c_double(dt), C.c_double(rtol), C.c_double(atol), C.byref(o),
                           _p(steps), _p(rej), _p(status), C.c_int(nthreads))
    return st, hh, steps, rej, status


def integrate_refmap(mech, state, h, p, dt, rtol, atol, weight, z0, z_max, dT, method="ros4", max_steps=100000,
                     nthreads=0, **kw):
    """Integration with reference-cell mapping (see oracle_integrate_refmap);
    returns (state, h, steps, rejects, status, ref_of)."""
    m = _as_mech(mech)
    st = np.array(state, dtype=np.float64, order="C")
    N, nc = st.shape
    hh = np.array(h, dtype=np.float64) if h is not None else np.zeros(nc)
    w = np.ascontiguousarray(weight, np.float64)
    assert w.shape == (N - 1,)
    steps, rej, status = np.zeros(nc, np.int32), np.zeros(nc, np.int32), np.zeros(nc, np.int32)
    ref_of = np.zeros(nc, np.int32)
    o = opts(method, max_steps, **kw)
    lib().oracle_integrate_refmap(C.byref(m.s), C.c_int64(nc), C.c_int64(nc), _p(st), _p(hh), C.c_double(p),
                                  C.c_double(dt), C.c_double(rtol), C.c_double(atol), C.byref(o), _p(w),
                                  C.c_double(z0), C.c_double(z_max), C.c_double(dT), _p(ref_of), _p(steps),
                                  _p(rej), _p(status), C.c_int(nthreads))
    return st, hh, steps, rej, status, ref_of


def integrate_record(mech, y0, h, p, dt, rtol, atol, method="ros4", max_steps=100000, cap=200000, **kw):
    """One cell; returns (y, h_out, hs, status, rejects)."""
    m = _as_mech(mech)
    y = np.array(y0, dtype=np.float64)
    hh = np.array([h if h is not None else 0.0])
    hs = np.zeros(cap)
    n, nr = C.c_int32(0), C.c_int32(0)
    o = opts(method, max_steps, **kw)
    st = lib().oracle_integrate_record(C.byref(m.s), C.c_double(p), C.c_double(dt), C.c_double(rtol),
                                       C.c_double(atol), C.byref(o), _p(y), _p(hh), _p(hs), cap,
                                       C.byref(n), C.byref(nr))
    return y, float(hh[0]), hs[:n.value].copy(), st, nr.value


def replay(mech, y0, hs, p, method="ros4"):
    m = _as_mech(mech)
    y0 = np.ascontiguousarray(y0, np.float64)
    hs = np.ascontiguousarray(hs, np.float64)
    out = np.zeros(m.N)
    rc = lib().oracle_replay(C.byref(m.s), C.c_double(p), METHOD.get(method, method), _p(y0), _p(hs),
                             len(hs), _p(out))
    if rc:
        raise RuntimeError("singular matrix during replay")
    return out


def tlm(mech, y0, hs, p, dy0=None, dlnA=None, db=None, dtheta=None, method="ros4"):
    """Final state and its derivative along the given direction (frozen step sizes)."""
    m = _as_mech(mech)
    y0 = np.ascontiguousarray(y0, np.float64)
    hs = np.ascontiguousarray(hs, np.float64)
    c = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
    dy0, dlnA, db, dtheta = c(dy0), c(dlnA), c(db), c(dtheta)
    yo, dyo = np.zeros(m.N), np.zeros(m.N)
    rc = lib().oracle_tlm(C.byref(m.s), C.c_double(p), METHOD.get(method, method), _p(y0), _p(hs),
                          len(hs), _p(dy0), _p(dlnA), _p(db), _p(dtheta), _p(yo), _p(dyo))
    if rc:
        raise RuntimeError("singular matrix during tangent-linear replay")
    return yo, dyo


def ros_test(method, problem, h, nsteps, y0):
    y0 = np.ascontiguousarray(y0, np.float64)
    n = 2 if problem == 0 else 1
    yo, eo = np.zeros(n), np.zeros(n)
    rc = lib().oracle_ros_test(METHOD.get(method, method), problem, C.c_double(h), nsteps, _p(y0), _p(yo),
                               _p(eo))
    if rc:
        raise RuntimeError("singular")
    return yo, eo


def sx_test(problem, H, nsteps, kcols, y0):
    """Fixed-column extrapolated linearly implicit Euler on a built-in test problem."""
    y0 = np.ascontiguousarray(y0, np.float64)
    n = 2 if problem == 0 else 1
    yo = np.zeros(n)
    rc = lib().oracle_sx_test(problem, C.c_double(H), nsteps, kcols, _p(y0), _p(yo))
    if rc:
        raise RuntimeError("sx_test failed")
    return yo


def num_threads():
    return lib().oracle_num_threads()


OUTCOME = {0: "accept", 1: "reject", 2: "nonfinite", 3: "singular", 4: "unstable"}


def controller_test(method, lam, y0, dt, rtol, atol, h=None, bound=0.0, cap=100000, **kw):
    """The adaptive integrator on y' = diag(lam) y (f NaN where |y_i| > bound).

    Returns (y, h_out, status, steps, rejects, trace) with trace an array of
    rows (h, err, outcome, k), one per step attempt."""
    lam = np.ascontiguousarray(lam, np.float64)
    y = np.array(y0, dtype=np.float64)
    n = lam.shape[0]
    assert y.shape == (n,)
    hh = np.array([h if h is not None else 0.0])
    tr = np.zeros((cap, 4))
    na, ns, nr = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    o = opts(method, **kw)
    st = lib().oracle_controller_test(METHOD.get(method, method), n, _p(lam), C.c_double(bound), _p(y),
                                      C.c_double(dt), C.c_double(rtol), C.c_double(atol), C.byref(o), _p(hh),
                                      _p(tr), cap, C.byref(na), C.byref(ns), C.byref(nr))
    return y, float(hh[0]), st, ns.value, nr.value, tr[:min(na.value, cap)].copy()


OP_KINDS = ("add", "mul", "div", "exp", "log")


def op_counts(mech, p, y):
    """Floating-point operations of one f evaluation and of one analytic
    Jacobian pass (which also yields f) at state y, counted on the oracle's
    counting scalar: {"rhs": {...}, "jac": {...}} by kind."""
    m = _as_mech(mech)
    y = np.ascontiguousarray(y, np.float64)
    out = np.zeros(10)
    lib().oracle_op_counts(C.byref(m.s), C.c_double(p), _p(y), _p(out))
    return {"rhs": dict(zip(OP_KINDS, out[:5].tolist())), "jac": dict(zip(OP_KINDS, out[5:].tolist()))}


def tlm_matrix(mech, y0, hs, p, method="ros4", nthreads=0):
    """Full sensitivity matrix of the replayed integration: [N, N + 3R], the
    derivatives of the final state w.r.t. (y0, lnA, b, theta)."""
    m = _as_mech(mech)
    y0 = np.ascontiguousarray(y0, np.float64)
    hs = np.ascontiguousarray(hs, np.float64)
    S = np.zeros((m.N, m.N + 3 * m.R))
    rc = lib().oracle_tlm_matrix(C.byref(m.s), C.c_double(p), METHOD.get(method, method), _p(y0), _p(hs),
                                 len(hs), _p(S), C.c_int(nthreads))
    if rc:
        raise RuntimeError("singular matrix during tangent-linear replay")
    return S
