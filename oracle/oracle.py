"""ctypes front end of the CPU oracle (test infrastructure only).

The oracle library works on array-of-structures states; these helpers take
and return the structure-of-arrays layout the GPU library uses (float64
[N][n], row 0 = T, rows 1.. = Y_k) and transpose internally.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h0", C.c_double),
                ("h_fixed", C.c_double), ("max_steps", C.c_int64), ("jac_fd", C.c_int32), ("cv", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        vp, dp, ip, i64 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int64
        L.orc_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.orc_free.argtypes = [vp]
        L.orc_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_species_data.argtypes = [vp, dp, C.POINTER(C.c_int)]
        L.orc_thermo.argtypes = [vp, C.c_double, dp, dp, dp]
        L.orc_rhs.argtypes = [vp, i64, dp, dp, dp, C.c_int]
        L.orc_jac.argtypes = [vp, i64, dp, dp, dp, C.c_int]
        L.orc_rhs_cv.argtypes = [vp, i64, dp, dp, dp, C.c_int]
        L.orc_jac_cv.argtypes = [vp, i64, dp, dp, dp, C.c_int]
        L.orc_jac_fd.argtypes = [vp, i64, dp, dp, C.c_double, C.c_double, C.c_double, dp, C.c_int]
        L.orc_rates.argtypes = [vp, dp, C.c_double, dp, dp, dp, dp, dp]
        L.orc_stoich.argtypes = [vp, C.POINTER(C.c_int)]
        L.orc_integrate.argtypes = [vp, C.c_int, i64, dp, dp, dp, dp, dp, C.POINTER(Opts), ip, ip, ip, C.c_int]
        L.orc_integrate_linear.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, dp, dp, C.POINTER(Opts), ip, ip,
                                           ip, C.POINTER(C.c_long)]
        L.orc_step_linear.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, dp, dp]
        L.orc_lu_solve.argtypes = [C.c_int, dp, dp]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


METHODS = {"ros4": 0, "rkf45": 1}


JACOBIANS = {"analytic": 0, "fd": 1}
REACTORS = {"cp": 0, "cv": 1}     # constant pressure (P in Pa) / constant volume (P holds densities, kg/m^3)


def make_opts(rtol=1e-8, atol=1e-12, h0=0.0, h_fixed=0.0, max_steps=1_000_000, jacobian="analytic", reactor="cp"):
    return Opts(rtol, atol, h0, h_fixed, max_steps, JACOBIANS[jacobian], REACTORS[reactor])


class Mechanism:
    def __init__(self, path):
        L = lib()
        h = C.c_void_p()
        rc = L.orc_load(path.encode(), C.byref(h))
        if rc != 0:
            raise IOError(f"oracle could not load {path} (code {rc})")
        self._h = h
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        L.orc_info(h, C.byref(a), C.byref(b), C.byref(c))
        self.n_species, self.n_reactions, self.n_elements = a.value, b.value, c.value
        self.N = self.n_species + 1
        self.W = np.zeros(self.n_species)
        comp = np.zeros((self.n_species, self.n_elements), dtype=np.int32)
        L.orc_species_data(h, _d(self.W), comp.ctypes.data_as(C.POINTER(C.c_int)))
        self.comp = comp

    def __del__(self):
        try:
            if self._h:
                lib().orc_free(self._h)
        except Exception:
            pass

    # --- thermo / rates -------------------------------------------------------------------
    def thermo(self, T):
        cp, h, s = (np.zeros(self.n_species) for _ in range(3))
        lib().orc_thermo(self._h, float(T), _d(cp), _d(h), _d(s))
        return cp, h, s

    def rates(self, y_col, P):
        y = np.ascontiguousarray(y_col, dtype=np.float64)
        qf, qr = np.zeros(self.n_reactions), np.zeros(self.n_reactions)
        rho, cp = C.c_double(), C.c_double()
        hRT = np.zeros(self.n_species)
        lib().orc_rates(self._h, _d(y), float(P), _d(qf), _d(qr), C.byref(rho), C.byref(cp), _d(hRT))
        return qf, qr, rho.value, cp.value, hRT

    def stoich(self):
        nu = np.zeros((self.n_species, self.n_reactions), dtype=np.int32)
        lib().orc_stoich(self._h, nu.ctypes.data_as(C.POINTER(C.c_int)))
        return nu

    # --- batch calls (SoA in, SoA out) ------------------------------------------------------
    def rhs(self, y, P, nthreads=0, reactor="cp"):
        """dy/dt [N][n]; P holds pressures (Pa) for reactor="cp", densities (kg/m^3) for "cv"."""
        y = np.asarray(y, dtype=np.float64)
        n = y.shape[1]
        aos = np.array(y.T, dtype=np.float64, order="C", copy=True)
        out = np.zeros_like(aos)
        Pa = np.ascontiguousarray(np.broadcast_to(P, (n,)), dtype=np.float64)
        fn = lib().orc_rhs if reactor == "cp" else lib().orc_rhs_cv
        fn(self._h, n, _d(aos), _d(Pa), _d(out), nthreads)
        return np.ascontiguousarray(out.T)

    def jac(self, y, P, nthreads=0, reactor="cp"):
        """Returns J as [n][N][N] (reactor, row i = df_i, column j = d/dy_j)."""
        y = np.asarray(y, dtype=np.float64)
        n = y.shape[1]
        aos = np.array(y.T, dtype=np.float64, order="C", copy=True)
        out = np.zeros((n, self.N, self.N))
        Pa = np.ascontiguousarray(np.broadcast_to(P, (n,)), dtype=np.float64)
        fn = lib().orc_jac if reactor == "cp" else lib().orc_jac_cv
        fn(self._h, n, _d(aos), _d(Pa), _d(out), nthreads)
        return out

    def jac_fd(self, y, P, h, rtol=1e-8, atol=1e-12, nthreads=0):
        """Forward-difference Jacobian (increments for step h and tolerances rtol / atol), as jac()."""
        y = np.asarray(y, dtype=np.float64)
        n = y.shape[1]
        aos = np.array(y.T, dtype=np.float64, order="C", copy=True)
        out = np.zeros((n, self.N, self.N))
        Pa = np.ascontiguousarray(P, dtype=np.float64)
        lib().orc_jac_fd(self._h, n, _d(aos), _d(Pa), float(rtol), float(atol), float(h), _d(out), nthreads)
        return out

    def integrate(self, y, P, t_end, method="ros4", rtol=1e-8, atol=1e-12, h0=0.0, h_fixed=0.0,
                  max_steps=1_000_000, t=None, h=None, nthreads=0, jacobian="analytic", reactor="cp"):
        """Integrate each reactor to t_end.  Returns dict(y, t, h, status, n_accept, n_reject)."""
        y = np.asarray(y, dtype=np.float64)
        n = y.shape[1]
        aos = np.array(y.T, dtype=np.float64, order="C", copy=True)
        Pa = np.ascontiguousarray(np.broadcast_to(P, (n,)), dtype=np.float64)
        te = np.ascontiguousarray(np.broadcast_to(t_end, (n,)), dtype=np.float64)
        tt = np.zeros(n) if t is None else np.array(t, dtype=np.float64)
        hh = np.zeros(n) if h is None else np.array(h, dtype=np.float64)
        st, na, nr = (np.zeros(n, dtype=np.int32) for _ in range(3))
        o = make_opts(rtol, atol, h0, h_fixed, max_steps, jacobian, reactor)
        lib().orc_integrate(self._h, METHODS[method], n, _d(aos), _d(Pa), _d(te), _d(tt), _d(hh), C.byref(o),
                            _i(st), _i(na), _i(nr), nthreads)
        return dict(y=np.ascontiguousarray(aos.T), t=tt, h=hh, status=st, n_accept=na, n_reject=nr)


def integrate_linear(A, y0, t_end, method="ros4", rtol=1e-8, atol=1e-12, h0=0.0, h_fixed=0.0, max_steps=1_000_000,
                     jacobian="analytic", t0=0.0):
    """y' = A y from t0 to t_end.  Returns dict(y, t, h, status, n_accept, n_reject, nfev)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    N = A.shape[0]
    y = np.array(y0, dtype=np.float64)
    t, h = C.c_double(float(t0)), C.c_double(0.0)
    st, na, nr = C.c_int32(), C.c_int32(), C.c_int32()
    nfev = C.c_long()
    o = make_opts(rtol, atol, h0, h_fixed, max_steps, jacobian)
    lib().orc_integrate_linear(METHODS[method], N, _d(A), _d(y), float(t_end), C.byref(t), C.byref(h), C.byref(o),
                               C.byref(st), C.byref(na), C.byref(nr), C.byref(nfev))
    return dict(y=y, t=t.value, h=h.value, status=st.value, n_accept=na.value, n_reject=nr.value, nfev=nfev.value)


def step_linear(A, y, h, method="ros4"):
    A = np.ascontiguousarray(np.atleast_2d(A), dtype=np.float64)
    N = A.shape[0]
    y = np.ascontiguousarray(np.atleast_1d(y), dtype=np.float64)
    yn, err = np.zeros(N), np.zeros(N)
    info = lib().orc_step_linear(METHODS[method], N, _d(A), _d(y), float(h), _d(yn), _d(err))
    if info:
        raise ArithmeticError("singular iteration matrix")
    return yn, err


def lu_solve(a, b):
    a = np.array(a, dtype=np.float64, order="C")
    b = np.array(b, dtype=np.float64)
    info = lib().orc_lu_solve(a.shape[0], _d(a), _d(b))
    if info:
        raise ArithmeticError("singular matrix")
    return b


def max_threads():
    return lib().orc_max_threads()
