"""Plain FP64 CPU oracle for the fRG right-hand side -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``libfrg_oracle.so`` (plain C, see
``frg_oracle.c``) with numpy arrays and shares no code with the GPU library.

The paper (Rohe, hp-fRG) states the problem in Sec. 2 (Eq. (1): an explicit
ODE over one flat array of couplings, rhs evaluated with V frozen) and Sec. 4
(2D Hubbard model, three one-loop diagrams, Brillouin-zone quadrature, N
patches).  The concrete formulas this oracle implements are the readings
G1-G10 documented in ``frg_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frg_oracle.c")
_LIB = os.path.join(_HERE, "libfrg_oracle.so")
# A test that plants a mistake in a copy of the oracle (to show that a pin
# catches it) points this at the mutant's shared library.
_LIB_OVERRIDE = os.environ.get("FRG_ORACLE_LIB")

PH, PP = 0, 1
STOP_NONE, STOP_TMIN, STOP_DIVERGED, STOP_MAXSTEPS, STOP_NONFINITE, STOP_HMIN = range(6)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FP contraction, sin and cos
    as separate libm calls)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin-sin",
               "-fno-builtin-cos", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("t", C.c_double), ("tp", C.c_double), ("mu", C.c_double), ("U", C.c_double),
                ("N", C.c_int32), ("n_rad", C.c_int32), ("n_ang", C.c_int32)]


class _Egrid(C.Structure):
    _fields_ = [("n_E", C.c_int32), ("max_level", C.c_int32), ("rtol", C.c_double)]


class _OdeResult(C.Structure):
    _fields_ = [("reason", C.c_int32), ("s_end", C.c_double), ("s_c", C.c_double),
                ("s_c_interp", C.c_double), ("accepted", C.c_int32), ("rejected", C.c_int32),
                ("rhs_evals", C.c_int32), ("first_step_rhs", C.c_int32)]


class _FlowOpts(C.Structure):
    _fields_ = [("stepper", C.c_int32), ("T0", C.c_double), ("T_min", C.c_double),
                ("rtol", C.c_double), ("atol", C.c_double), ("vmax", C.c_double),
                ("h0", C.c_double), ("fixed_steps", C.c_int32), ("max_steps", C.c_int32)]


ODE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_double, C.POINTER(C.c_double),
                     C.POINTER(C.c_double), C.c_int64)

_lib = None
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build(force=True)
            L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params)]
        L.orc_create_egrid.restype = C.c_void_p
        L.orc_create_egrid.argtypes = [C.POINTER(_Params), C.POINTER(_Egrid)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        for f in ("orc_N", "orc_nf", "orc_num_pp", "orc_num_ph"):
            getattr(L, f).restype = C.c_int32
            getattr(L, f).argtypes = [C.c_void_p]
        L.orc_tables.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP, _IP]
        L.orc_row_pp.restype = C.c_int32
        L.orc_row_pp.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.orc_row_ph.restype = C.c_int32
        L.orc_row_ph.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.orc_eps.restype = C.c_double
        L.orc_eps.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_fold.restype = C.c_double
        L.orc_fold.argtypes = [C.c_double]
        L.orc_project.restype = C.c_int32
        L.orc_project.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_L.restype = C.c_double
        L.orc_L.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_bins.argtypes = [C.c_void_p, C.c_int32, _IP]
        L.orc_bubbles.argtypes = [C.c_void_p, C.c_double, C.c_int32, _DP, _DP]
        L.orc_rhs.argtypes = [C.c_void_p, C.c_double, _DP, _DP]
        L.orc_contract.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP]
        L.orc_rhs_entries.argtypes = [C.c_void_p, C.c_double, _DP, C.c_int64, _IP, _DP]
        L.orc_bubbles_se.argtypes = [C.c_void_p, C.c_double, C.c_int32, _DP, _DP, _DP]
        L.orc_dsigma.argtypes = [C.c_void_p, C.c_double, _DP, _DP, _DP]
        L.orc_rhs_se.argtypes = [C.c_void_p, C.c_double, _DP, _DP, _DP, _DP]
        L.orc_rhs_entries_se.argtypes = [C.c_void_p, C.c_double, _DP, _DP, C.c_int64, _IP, _DP]
        L.orc_rk4.restype = C.c_int32
        L.orc_rk4.argtypes = [ODE_FN, C.c_void_p, C.c_int64, _DP, C.c_double, C.c_double,
                              C.c_int32, C.c_double, C.POINTER(_OdeResult)]
        L.orc_dp54.restype = C.c_int32
        L.orc_dp54.argtypes = [ODE_FN, C.c_void_p, C.c_int64, _DP, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                               C.POINTER(_OdeResult), _DP, C.c_int32]
        L.orc_flow.restype = C.c_int32
        L.orc_flow.argtypes = [C.c_void_p, C.POINTER(_FlowOpts), _DP, C.POINTER(_OdeResult),
                               _DP, C.c_int32]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(_IP) if a is not None else None


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def fold(x: float) -> float:
    return lib().orc_fold(float(x))


def L(kind: int, deriv: int, xi1: float, xi2: float, T: float) -> float:
    """Bubble integrand: kind PH/PP, deriv 0 (L) or 1 (dL/dT)."""
    return lib().orc_L(int(kind), int(deriv), float(xi1), float(xi2), float(T))


def _result(r: _OdeResult) -> dict:
    return {k: getattr(r, k) for k, _ in _OdeResult._fields_}


def rk4(f, y0, s0, s1, nsteps, vmax=float("inf")):
    """Classical RK4 on dy/ds = f(s, y) (numpy callback); returns (y, result)."""
    y = np.ascontiguousarray(y0, dtype=np.float64).copy()
    n = y.size

    def cb(ctx, s, yp, dyp, nn):
        yy = np.ctypeslib.as_array(yp, shape=(nn,))
        dy = np.ctypeslib.as_array(dyp, shape=(nn,))
        dy[:] = f(s, yy.copy())

    fn = ODE_FN(cb)
    r = _OdeResult()
    lib().orc_rk4(fn, None, n, _dp(y), s0, s1, nsteps, vmax, C.byref(r))
    return y, _result(r)


def dp54(f, y0, s0, s_min, h0, rtol, atol, vmax, max_steps=0, log_cap=4096):
    """Dormand-Prince 5(4) on dy/ds = f(s, y); returns (y, result, log[accepted, 6])."""
    y = np.ascontiguousarray(y0, dtype=np.float64).copy()
    n = y.size

    def cb(ctx, s, yp, dyp, nn):
        yy = np.ctypeslib.as_array(yp, shape=(nn,))
        dy = np.ctypeslib.as_array(dyp, shape=(nn,))
        dy[:] = f(s, yy.copy())

    fn = ODE_FN(cb)
    r = _OdeResult()
    log = np.zeros((log_cap, 6))
    lib().orc_dp54(fn, None, n, _dp(y), s0, s_min, h0, rtol, atol, vmax, max_steps,
                   C.byref(r), _dp(log), log_cap)
    res = _result(r)
    return y, res, log[: min(res["accepted"], log_cap)]


class Model:
    """Geometry + rhs of one parameter set (t, t', mu, U, N, n_rad, n_ang).

    egrid = dict(n_E=..., max_level=..., rtol=...) replaces the polar fine grid
    by the energy-angle quadrature (Sec. 4); n_rad and n_ang are then ignored and
    every patch holds nf points (the longest sector's count, the others padded
    with zero weight)."""

    def __init__(self, t=1.0, tp=0.0, mu=0.0, U=2.0, N=16, n_rad=8, n_ang=8, egrid=None):
        t, tp, mu, U = float(t), float(tp), float(mu), float(U)
        self.params = dict(t=t, tp=tp, mu=mu, U=U, N=N, n_rad=n_rad, n_ang=n_ang)
        p = _Params(t, tp, mu, U, N, n_rad, n_ang)
        if egrid is None:
            self._h = lib().orc_create(C.byref(p))
        else:
            e = _Egrid(int(egrid["n_E"]), int(egrid["max_level"]), float(egrid["rtol"]))
            self.params["egrid"] = dict(n_E=e.n_E, max_level=e.max_level, rtol=e.rtol)
            self._h = lib().orc_create_egrid(C.byref(p), C.byref(e))
        if not self._h:
            raise ValueError(f"oracle rejected parameters {self.params}")
        self.N = N
        self.nf = lib().orc_nf(self._h)
        self.U = U
        self.Tpp = lib().orc_num_pp(self._h)
        self.Tph = lib().orc_num_ph(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # geometry -------------------------------------------------------------
    def tables(self, idx4: bool = True) -> dict:
        N, nf = self.N, self.nf
        kc = np.zeros((N, 2))
        bnd = np.zeros((N + 1, 2))
        fine = np.zeros((N * nf, 4))
        qpp = np.zeros((self.Tpp, 2))
        qph = np.zeros((self.Tph, 2))
        i4 = np.zeros((N, N, N), dtype=np.int32) if idx4 else None
        lib().orc_tables(self._h, _dp(kc), _dp(bnd), _dp(fine), _dp(qpp), _dp(qph), _ip(i4))
        out = dict(kc=kc, bnd=bnd, px=fine[:, 0].copy(), py=fine[:, 1].copy(),
                   w=fine[:, 2].copy(), xi=fine[:, 3].copy(), qpp=qpp, qph=qph)
        if idx4:
            out["idx4"] = i4
        return out

    def row_pp(self, j1, j2):
        return lib().orc_row_pp(self._h, j1, j2)

    def row_ph(self, x, y):
        return lib().orc_row_ph(self._h, x, y)

    def eps(self, kx, ky):
        return lib().orc_eps(self._h, float(kx), float(ky))

    def project(self, kx, ky):
        return lib().orc_project(self._h, float(kx), float(ky))

    def bins(self, kind: int) -> np.ndarray:
        T = self.Tpp if kind == PP else self.Tph
        out = np.zeros((T, self.N * self.nf), dtype=np.int32)
        lib().orc_bins(self._h, kind, _ip(out))
        return out

    # bubbles / rhs --------------------------------------------------------
    def bubbles(self, T: float, deriv: int = 1):
        N = self.N
        Bpp = np.zeros((self.Tpp, N, N))
        Bph = np.zeros((self.Tph, N, N))
        lib().orc_bubbles(self._h, float(T), int(deriv), _dp(Bpp), _dp(Bph))
        return Bpp, Bph

    def contract(self, Bpp, Bph, V):
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.zeros_like(V)
        lib().orc_contract(self._h, _dp(np.ascontiguousarray(Bpp)), _dp(np.ascontiguousarray(Bph)),
                           _dp(V), _dp(F))
        return F

    def rhs(self, T: float, V: np.ndarray) -> np.ndarray:
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(self.N, self.N, self.N)
        F = np.zeros_like(V)
        lib().orc_rhs(self._h, float(T), _dp(V), _dp(F))
        return F

    def rhs_full(self, T: float, V: np.ndarray) -> np.ndarray:
        """Interaction flow (Sec. 4's working example: at fixed T the bare
        on-site interaction carries the flow parameter g): dV/dg has the three
        one-loop channels of the temperature flow with the full bubbles L_T in
        place of their T-derivative."""
        Bpp, Bph = self.bubbles(T, deriv=0)
        return self.contract(Bpp, Bph, np.ascontiguousarray(V, dtype=np.float64).reshape(self.N, self.N, self.N))

    def iflow(self, T: float, V0=None, stepper="rk4", g0=0.0, g1=1.0, fixed_steps=40, rtol=1e-6,
              atol=1e-10, vmax=20.0, h0=0.01, max_steps=0, log_cap=4096):
        """Interaction flow dV/dg = F_L(V) from V(g0) = V0 (default U) to g1; the
        bubbles L_T are computed once.  Returns (V, result, log)."""
        N = self.N
        V = (np.full((N, N, N), float(self.U)) if V0 is None
             else np.ascontiguousarray(V0, dtype=np.float64).copy())
        Bpp, Bph = self.bubbles(T, deriv=0)
        f = lambda g, y: self.contract(Bpp, Bph, y.reshape(N, N, N)).ravel()
        if stepper == "rk4":
            y, res = rk4(f, V.ravel(), g0, g1, fixed_steps, vmax)
            log = np.zeros((0, 6))
        else:
            y, res, log = dp54(f, V.ravel(), g0, g1, h0, rtol, atol, vmax, max_steps, log_cap)
        return y.reshape(N, N, N), res, log

    def rhs_entries(self, T: float, V: np.ndarray, j123) -> np.ndarray:
        V = np.ascontiguousarray(V, dtype=np.float64)
        idx = np.ascontiguousarray(np.asarray(j123, dtype=np.int32).reshape(-1, 3))
        out = np.zeros(idx.shape[0])
        lib().orc_rhs_entries(self._h, float(T), _dp(V), idx.shape[0], _ip(idx), _dp(out))
        return out

    # self-energy ----------------------------------------------------------
    def bubbles_se(self, T: float, S, deriv: int = 1):
        N = self.N
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(N)
        Bpp = np.zeros((self.Tpp, N, N))
        Bph = np.zeros((self.Tph, N, N))
        lib().orc_bubbles_se(self._h, float(T), int(deriv), _dp(S), _dp(Bpp), _dp(Bph))
        return Bpp, Bph

    def dsigma(self, T: float, V, S) -> np.ndarray:
        N = self.N
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(N, N, N)
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(N)
        out = np.zeros(N)
        lib().orc_dsigma(self._h, float(T), _dp(V), _dp(S), _dp(out))
        return out

    def rhs_se(self, T: float, V, S):
        """(dV/dT, dS/dT) with the self-energy S in every loop line."""
        N = self.N
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(N, N, N)
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(N)
        F = np.zeros_like(V)
        dS = np.zeros(N)
        lib().orc_rhs_se(self._h, float(T), _dp(V), _dp(S), _dp(F), _dp(dS))
        return F, dS

    def rhs_entries_se(self, T: float, V, S, j123) -> np.ndarray:
        V = np.ascontiguousarray(V, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(self.N)
        idx = np.ascontiguousarray(np.asarray(j123, dtype=np.int32).reshape(-1, 3))
        out = np.zeros(idx.shape[0])
        lib().orc_rhs_entries_se(self._h, float(T), _dp(V), _dp(S), idx.shape[0], _ip(idx), _dp(out))
        return out

    def flow_se(self, V0=None, S0=None, stepper="dp54", T0=1.0, T_min=0.05, fixed_steps=40, rtol=1e-6,
                atol=1e-10, vmax=20.0, h0=-0.01, max_steps=0, log_cap=4096):
        """Temperature flow of the vertex and the self-energy together: y = (V, S)
        in s = ln T with dy/ds = T (dV/dT, dS/dT); returns (V, S, result, log)."""
        N = self.N
        n3 = N ** 3
        V = (np.full((N, N, N), float(self.U)) if V0 is None
             else np.ascontiguousarray(V0, dtype=np.float64))
        S = np.zeros(N) if S0 is None else np.ascontiguousarray(S0, dtype=np.float64)
        y0 = np.concatenate([V.ravel(), S.ravel()])

        def f(s, y):
            T = math.exp(s)
            F, dS = self.rhs_se(T, y[:n3], y[n3:])
            return T * np.concatenate([F.ravel(), dS])
        s0, s1 = math.log(T0), math.log(T_min)
        if stepper == "rk4":
            y, res = rk4(f, y0, s0, s1, fixed_steps, vmax)
            log = np.zeros((0, 6))
        else:
            y, res, log = dp54(f, y0, s0, s1, h0, rtol, atol, vmax, max_steps, log_cap)
        return y[:n3].reshape(N, N, N), y[n3:].copy(), res, log

    def flow(self, V0=None, stepper="rk4", T0=1.0, T_min=0.05, fixed_steps=40, rtol=1e-6,
             atol=1e-10, vmax=20.0, h0=-0.01, max_steps=0, log_cap=4096):
        """Temperature flow dV/ds = T F(V,T) in s = ln T; returns (V, result, log)."""
        N = self.N
        V = (np.full((N, N, N), float(self.U)) if V0 is None
             else np.ascontiguousarray(V0, dtype=np.float64).copy())
        o = _FlowOpts(0 if stepper == "rk4" else 1, T0, T_min, rtol, atol, vmax, h0,
                      fixed_steps, max_steps)
        r = _OdeResult()
        log = np.zeros((log_cap, 6))
        lib().orc_flow(self._h, C.byref(o), _dp(V), C.byref(r), _dp(log), log_cap)
        res = _result(r)
        return V, res, log[: min(res["accepted"], log_cap)]
