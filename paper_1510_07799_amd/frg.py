"""Thin ctypes binding of libfrg (include/frg.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libfrg.so``; torch is used for
device memory and the current stream.  If the library is missing the import
of this module fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrg.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP, ENONFINITE = range(6)
PREC_FP64, PREC_SPLIT_BF16 = 0, 1
RK4, DP54 = 0, 1
STOP_NONE, STOP_TMIN, STOP_DIVERGED, STOP_MAXSTEPS, STOP_NONFINITE, STOP_HMIN = range(6)
STATE_LEN = 32
ST_S, ST_H, ST_ERR, ST_REASON, ST_ACCEPTED, ST_REJECTED, ST_RHS, ST_VMAX = range(8)
KERNEL_CLASSES = ("prep", "bubbles", "layout", "contract", "combine", "rk")


class FRGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfrg error {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("t", C.c_double), ("tp", C.c_double), ("mu", C.c_double), ("U", C.c_double),
                ("N", C.c_int32), ("n_rad", C.c_int32), ("n_ang", C.c_int32)]


class FlowOpts(C.Structure):
    _fields_ = [("stepper", C.c_int32), ("prec", C.c_int32), ("T0", C.c_double),
                ("T_min", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("vmax", C.c_double), ("h0", C.c_double), ("fixed_steps", C.c_int32),
                ("max_steps", C.c_int32)]


class FlowResult(C.Structure):
    _fields_ = [("reason", C.c_int32), ("T_end", C.c_double), ("T_c", C.c_double),
                ("T_c_interp", C.c_double), ("accepted", C.c_int32), ("rejected", C.c_int32),
                ("rhs_evals", C.c_int32), ("first_step_rhs", C.c_int32)]


class IFlowOpts(C.Structure):
    _fields_ = [("stepper", C.c_int32), ("prec", C.c_int32), ("T", C.c_double), ("g0", C.c_double),
                ("g1", C.c_double), ("rtol", C.c_double), ("atol", C.c_double), ("vmax", C.c_double),
                ("h0", C.c_double), ("fixed_steps", C.c_int32), ("max_steps", C.c_int32)]


class IFlowResult(C.Structure):
    _fields_ = [("reason", C.c_int32), ("g_end", C.c_double), ("g_c", C.c_double),
                ("g_c_interp", C.c_double), ("accepted", C.c_int32), ("rejected", C.c_int32),
                ("rhs_evals", C.c_int32), ("first_step_rhs", C.c_int32)]


class Egrid(C.Structure):
    _fields_ = [("n_E", C.c_int32), ("max_level", C.c_int32), ("rtol", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("kparts", C.c_int32), ("sweep_rows", C.c_int32), ("block_rows", C.c_int32)]


_lib = None
_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)
_SZ = C.POINTER(C.c_size_t)

# name -> (restype, argtypes)
SIGNATURES = {
    "frg_create": (C.c_int, [C.POINTER(Params), C.POINTER(_P)]),
    "frg_destroy": (C.c_int, [_P]),
    "frg_sizes": (C.c_int, [_P, _SZ, _SZ, _SZ, _SZ]),
    "frg_tables": (C.c_int, [_P, _DP, _DP, _DP, _DP, _DP, _IP]),
    "frg_host_tables": (C.c_int, [C.POINTER(Params), _DP, _DP, _DP, _DP, _DP, _IP]),
    "frg_create_egrid": (C.c_int, [C.POINTER(Params), C.POINTER(Egrid), C.POINTER(_P)]),
    "frg_points": (C.c_int, [_P, _IP, _IP]),
    "frg_set_self_energy": (C.c_int, [_P, C.c_int32]),
    "frg_self_energy": (C.c_int, [_P, _IP]),
    "frg_host_tables_egrid": (C.c_int, [C.POINTER(Params), C.POINTER(Egrid), _IP, _IP, _DP, _DP, _DP, _DP, _DP,
                                        _IP]),
    "frg_bins": (C.c_int, [_P, C.c_int32, _P, _P]),
    "frg_bubbles": (C.c_int, [_P, C.c_double, C.c_int, _P, _P, _P]),
    "frg_bubble_reps": (C.c_int, [_P, _IP, _IP, _IP]),
    "frg_bubbles_reps": (C.c_int, [_P, C.c_double, C.c_int, _P, _P, _P]),
    "frg_rhs": (C.c_int, [_P, C.c_double, _P, _P, C.c_int, _P]),
    "frg_rhs_noalloc": (C.c_int, [_P, C.c_double, _P, _P, C.c_int, _P]),
    "frg_flow_init": (C.c_int, [_P, C.POINTER(FlowOpts), _P, _P, _P]),
    "frg_flow_step": (C.c_int, [_P, C.POINTER(FlowOpts), _P, _P, _P]),
    "frg_flow": (C.c_int, [_P, C.POINTER(FlowOpts), _P, _P, C.c_int32, C.POINTER(FlowResult), _P]),
    "frg_batch_create": (C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(_P)]),
    "frg_batch_destroy": (C.c_int, [_P]),
    "frg_batch_context": (C.c_int, [_P, C.c_int32, C.POINTER(_P)]),
    "frg_batch_rhs": (C.c_int, [_P, _DP, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int, _P]),
    "frg_batch_flow": (C.c_int, [_P, C.POINTER(FlowOpts), C.POINTER(C.c_void_p), _P, C.c_int32,
                                 C.POINTER(FlowResult), _P]),
    "frg_batch_flow_init": (C.c_int, [_P, C.POINTER(FlowOpts), C.POINTER(C.c_void_p), _P, C.c_int32, _P]),
    "frg_batch_flow_step": (C.c_int, [_P, _P]),
    "frg_batch_results": (C.c_int, [_P, C.POINTER(FlowResult), _IP]),
    "frg_bubbles_full": (C.c_int, [_P, C.c_double, C.c_int, _P, _P, _P]),
    "frg_rhs_full": (C.c_int, [_P, C.c_double, _P, _P, C.c_int, _P]),
    "frg_iflow_init": (C.c_int, [_P, C.POINTER(IFlowOpts), _P, _P, _P]),
    "frg_iflow_step": (C.c_int, [_P, C.POINTER(IFlowOpts), _P, _P, _P]),
    "frg_iflow": (C.c_int, [_P, C.POINTER(IFlowOpts), _P, _P, C.c_int32, C.POINTER(IFlowResult), _P]),
    "frg_set_symmetry": (C.c_int, [_P, C.c_int32]),
    "frg_symmetry": (C.c_int, [_P, _IP, _IP]),
    "frg_set_kskip": (C.c_int, [_P, C.c_int32]),
    "frg_kskip": (C.c_int, [_P, _IP, _DP]),
    "frg_set_vsym": (C.c_int, [_P, C.c_int32]),
    "frg_vsym": (C.c_int, [_P, _IP, _IP]),
    "frg_check_vsym": (C.c_int, [_P, _P, _DP, _P]),
    "frg_batch_set_vsym": (C.c_int, [_P, C.c_int32]),
    "frg_profile_begin": (C.c_int, [_P]),
    "frg_profile_end": (C.c_int, [_P, _DP, _IP]),
    "frg_get_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "frg_set_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "frg_tune": (C.c_int, [_P, C.c_double, _P, _P, C.c_int, C.c_int32, C.POINTER(Tuning), _DP, _DP, C.c_int32,
                           _IP, _P]),
    "frg_batch_set_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "frg_batch_tune": (C.c_int, [_P, _DP, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int, C.c_int32,
                                 C.POINTER(Tuning), _DP, _DP, C.c_int32, _IP, _P]),
    "frg_batch_profile_begin": (C.c_int, [_P]),
    "frg_batch_profile_end": (C.c_int, [_P, _DP, _IP]),
    "frg_status_str": (C.c_char_p, [C.c_int]),
    "frg_last_error": (C.c_char_p, []),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python -m paper_1510_07799_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        msg = lib().frg_last_error().decode(errors="replace")
        raise FRGError(st, msg)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def params(t=1.0, tp=0.0, mu=0.0, U=2.0, N=16, n_rad=8, n_ang=8) -> Params:
    return Params(float(t), float(tp), float(mu), float(U), int(N), int(n_rad), int(n_ang))


def egrid(n_E, max_level, rtol) -> Egrid:
    return Egrid(int(n_E), int(max_level), float(rtol))


def host_tables(t=1.0, tp=0.0, mu=0.0, U=2.0, N=16, n_rad=8, n_ang=8, idx4=True, egrid=None) -> dict:
    """Geometry tables built by the library's host code (no device needed).
    egrid = dict(n_E, max_level, rtol): the energy-angle grid (adds n_f and the
    per-patch live counts)."""
    p = params(t, tp, mu, U, N, n_rad, n_ang)
    Tpp, Tph = N * (N + 1) // 2, N * (N - 1) + 1
    if egrid is not None:
        e = Egrid(int(egrid["n_E"]), int(egrid["max_level"]), float(egrid["rtol"]))
        nfv = C.c_int32()
        cnt = np.zeros(N, dtype=np.int32)
        _check(lib().frg_host_tables_egrid(C.byref(p), C.byref(e), C.byref(nfv), None, None, None, None, None,
                                           None, None))
        nf = nfv.value
        kc = np.zeros((N, 2))
        bnd = np.zeros((N + 1, 2))
        fine = np.zeros((N * nf, 4))
        qpp = np.zeros((Tpp, 2))
        qph = np.zeros((Tph, 2))
        i4 = np.zeros((N, N, N), dtype=np.int32) if idx4 else None
        dp = lambda a: a.ctypes.data_as(_DP)
        _check(lib().frg_host_tables_egrid(C.byref(p), C.byref(e), C.byref(nfv), cnt.ctypes.data_as(_IP), dp(kc),
                                           dp(bnd), dp(fine), dp(qpp), dp(qph),
                                           i4.ctypes.data_as(_IP) if idx4 else None))
        out = dict(kc=kc, bnd=bnd, px=fine[:, 0].copy(), py=fine[:, 1].copy(), w=fine[:, 2].copy(),
                   xi=fine[:, 3].copy(), qpp=qpp, qph=qph, nf=nf, count=cnt)
        if idx4:
            out["idx4"] = i4
        return out
    nf = n_rad * n_ang
    kc = np.zeros((N, 2))
    bnd = np.zeros((N + 1, 2))
    fine = np.zeros((N * nf, 4))
    qpp = np.zeros((Tpp, 2))
    qph = np.zeros((Tph, 2))
    i4 = np.zeros((N, N, N), dtype=np.int32) if idx4 else None
    dp = lambda a: a.ctypes.data_as(_DP)
    _check(lib().frg_host_tables(C.byref(p), dp(kc), dp(bnd), dp(fine), dp(qpp), dp(qph),
                                 i4.ctypes.data_as(_IP) if idx4 else None))
    out = dict(kc=kc, bnd=bnd, px=fine[:, 0].copy(), py=fine[:, 1].copy(), w=fine[:, 2].copy(),
               xi=fine[:, 3].copy(), qpp=qpp, qph=qph)
    if idx4:
        out["idx4"] = i4
    return out


def flow_opts(stepper="rk4", prec=PREC_FP64, T0=1.0, T_min=0.05, rtol=1e-6, atol=1e-10,
              vmax=20.0, h0=-0.01, fixed_steps=40, max_steps=0) -> FlowOpts:
    st = RK4 if stepper in ("rk4", RK4) else DP54
    return FlowOpts(st, int(prec), float(T0), float(T_min), float(rtol), float(atol),
                    float(vmax), float(h0), int(fixed_steps), int(max_steps))


def iflow_opts(stepper="rk4", prec=PREC_FP64, T=0.1, g0=0.0, g1=1.0, rtol=1e-6, atol=1e-10,
               vmax=20.0, h0=0.01, fixed_steps=40, max_steps=0) -> IFlowOpts:
    st = RK4 if stepper in ("rk4", RK4) else DP54
    return IFlowOpts(st, int(prec), float(T), float(g0), float(g1), float(rtol), float(atol),
                     float(vmax), float(h0), int(fixed_steps), int(max_steps))


class Context:
    """One parameter set on the current HIP device (owns geometry + workspace)."""

    def __init__(self, t=1.0, tp=0.0, mu=0.0, U=2.0, N=16, n_rad=8, n_ang=8, egrid=None):
        import torch
        self.torch = torch
        self.N, self.nf, self.U = int(N), int(n_rad) * int(n_ang), float(U)
        self.Tpp, self.Tph = N * (N + 1) // 2, N * (N - 1) + 1
        self.params = dict(t=t, tp=tp, mu=mu, U=U, N=N, n_rad=n_rad, n_ang=n_ang)
        p = params(t, tp, mu, U, N, n_rad, n_ang)
        h = _P()
        if egrid is None:
            _check(lib().frg_create(C.byref(p), C.byref(h)))
        else:
            e = Egrid(int(egrid["n_E"]), int(egrid["max_level"]), float(egrid["rtol"]))
            self.params["egrid"] = dict(n_E=e.n_E, max_level=e.max_level, rtol=e.rtol)
            _check(lib().frg_create_egrid(C.byref(p), C.byref(e), C.byref(h)))
        self._h = h
        nfv = C.c_int32()
        _check(lib().frg_points(h, C.byref(nfv), None))
        self.nf = nfv.value

    def counts(self):
        """live points of every patch (n_f each on a polar grid)"""
        c = np.zeros(self.N, dtype=np.int32)
        _check(lib().frg_points(self._h, None, c.ctypes.data_as(_IP)))
        return c

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().frg_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def sizes(self):
        a, b, c, d = C.c_size_t(), C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(lib().frg_sizes(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return dict(n_v=a.value, n_bpp=b.value, n_bph=c.value, workspace_bytes=d.value)

    def tables(self, idx4=True):
        N, nf = self.N, self.nf
        kc = np.zeros((N, 2))
        bnd = np.zeros((N + 1, 2))
        fine = np.zeros((N * nf, 4))
        qpp = np.zeros((self.Tpp, 2))
        qph = np.zeros((self.Tph, 2))
        i4 = np.zeros((N, N, N), dtype=np.int32) if idx4 else None
        dp = lambda a: a.ctypes.data_as(_DP)
        _check(lib().frg_tables(self._h, dp(kc), dp(bnd), dp(fine), dp(qpp), dp(qph),
                                i4.ctypes.data_as(_IP) if idx4 else None))
        out = dict(kc=kc, bnd=bnd, px=fine[:, 0].copy(), py=fine[:, 1].copy(),
                   w=fine[:, 2].copy(), xi=fine[:, 3].copy(), qpp=qpp, qph=qph)
        if idx4:
            out["idx4"] = i4
        return out

    def bins(self, kind: int):
        torch = self.torch
        rows = self.Tpp if kind == 1 else self.Tph
        out = torch.empty((rows, self.N * self.nf), dtype=torch.uint8, device="cuda")
        _check(lib().frg_bins(self._h, int(kind), _ptr(out), _stream()))
        return out

    def bubbles(self, T: float, prec=PREC_FP64):
        torch = self.torch
        dt = torch.float64 if prec == PREC_FP64 else torch.float32
        N = self.N
        Bpp = torch.empty((self.Tpp, N, N), dtype=dt, device="cuda")
        Bph = torch.empty((self.Tph, N, N), dtype=dt, device="cuda")
        _check(lib().frg_bubbles(self._h, float(T), int(prec), _ptr(Bpp), _ptr(Bph), _stream()))
        return Bpp, Bph

    def bubble_reps(self):
        """(pp rows, paired ph rows) that the C4v-reduced sweep evaluates."""
        n = C.c_int32()
        _check(lib().frg_bubble_reps(self._h, C.byref(n), None, None))
        pp = np.zeros(n.value, dtype=np.int32)
        ph = np.zeros(n.value, dtype=np.int32)
        _check(lib().frg_bubble_reps(self._h, C.byref(n), pp.ctypes.data_as(_IP), ph.ctypes.data_as(_IP)))
        return pp, ph

    def bubbles_reps(self, T: float, prec=PREC_FP64):
        """The paired sweep of the rhs: rows [n_rep][N][N] of both kinds."""
        torch = self.torch
        dt = torch.float64 if prec == PREC_FP64 else torch.float32
        n = len(self.bubble_reps()[0])
        Bpp = torch.empty((n, self.N, self.N), dtype=dt, device="cuda")
        Bph = torch.empty((n, self.N, self.N), dtype=dt, device="cuda")
        _check(lib().frg_bubbles_reps(self._h, float(T), int(prec), _ptr(Bpp), _ptr(Bph), _stream()))
        return Bpp, Bph

    def bubbles_full(self, T: float, prec=PREC_FP64):
        """The full bubbles L_T (interaction flow), every row."""
        torch = self.torch
        dt = torch.float64 if prec == PREC_FP64 else torch.float32
        N = self.N
        Bpp = torch.empty((self.Tpp, N, N), dtype=dt, device="cuda")
        Bph = torch.empty((self.Tph, N, N), dtype=dt, device="cuda")
        _check(lib().frg_bubbles_full(self._h, float(T), int(prec), _ptr(Bpp), _ptr(Bph), _stream()))
        return Bpp, Bph

    def rhs_full(self, T: float, V, prec=PREC_FP64, out=None):
        """dV/dg of the interaction flow at temperature T."""
        torch = self.torch
        N = self.N
        assert V.dtype == torch.float64 and V.is_cuda and V.is_contiguous() and V.numel() == N ** 3
        F = out if out is not None else torch.empty_like(V)
        _check(lib().frg_rhs_full(self._h, float(T), _ptr(V), _ptr(F), int(prec), _stream()))
        return F

    def iflow_init(self, opts: IFlowOpts, V, state):
        _check(lib().frg_iflow_init(self._h, C.byref(opts), _ptr(V), _ptr(state), _stream()))

    def iflow_step(self, opts: IFlowOpts, V, state):
        _check(lib().frg_iflow_step(self._h, C.byref(opts), _ptr(V), _ptr(state), _stream()))

    def iflow(self, V, opts: IFlowOpts, log_cap=4096):
        """Run a whole interaction flow in place on V; returns (result dict, log [accepted, 8])."""
        torch = self.torch
        log = torch.zeros((max(log_cap, 1), 8), dtype=torch.float64, device="cuda")
        r = IFlowResult()
        st = lib().frg_iflow(self._h, C.byref(opts), _ptr(V), _ptr(log), int(log_cap), C.byref(r), _stream())
        res = {k: getattr(r, k) for k, _ in IFlowResult._fields_}
        if st not in (OK, ENONFINITE):
            _check(st)
        torch.cuda.synchronize()
        n = min(res["accepted"], log_cap)
        return res, log[:n].cpu().numpy()

    def rhs(self, T: float, V, prec=PREC_FP64, out=None):
        torch = self.torch
        N = self.N
        n = N ** 3 + (N if self.self_energy() else 0)
        assert V.dtype == torch.float64 and V.is_cuda and V.is_contiguous() and V.numel() == n
        F = out if out is not None else torch.empty_like(V)
        _check(lib().frg_rhs(self._h, float(T), _ptr(V), _ptr(F), int(prec), _stream()))
        return F

    def rhs_noalloc(self, T: float, V, F, prec=PREC_FP64):
        """frg_rhs_noalloc: F (caller's buffer) from the library's static scratch."""
        torch = self.torch
        N = self.N
        assert V.dtype == torch.float64 and V.is_cuda and V.is_contiguous() and V.numel() == N ** 3
        assert F.dtype == torch.float64 and F.is_cuda and F.is_contiguous() and F.numel() == N ** 3
        _check(lib().frg_rhs_noalloc(self._h, float(T), _ptr(V), _ptr(F), int(prec), _stream()))
        return F

    def flow_init(self, opts: FlowOpts, V, state):
        _check(lib().frg_flow_init(self._h, C.byref(opts), _ptr(V), _ptr(state), _stream()))

    def flow_step(self, opts: FlowOpts, V, state):
        _check(lib().frg_flow_step(self._h, C.byref(opts), _ptr(V), _ptr(state), _stream()))

    def set_self_energy(self, enable: bool, symmetric: bool = False):
        """frg_set_self_energy: V and F then hold N^3 + N doubles (the self-energy after V);
        symmetric: the self-energy is C4v invariant (switch value 2)."""
        _check(lib().frg_set_self_energy(self._h, (2 if symmetric else 1) if enable else 0))

    def self_energy(self) -> bool:
        return self.self_energy_mode() != 0

    def self_energy_mode(self) -> int:
        """0 off, 1 general, 2 C4v invariant."""
        a = C.c_int32()
        _check(lib().frg_self_energy(self._h, C.byref(a)))
        return int(a.value)

    def rhs_se(self, T: float, V, S, prec=PREC_FP64):
        """(dV/dT, dS/dT) with the self-energy on (switched on here if it is not)."""
        torch = self.torch
        if not self.self_energy():
            self.set_self_energy(True)
        y = torch.cat([V.reshape(-1), S.reshape(-1)]).contiguous()
        F = torch.empty_like(y)
        _check(lib().frg_rhs(self._h, float(T), _ptr(y), _ptr(F), int(prec), _stream()))
        n3 = self.N ** 3
        return F[:n3].reshape(self.N, self.N, self.N), F[n3:]

    def set_symmetry(self, enable: bool):
        _check(lib().frg_set_symmetry(self._h, 1 if enable else 0))

    def symmetry(self):
        """(active, bubble rows computed per rhs)."""
        a, r = C.c_int32(), C.c_int32()
        _check(lib().frg_symmetry(self._h, C.byref(a), C.byref(r)))
        return bool(a.value), int(r.value)

    def set_kskip(self, enable: bool):
        _check(lib().frg_set_kskip(self._h, 1 if enable else 0))

    def set_vsym(self, enable: bool):
        _check(lib().frg_set_vsym(self._h, 1 if enable else 0))

    def vsym(self):
        """(symmetric-vertex mode on, columns computed per channel)."""
        a, n = C.c_int32(), C.c_int32()
        _check(lib().frg_vsym(self._h, C.byref(a), C.byref(n)))
        return bool(a.value), int(n.value)

    def check_vsym(self, V):
        """Largest relative deviation of V from C4v invariance."""
        d = C.c_double()
        _check(lib().frg_check_vsym(self._h, _ptr(V), C.byref(d), _stream()))
        return float(d.value)

    def kskip(self):
        """(zero-block skipping on, executed share of the dense contraction work)."""
        a, f = C.c_int32(), C.c_double()
        _check(lib().frg_kskip(self._h, C.byref(a), C.byref(f)))
        return bool(a.value), float(f.value)

    def tuning(self):
        t = Tuning()
        _check(lib().frg_get_tuning(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_tuning(self, kparts=0, sweep_rows=0, block_rows=0):
        _check(lib().frg_set_tuning(self._h, C.byref(Tuning(int(kparts), int(sweep_rows), int(block_rows)))))

    def tune(self, T, V, prec=PREC_FP64, reps=5, log_cap=256):
        """frg_tune: search and apply the launch parameters; returns (tuning, ms per
        rhs, candidate log [rows, 6])."""
        F = self.torch.empty_like(V)
        t, ms, nrow = Tuning(), C.c_double(), C.c_int32()
        log = np.zeros((log_cap, 6))
        _check(lib().frg_tune(self._h, float(T), _ptr(V), _ptr(F), int(prec), int(reps), C.byref(t),
                              C.byref(ms), log.ctypes.data_as(_DP), int(log_cap), C.byref(nrow), _stream()))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}, ms.value, log[:min(nrow.value, log_cap)]

    def profile_begin(self):
        _check(lib().frg_profile_begin(self._h))

    def profile_end(self):
        """Summed event time (ms) and launch count per kernel class since profile_begin."""
        ms = np.zeros(len(KERNEL_CLASSES))
        cnt = np.zeros(len(KERNEL_CLASSES), dtype=np.int32)
        _check(lib().frg_profile_end(self._h, ms.ctypes.data_as(_DP), cnt.ctypes.data_as(_IP)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def flow(self, V, opts: FlowOpts, log_cap=4096):
        """Run a whole flow in place on V; returns (result dict, log [accepted, 8])."""
        torch = self.torch
        log = torch.zeros((max(log_cap, 1), 8), dtype=torch.float64, device="cuda")
        r = FlowResult()
        st = lib().frg_flow(self._h, C.byref(opts), _ptr(V), _ptr(log), int(log_cap), C.byref(r),
                            _stream())
        res = {k: getattr(r, k) for k, _ in FlowResult._fields_}
        if st not in (OK, ENONFINITE):
            _check(st)
        torch.cuda.synchronize()
        n = min(res["accepted"], log_cap)
        return res, log[:n].cpu().numpy()


class Batch:
    """Independent flows (different parameters, uneven N, same n_rad x n_ang) run together."""

    def __init__(self, param_dicts):
        import torch
        self.torch = torch
        self.params = [dict(p) for p in param_dicts]
        n = len(self.params)
        arr = (Params * n)(*[params(**p) for p in self.params])
        h = _P()
        _check(lib().frg_batch_create(arr, n, C.byref(h)))
        self._h = h
        self.n = n
        self.Ns = [int(p["N"]) for p in self.params]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().frg_batch_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, tensors):
        arr = (C.c_void_p * self.n)(*[t.data_ptr() for t in tensors])
        return arr

    def rhs(self, Ts, Vs, prec=PREC_FP64):
        torch = self.torch
        Fs = [torch.empty_like(V) for V in Vs]
        T = np.ascontiguousarray(Ts, dtype=np.float64)
        _check(lib().frg_batch_rhs(self._h, T.ctypes.data_as(_DP), self._ptrs(Vs), self._ptrs(Fs),
                                   int(prec), _stream()))
        return Fs

    def set_vsym(self, enable: bool):
        """Symmetric-vertex mode for every flow (flow_init again afterwards)."""
        _check(lib().frg_batch_set_vsym(self._h, 1 if enable else 0))

    def symmetry(self):
        """(active, bubble rows per rhs) of every member."""
        out = []
        for i in range(self.n):
            h = _P()
            _check(lib().frg_batch_context(self._h, i, C.byref(h)))
            a, r = C.c_int32(), C.c_int32()
            _check(lib().frg_symmetry(h, C.byref(a), C.byref(r)))
            out.append((bool(a.value), int(r.value)))
        return out

    def flow_init(self, Vs, opts: FlowOpts):
        self._keep = (list(Vs), opts)
        _check(lib().frg_batch_flow_init(self._h, C.byref(opts), self._ptrs(Vs), None, 0, _stream()))

    def flow_step(self):
        _check(lib().frg_batch_flow_step(self._h, _stream()))

    def set_tuning(self, kparts=0, sweep_rows=0, block_rows=0):
        """One tuning for every member (flow_init again afterwards)."""
        _check(lib().frg_batch_set_tuning(self._h, C.byref(Tuning(int(kparts), int(sweep_rows), int(block_rows)))))

    def tune(self, Ts, Vs, prec=PREC_FP64, reps=3, log_cap=256):
        """frg_batch_tune on the batched rhs; returns (tuning, ms per batched rhs,
        candidate log [rows, 6])."""
        Fs = [self.torch.empty_like(V) for V in Vs]
        T = np.ascontiguousarray(Ts, dtype=np.float64)
        t, ms, nrow = Tuning(), C.c_double(), C.c_int32()
        log = np.zeros((log_cap, 6))
        _check(lib().frg_batch_tune(self._h, T.ctypes.data_as(_DP), self._ptrs(Vs), self._ptrs(Fs), int(prec),
                                    int(reps), C.byref(t), C.byref(ms), log.ctypes.data_as(_DP), int(log_cap),
                                    C.byref(nrow), _stream()))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}, ms.value, log[:min(nrow.value, log_cap)]

    def profile_begin(self):
        _check(lib().frg_batch_profile_begin(self._h))

    def profile_end(self):
        """Summed event time (ms) and launch count per kernel class since profile_begin."""
        ms = np.zeros(len(KERNEL_CLASSES))
        cnt = np.zeros(len(KERNEL_CLASSES), dtype=np.int32)
        _check(lib().frg_batch_profile_end(self._h, ms.ctypes.data_as(_DP), cnt.ctypes.data_as(_IP)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def results(self):
        res = (FlowResult * self.n)()
        allst = C.c_int32()
        st = lib().frg_batch_results(self._h, res, C.byref(allst))
        if st not in (OK, ENONFINITE):
            _check(st)
        return [{k: getattr(r, k) for k, _ in FlowResult._fields_} for r in res], bool(allst.value)

    def flow(self, Vs, opts: FlowOpts, log_cap=0):
        """Run all flows in place on Vs; returns (list of result dicts, log or None)."""
        torch = self.torch
        log = (torch.zeros((self.n, log_cap, 8), dtype=torch.float64, device="cuda")
               if log_cap > 0 else None)
        res = (FlowResult * self.n)()
        st = lib().frg_batch_flow(self._h, C.byref(opts), self._ptrs(Vs), _ptr(log), int(log_cap),
                                  res, _stream())
        if st not in (OK, ENONFINITE):
            _check(st)
        torch.cuda.synchronize()
        out = [{k: getattr(r, k) for k, _ in FlowResult._fields_} for r in res]
        return out, (log.cpu().numpy() if log is not None else None)


def T_of_s(s: float) -> float:
    return math.exp(s)
