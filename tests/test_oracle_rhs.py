"""Pins of the oracle's bubble tensors, rhs and steppers (no GPU).

Eq. (1) of the paper is an explicit ODE whose rhs is evaluated with V frozen;
Sec. 4 makes it three one-loop diagrams over the Brillouin zone and reports
seven rhs evaluations in the first step.  The pins: binning conserves the
unbinned sum, exact symmetries, the second-order identity for constant V,
brute force without bubble tensors, and textbook ODE cases.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1510_07799_amd import inputs as I


@pytest.fixture(scope="module")
def m8():
    return O.Model(t=1, tp=-0.2, mu=-0.5, U=2.0, N=8, n_rad=5, n_ang=3)


@pytest.fixture(scope="module")
def m16():
    return O.Model(**I.model_params("C1"))


def _second_line_energy(m, tb, kind, t, p):
    """eps at q - p (pp) or p + Q (ph), straight from the dispersion in numpy."""
    t_, tp, mu = m.params["t"], m.params["tp"], m.params["mu"]
    if kind == O.PP:
        kx, ky = tb["qpp"][t, 0] - tb["px"][p], tb["qpp"][t, 1] - tb["py"][p]
    else:
        kx, ky = tb["px"][p] + tb["qph"][t, 0], tb["py"][p] + tb["qph"][t, 1]
    cx, cy = math.cos(kx), math.cos(ky)
    return -2 * t_ * (cx + cy) - 4 * tp * cx * cy - mu


@pytest.mark.parametrize("deriv", [0, 1])
def test_binning_conserves_the_sum(m8, deriv):
    """sum_b B_t(a,b) = sum_{p in a} w_p L(xi_p, eps(second line))."""
    T = 0.13
    tb = m8.tables(idx4=False)
    Bpp, Bph = m8.bubbles(T, deriv)
    N, nf = m8.N, m8.nf
    for kind, B in ((O.PP, Bpp), (O.PH, Bph)):
        for t in range(0, B.shape[0], 5):
            for a in range(N):
                ref = 0.0
                for k in range(nf):
                    p = a * nf + k
                    ref += tb["w"][p] * O.L(kind, deriv, tb["xi"][p],
                                            _second_line_energy(m8, tb, kind, t, p), T)
                assert B[t, a].sum() == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_bins_match_projection(m8):
    tb = m8.tables(idx4=False)
    bins = m8.bins(O.PH)
    for t in range(0, m8.Tph, 7):
        for p in range(0, m8.N * m8.nf, 5):
            kx = O.fold(tb["px"][p] + tb["qph"][t, 0])
            ky = O.fold(tb["py"][p] + tb["qph"][t, 1])
            assert bins[t, p] == m8.project(kx, ky)


def test_zero_transfer_row_is_diagonal(m16):
    Bpp, Bph = m16.bubbles(0.2)
    B0 = Bph[0]
    assert np.count_nonzero(B0 - np.diag(np.diag(B0))) == 0
    assert np.all(np.diag(B0) != 0)


def test_bubbles_c4v_covariant(m16):
    """B_{g t}(g a, g b) = B_t(a, b) on the bitwise C4v-symmetric grid."""
    N = m16.N
    Bpp, Bph = m16.bubbles(0.1)
    scale = max(np.abs(Bpp).max(), np.abs(Bph).max())
    for o in range(1, 8):
        g = I.c4v_patch_perm(N, o)
        for i in range(N):
            for j in range(N):
                t, gt = m16.row_pp(i, j), m16.row_pp(g[i], g[j])
                d = np.abs(Bpp[gt][np.ix_(g, g)] - Bpp[t]).max()
                assert d <= 1e-13 * scale
                t, gt = m16.row_ph(i, j), m16.row_ph(g[i], g[j])
                d = np.abs(Bph[gt][np.ix_(g, g)] - Bph[t]).max()
                assert d <= 1e-13 * scale


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_rhs_is_quadratic(m8):
    V = I.random_vertex(8, 2.0, seed=1, symmetrise=False)
    W = I.random_vertex(8, 1.0, seed=2, symmetrise=False)
    T = 0.2
    F = m8.rhs(T, V)
    assert _rel(m8.rhs(T, 1.7 * V), 1.7 ** 2 * F) < 1e-13
    lhs = m8.rhs(T, V + W) + m8.rhs(T, V - W)
    rhs = 2 * F + 2 * m8.rhs(T, W)
    assert _rel(lhs, rhs) < 1e-12


def test_constant_vertex_is_second_order(m16):
    """V = c: F = c^2 [ -sum_ab Bpp_q + sum_ab Bph_Qc ]; the direct ph channel
    cancels (-2 + 1 + 1 = 0)."""
    N, c, T = m16.N, 1.7, 0.15
    Bpp, Bph = m16.bubbles(T)
    F = m16.rhs(T, np.full((N, N, N), c))
    ref = np.zeros((N, N, N))
    for j1 in range(N):
        for j2 in range(N):
            for j3 in range(N):
                ref[j1, j2, j3] = c * c * (-Bpp[m16.row_pp(j1, j2)].sum()
                                           + Bph[m16.row_ph(j3, j2)].sum())
    assert _rel(F, ref) < 1e-13


@pytest.mark.parametrize("N,nr,na", [(4, 3, 2), (8, 4, 3)])
def test_binned_equals_brute_force(N, nr, na):
    m = O.Model(t=1, tp=-0.15, mu=-0.3, U=2.0, N=N, n_rad=nr, n_ang=na)
    V = I.random_vertex(N, 2.0, seed=5, symmetrise=False)
    T = 0.11
    F = m.rhs(T, V)
    idx = np.array([(a, b, c) for a in range(N) for b in range(N) for c in range(N)], np.int32)
    Fb = m.rhs_entries(T, V, idx).reshape(N, N, N)
    assert _rel(Fb, F) < 1e-13


def test_brute_force_sampled_production_grid():
    m = O.Model(**I.model_params("C2"))
    V = I.random_vertex(m.N, 3.0, seed=8)
    T = 0.07
    F = m.rhs(T, V)
    idx = I.random_entries(m.N, 40, seed=9)
    Fb = m.rhs_entries(T, V, idx)
    Fs = F[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.abs(Fb - Fs).max() < 1e-12 * np.abs(F).max()


def test_rhs_c4v_equivariant(m16):
    N = m16.N
    V = I.random_vertex(N, 2.0, seed=3, symmetrise=True)
    F = m16.rhs(0.1, V)
    for o in range(8):
        g = I.c4v_patch_perm(N, o)
        assert np.abs(F[np.ix_(g, g, g)] - F).max() <= 1e-13 * np.abs(F).max()


def test_crossing_and_time_reversal_subsets(m16):
    """For V = U, F obeys V(k1,k2,k1) = V(k2,k1,k2) (crossing with k3 = k1) and
    V(k1,k2,k2) = V(k2,k1,k1) (time reversal with k3 = k2), where k4 is exactly
    a patch centre."""
    N = m16.N
    F = m16.rhs(0.1, np.full((N, N, N), 2.0))
    s = np.abs(F).max()
    for j1 in range(N):
        for j2 in range(N):
            assert abs(F[j1, j2, j1] - F[j2, j1, j2]) <= 1e-13 * s
            assert abs(F[j1, j2, j2] - F[j2, j1, j1]) <= 1e-13 * s


# ----------------------------------------------------------------- steppers
def test_rk4_riccati_and_order():
    c, y0 = 0.7, 1.3
    exact = lambda s: y0 / (1 + c * y0 * s)
    errs = []
    for n in (10, 20, 40):
        y, r = O.rk4(lambda s, y: -c * y * y, [y0], 0.0, 2.0, n)
        errs.append(abs(y[0] - exact(2.0)))
        assert r["rhs_evals"] == 4 * n
    p1, p2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 3.8 < p1 < 4.3 and 3.8 < p2 < 4.3


def test_dp54_riccati_accuracy_and_first_step():
    c, y0 = 0.7, 1.3
    exact = lambda s: y0 / (1 + c * y0 * s)
    y, r, log = O.dp54(lambda s, y: -c * y * y, [y0], 0.0, 3.0, 0.01, 1e-10, 1e-12, 1e9)
    assert abs(y[0] - exact(3.0)) < 1e-8
    assert r["reason"] == O.STOP_TMIN and r["s_end"] == 3.0
    # seven rhs evaluations in the first step (FSAL), as the paper reports
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
    assert r["first_step_rhs"] == golden["rhs_evals_first_step"]["value"] == 7


def test_dp54_local_order_five():
    """One accepted step of size h: local error ~ h^6 (a wrong coefficient drops
    the exponent to 5 or less)."""
    c, y0 = 0.7, 1.3
    exact = lambda s: y0 / (1 + c * y0 * s)
    errs = []
    for h in (0.1, 0.05, 0.025):
        y, r, _ = O.dp54(lambda s, y: -c * y * y, [y0], 0.0, h, h, 1e6, 1e6, 1e9)
        assert r["accepted"] == 1
        errs.append(abs(y[0] - exact(h)))
    p1, p2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 5.6 < p1 < 7.5 and 5.6 < p2 < 7.5


def test_dp54_stop_conditions():
    # divergence: y' = y^2 blows up at s = 1/y0
    y, r, log = O.dp54(lambda s, y: y * y, [1.0], 0.0, 5.0, 0.01, 1e-8, 1e-12, 20.0)
    assert r["reason"] == O.STOP_DIVERGED
    assert 0.95 < r["s_c"] < 1.0 and y[0] > 20.0          # y = 1/(1-s) passes 20 at s = 0.95
    assert 0.9 < r["s_c_interp"] <= r["s_c"]
    # max steps
    y, r, log = O.dp54(lambda s, y: -y, [1.0], 0.0, 50.0, 0.01, 1e-8, 1e-12, 1e9, max_steps=3)
    assert r["reason"] == O.STOP_MAXSTEPS and r["accepted"] == 3
    # non-finite state
    y, r, log = O.dp54(lambda s, y: np.full_like(y, np.nan), [1.0], 0.0, 1.0, 0.01, 1e-8, 1e-12, 1e9)
    assert r["reason"] == O.STOP_NONFINITE
    # rejections happen and are counted when the first step is far too large
    y, r, log = O.dp54(lambda s, y: -50 * y, [1.0], 0.0, 1.0, 0.9, 1e-10, 1e-14, 1e9)
    assert r["rejected"] >= 1 and r["reason"] == O.STOP_TMIN


def test_flow_downward_in_log_T(m16):
    """The C1 flow (RK4, T 1 -> 0.05) diverges at T_c inside the window; DP5(4)
    finds the same crossing."""
    V1, r1, _ = m16.flow(stepper="rk4", fixed_steps=40, T_min=0.05, vmax=20.0)
    V2, r2, _ = m16.flow(stepper="dp54", T_min=0.05, rtol=1e-8, vmax=20.0)
    assert r1["reason"] == O.STOP_DIVERGED and r2["reason"] == O.STOP_DIVERGED
    Tc1, Tc2 = math.exp(r1["s_c_interp"]), math.exp(r2["s_c_interp"])
    assert 0.05 < Tc2 < 0.2
    assert abs(Tc1 - Tc2) < 0.01 * Tc2


def test_small_U_scaling():
    """V(T) - [U + U^2 (K(T) - K(T0))] = O(U^3): halving U divides it by ~8.
    K is the constant-vertex second-order kernel built from the L (not dL/dT)
    bubbles, so this checks the flow integration against the integrated bubbles."""
    N, T0, T1 = 8, 1.0, 0.25
    m = O.Model(t=1, tp=-0.1, mu=-0.2, U=1.0, N=N, n_rad=4, n_ang=3)

    def K(T):
        Bpp, Bph = m.bubbles(T, deriv=0)
        out = np.zeros((N, N, N))
        for j1 in range(N):
            for j2 in range(N):
                for j3 in range(N):
                    out[j1, j2, j3] = -Bpp[m.row_pp(j1, j2)].sum() + Bph[m.row_ph(j3, j2)].sum()
        return out

    dK = K(T1) - K(T0)
    res = []
    for U in (0.2, 0.1, 0.05):
        V, r, _ = m.flow(V0=np.full((N, N, N), U), stepper="dp54", T0=T0, T_min=T1,
                         rtol=1e-11, atol=1e-14, vmax=1e9)
        assert r["reason"] == O.STOP_TMIN
        res.append(np.abs(V - (U + U * U * dK)).max())
    assert 7.0 < res[0] / res[1] < 9.0
    assert 7.0 < res[1] / res[2] < 9.0
