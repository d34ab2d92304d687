"""Pins of the oracle's interaction flow (no GPU).

Sec. 4's working example flows in the bare interaction at fixed temperature:
dV/dg has the three one-loop channels of the temperature flow with the full
bubble L_T in place of dL/dT, and the bubbles do not depend on g.  The pins:
the full bubbles are the T-antiderivative of the derivative bubbles (which the
brute-force and Matsubara pins of the temperature flow already fix), the
second-order identity for a constant vertex, the U^3 scaling of the flow's
deviation from second order, and RK4's order against DP5(4).
"""
import numpy as np
import pytest

import oracle as O


def _rel(x, ref):
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def m8():
    return O.Model(t=1, tp=-0.01, mu=-0.02, U=1.0, N=8, n_rad=4, n_ang=3)


def _K(m, T):
    """Constant-vertex kernel: -sum_ab Bpp_L(q) + sum_ab Bph_L(Qc) per entry."""
    N = m.N
    Bpp, Bph = m.bubbles(T, deriv=0)
    out = np.zeros((N, N, N))
    for j1 in range(N):
        for j2 in range(N):
            for j3 in range(N):
                out[j1, j2, j3] = -Bpp[m.row_pp(j1, j2)].sum() + Bph[m.row_ph(j3, j2)].sum()
    return out


def test_full_bubbles_are_the_T_antiderivative(m8):
    """(B_L(T + d) - B_L(T - d)) / 2d = B_dL/dT(T) to the O(d^2) of the difference."""
    T, d = 0.1, 1e-4
    up, dn, der = m8.bubbles(T + d, 0), m8.bubbles(T - d, 0), m8.bubbles(T, 1)
    for k in range(2):
        fd = (up[k] - dn[k]) / (2 * d)
        assert _rel(fd, der[k]) < 1e-6


def test_full_rhs_constant_vertex_is_second_order(m8):
    """V = c: dV/dg = c^2 [ -sum_ab Bpp_L + sum_ab Bph_L ]; the direct ph channel cancels."""
    N, c, T = m8.N, 1.3, 0.1
    F = m8.rhs_full(T, np.full((N, N, N), c))
    assert _rel(F, c * c * _K(m8, T)) < 1e-13


def test_iflow_deviation_from_second_order_scales_as_U_cubed(m8):
    """V(g = 1) - [U + U^2 K_L] = O(U^3): halving U divides it by ~8."""
    N, T = m8.N, 0.1
    K = _K(m8, T)
    res = []
    for U in (0.2, 0.1, 0.05):
        V, r, _ = m8.iflow(T, V0=np.full((N, N, N), U), stepper="dp54", rtol=1e-11, atol=1e-14, vmax=1e9)
        assert r["reason"] == O.STOP_TMIN and r["s_end"] == 1.0
        res.append(np.abs(V - (U + U * U * K)).max())
    assert 7.0 < res[0] / res[1] < 9.0
    assert 7.0 < res[1] / res[2] < 9.0


def test_iflow_rk4_is_fourth_order_in_g(m8):
    """Fixed-step RK4 against a tight DP5(4) solution: doubling the steps
    divides the error by ~16 (the flow is smooth at U = 1, g in [0, 1])."""
    T = 0.1
    ref, r, _ = m8.iflow(T, stepper="dp54", rtol=1e-12, atol=1e-15, vmax=1e9)
    assert r["reason"] == O.STOP_TMIN
    errs = []
    for n in (8, 16):
        V, r4, _ = m8.iflow(T, stepper="rk4", fixed_steps=n, vmax=1e9)
        assert r4["reason"] == O.STOP_TMIN and r4["rhs_evals"] == 4 * n
        errs.append(np.abs(V - ref).max())
    assert 12.0 < errs[0] / errs[1] < 20.0


def test_paper_example_diverges_before_full_interaction():
    """The working example (t' = -0.01, mu = -0.02, T = 0.1) close to van Hove
    filling: at U = 2 the one-loop flow leaves any bound before g = 1 (here
    checked on a small grid; the exact g_c is grid dependent and unpinned)."""
    m = O.Model(t=1, tp=-0.01, mu=-0.02, U=2.0, N=16, n_rad=8, n_ang=8)
    _, r, _ = m.iflow(0.1, stepper="dp54", vmax=20.0)
    assert r["reason"] == O.STOP_DIVERGED
    assert 0.0 < r["s_c_interp"] < 1.0
