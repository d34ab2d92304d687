"""Pins of the oracle's bubble integrands against the mathematics (no GPU).

The paper (Sec. 4) names the three one-loop diagrams but prints no formula;
the integrands are the static, zero-frequency Matsubara sums of two free
propagators.  They are pinned here against the sums themselves, against
finite differences in T, and against textbook special values.
"""
import math

import numpy as np
import pytest
from scipy.special import expit, polygamma

import oracle as O


def matsubara(kind, xi1, xi2, T, M=400_000):
    """-T sum_n G(iw,xi1) G(iw,xi2) (ph) or T sum_n G(iw,xi1) G(-iw,xi2) (pp),
    with G(iw, xi) = 1/(iw - xi), n in [-M, M), plus the 1/w^2 tail."""
    n = np.arange(-M, M, dtype=np.float64)
    w = (2.0 * n + 1.0) * math.pi * T
    if kind == O.PH:
        z = (1j * w - xi1) * (1j * w - xi2)
        s = -T * np.sum(1.0 / z).real
    else:
        z = (1j * w - xi1) * (-1j * w - xi2)
        s = T * np.sum(1.0 / z).real
    tail = polygamma(1, M + 0.5) / (2.0 * math.pi ** 2 * T)
    return s + tail


def fermi(x, T):
    return expit(-x / T)


CASES = [(0.3, -0.7, 0.5), (1.2, 1.25, 0.2), (-0.4, 0.9, 1.0), (0.05, 0.05, 0.1),
         (2.0, -2.0, 0.3), (0.0, 0.6, 0.25)]


@pytest.mark.parametrize("xi1,xi2,T", CASES)
@pytest.mark.parametrize("kind", [O.PH, O.PP])
def test_L_equals_matsubara_sum(kind, xi1, xi2, T):
    ref = matsubara(kind, xi1, xi2, T)
    got = O.L(kind, 0, xi1, xi2, T)
    assert got == pytest.approx(ref, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("xi1,xi2,T", CASES + [(0.3, 0.3 + 1e-5, 0.05), (-1.0, 1.0 + 2e-6, 0.4)])
@pytest.mark.parametrize("kind", [O.PH, O.PP])
def test_Ldot_is_T_derivative(kind, xi1, xi2, T):
    """Richardson-extrapolated central difference of L in T."""
    def D(h):
        return (O.L(kind, 0, xi1, xi2, T + h) - O.L(kind, 0, xi1, xi2, T - h)) / (2 * h)
    h = 1e-3 * T
    fd = (4 * D(h / 2) - D(h)) / 3
    got = O.L(kind, 1, xi1, xi2, T)
    assert got == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_Ldot_matches_matsubara_difference():
    """dL/dT from the Matsubara sums themselves (independent of the closed form)."""
    for kind in (O.PH, O.PP):
        xi1, xi2, T = 0.35, -0.2, 0.4
        h = 1e-3
        fd = (matsubara(kind, xi1, xi2, T + h) - matsubara(kind, xi1, xi2, T - h)) / (2 * h)
        assert O.L(kind, 1, xi1, xi2, T) == pytest.approx(fd, rel=1e-5)


@pytest.mark.parametrize("xi,T", [(0.0, 0.1), (0.3, 0.2), (-0.7, 0.05), (1.5, 1.0)])
def test_special_values(xi, T):
    f = fermi(xi, T)
    # L_ph(xi, xi) = L_pp(xi, -xi) = f(1-f)/T = -df/dxi
    assert O.L(O.PH, 0, xi, xi, T) == pytest.approx(f * (1 - f) / T, rel=1e-12)
    assert O.L(O.PP, 0, xi, -xi, T) == pytest.approx(f * (1 - f) / T, rel=1e-12)
    if xi != 0.0:
        # nesting identity: L_ph(xi,-xi) = L_pp(xi,xi) = tanh(xi/2T)/(2 xi)
        ref = math.tanh(xi / (2 * T)) / (2 * xi)
        assert O.L(O.PH, 0, xi, -xi, T) == pytest.approx(ref, rel=1e-12)
        assert O.L(O.PP, 0, xi, xi, T) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("xi1,xi2,T", [(0.3, -0.8, 0.2), (1.1, 0.4, 0.07), (-2.0, 0.5, 1.0)])
def test_fermi_function_forms(xi1, xi2, T):
    f1, f2 = fermi(xi1, T), fermi(xi2, T)
    assert O.L(O.PH, 0, xi1, xi2, T) == pytest.approx((f1 - f2) / (xi2 - xi1), rel=1e-12)
    assert O.L(O.PP, 0, xi1, xi2, T) == pytest.approx((1 - f1 - f2) / (xi1 + xi2), rel=1e-12)


def test_symmetric_in_energies():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b = rng.uniform(-3, 3, 2)
        T = rng.uniform(0.01, 1)
        for kind in (O.PH, O.PP):
            for d in (0, 1):
                assert O.L(kind, d, a, b, T) == pytest.approx(O.L(kind, d, b, a, T), rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("kind", [O.PH, O.PP])
def test_taylor_branch_is_continuous(kind):
    """Values just inside and outside the Taylor window agree (same function)."""
    T = 0.1
    xi1 = 0.37
    sgn = 1.0 if kind == O.PH else -1.0
    for deriv in (0, 1):
        inside = O.L(kind, deriv, xi1, sgn * (xi1 - 2 * T * 1.999e-3), T)
        outside = O.L(kind, deriv, xi1, sgn * (xi1 - 2 * T * 2.001e-3), T)
        assert inside == pytest.approx(outside, rel=1e-5)


def test_no_overflow_at_low_T():
    """|xi|/2T ~ 4000 must not overflow (sech^2 and tanh from exp(-2|x|))."""
    for kind in (O.PH, O.PP):
        for d in (0, 1):
            v = O.L(kind, d, 8.0, -7.9, 1e-3)
            assert np.isfinite(v)
            v = O.L(kind, d, 8.0, 8.0, 1e-3)
            assert np.isfinite(v)
    # far from the Fermi surface with equal signs the ph bubble vanishes
    assert abs(O.L(O.PH, 0, 3.0, 3.5, 1e-3)) < 1e-300
    # opposite signs: L_ph -> 1/(xi1 - xi2) * ... = 1/|xi1 - xi2| at T -> 0
    assert O.L(O.PH, 0, 3.0, -3.5, 1e-3) == pytest.approx(1.0 / 6.5, rel=1e-12)
