"""Pins of the oracle's self-energy extension (no GPU).

The paper restricts itself to the four-point function and names self-energies
as the straightforward extension (Sec. 2); the reading built here is a static
self-energy S_j per patch that every loop line carries, flowing by the
one-loop tadpole with the temperature derivative of the occupation.  Pinned
against facts outside the oracle's own code:

  * the spin sum written out: the generic tadpole of the antisymmetrised spinful
    vertex built from V (explicit sums over both spins, Kronecker deltas), with
    the occupation derivative from finite differences of n_F, equals the
    oracle's SU(2) form for a vertex without crossing symmetry;
  * at V = U and a uniform shift s, dS/dT is U times the temperature derivative
    of the density per spin, integrated against the closed-form density of
    states of the nearest-neighbour band (complete elliptic integral, scipy);
  * the binned rhs with a random self-energy equals the brute-force per-entry
    sum (its own projection and shift of every second line);
  * S = 0 gives the vertex flow bit for bit;
  * at small U a flow of (V, S) from T = 1 gives S(T) = U (n(T) - n(1)) up to
    O(U^2), n the density per spin summed from the grid's own points.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import ellipk

import oracle as O
from paper_1510_07799_amd import inputs as I


def occupation(x, T):
    """Fermi function n_F(x / T), written through tanh (no overflow)"""
    return 0.5 * (1.0 - np.tanh(x / (2.0 * T)))


def test_zero_self_energy_is_the_vertex_rhs():
    m = O.Model(t=1.0, tp=-0.2, mu=-0.5, U=2.0, N=8, n_rad=6, n_ang=5)
    V = I.random_vertex(8, 2.0, seed=501, amp=0.3, symmetrise=False)
    F0 = m.rhs(0.2, V)
    F, dS = m.rhs_se(0.2, V, np.zeros(8))
    assert np.array_equal(F, F0)
    B0 = m.bubbles(0.3)
    B = m.bubbles_se(0.3, np.zeros(8))
    assert np.array_equal(B[0], B0[0]) and np.array_equal(B[1], B0[1])


def test_tadpole_is_the_spin_sum_of_the_antisymmetrised_vertex():
    N, T = 8, 0.25
    m = O.Model(t=1.0, tp=-0.25, mu=-0.7, U=2.0, N=N, n_rad=6, n_ang=5)
    tb = m.tables(idx4=False)
    rng = np.random.default_rng(502)
    V = I.random_vertex(N, 2.0, seed=503, amp=0.5, symmetrise=False)   # no crossing symmetry
    S = 0.2 * rng.standard_normal(N)
    # D_a: occupation derivative at fixed shifted energy, by central differences in T
    patch = np.arange(N * m.nf) // m.nf
    x = tb["xi"] + S[patch]
    h = 1e-5 * T
    dn = (occupation(x, T + h) - occupation(x, T - h)) / (2 * h)
    D = np.bincount(patch, weights=tb["w"] * dn, minlength=N)

    # antisymmetrised spinful vertex: G(1,2;3,4) = V(k1,k2,k3) d13 d24 - V(k2,k1,k3) d14 d23
    def gamma(k1, s1, k2, s2, k3, s3, s4):
        d = lambda a, b: 1.0 if a == b else 0.0
        return V[k1, k2, k3] * d(s1, s3) * d(s2, s4) - V[k2, k1, k3] * d(s1, s4) * d(s2, s3)

    ref = np.zeros((N, 2))
    for j in range(N):
        for s1 in range(2):
            acc = 0.0
            for a in range(N):
                for s2 in range(2):
                    # tadpole: outgoing legs equal the incoming ones, k3 = k1, k4 = k2
                    acc += gamma(j, s1, a, s2, j, s1, s2) * D[a]
            ref[j, s1] = acc
    assert np.allclose(ref[:, 0], ref[:, 1], rtol=1e-14, atol=0)   # SU(2): both spins alike
    got = m.dsigma(T, V, S)
    err = np.abs(got - ref[:, 0]).max() / np.abs(ref).max()
    print("tadpole spin sum: rel err %.2e" % err)
    assert err <= 1e-7


def test_hartree_shift_against_the_closed_form_density_of_states():
    """V = U, uniform S = s: dS/dT = U d/dT [sum_p w_p n_F((xi_p + s)/T)] for every
    patch; against U times the same derivative integrated over the closed-form
    density of states (t' = 0; xi = eps0 - mu), on the energy-angle grid.  The
    van Hove energy (xi = 1.5) sits ten T from the Fermi window: near it the
    energy midpoint rule is first order, and its share decays as sech^2."""
    t, mu, U, s, T = 1.0, -1.5, 1.5, 0.1, 0.15

    def rho0(e):
        return ellipk(1.0 - (e / (4 * t)) ** 2) / (2 * math.pi ** 2 * t)

    def dn(e):
        x = e - mu + s
        return x / (4 * T * T) / math.cosh(x / (2 * T)) ** 2

    ref = U * sum(integrate.quad(lambda e: rho0(e) * dn(e), a, b, limit=400, epsabs=1e-13, epsrel=1e-11)[0]
                  for a, b in ((-4 * t, 0.0), (0.0, 4 * t)))
    errs = []
    for n_E in (200, 400, 800):
        m = O.Model(t=t, tp=0.0, mu=mu, U=U, N=16, egrid=dict(n_E=n_E, max_level=7, rtol=1e-7))
        got = m.dsigma(T, np.full((16, 16, 16), U), np.full(16, s))
        assert np.allclose(got, got[0], rtol=1e-12, atol=0)
        errs.append(abs(got[0] - ref) / abs(ref))
    print("Hartree dS/dT: closed form %.10f, rel err by n_E:" % ref, errs)
    assert errs[-1] <= 1e-4
    assert errs[2] < errs[1] < errs[0]


def test_binned_equals_brute_force_with_a_self_energy():
    N, T = 8, 0.15
    m = O.Model(t=1.0, tp=-0.2, mu=-0.6, U=2.0, N=N, n_rad=8, n_ang=6)
    rng = np.random.default_rng(504)
    V = I.random_vertex(N, 2.0, seed=505, amp=0.4, symmetrise=False)
    S = 0.3 * rng.standard_normal(N)
    F, _ = m.rhs_se(T, V, S)
    idx = np.array([(a, b, c) for a in range(N) for b in range(N) for c in range(N)], dtype=np.int32)
    bf = m.rhs_entries_se(T, V, S, idx).reshape(N, N, N)
    err = np.abs(F - bf).max() / np.abs(bf).max()
    F0 = m.rhs(T, V)
    print("binned vs brute force with S: %.2e (S moves F by %.2e)" % (err, np.abs(F - F0).max() / np.abs(F0).max()))
    assert err <= 1e-12
    assert np.abs(F - F0).max() > 1e-3 * np.abs(F0).max()


def test_small_coupling_flow_gives_the_hartree_shift():
    N, U = 8, 0.02
    m = O.Model(t=1.0, tp=-0.2, mu=-0.6, U=U, N=N, n_rad=8, n_ang=6)
    tb = m.tables(idx4=False)
    T0, T1 = 1.0, 0.1
    V, S, res, log = m.flow_se(stepper="dp54", T0=T0, T_min=T1, rtol=1e-8, atol=1e-12, vmax=20.0, h0=-0.05)
    n = lambda T: float(np.sum(tb["w"] * occupation(tb["xi"], T)))
    ref = U * (n(T1) - n(T0))
    err = np.abs(S - ref).max() / abs(ref)
    print(f"S(T={T1}) = {S.mean():.3e} (spread {np.ptp(S):.1e}); U (n(T) - n(T0)) = {ref:.3e}; rel {err:.2e}")
    assert res["reason"] == O.STOP_TMIN
    assert err <= 10 * U
