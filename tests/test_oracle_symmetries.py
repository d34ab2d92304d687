"""Pins of the oracle's channel arrangement and quadrature against facts the
oracle's own formula does not state (no GPU).

Sec. 4 of the paper reduces the couplings with the lattice, spin and
time-reversal symmetries of the Hubbard model.  The oracle computes the
SU(2)-reduced vertex V(k1,k2,k3) with three channels in a particular index
arrangement.  These tests check that arrangement against:

  * SU(2): the generic antisymmetrised one-loop equation for a spinful vertex,
    written here from scratch with explicit sums over the spins of the loop
    lines, applied to Gamma built from V; every spin component of its result
    must be the SU(2) form built from the oracle's F.
  * particle-hole symmetry at t' = 0, mu = 0 (nested Fermi surface);
  * closed-form Brillouin-zone integrals of the quadrature weights.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O

UP, DN = 0, 1
SPINS = list(itertools.product((UP, DN), repeat=4))


# ---------------------------------------------------------------- SU(2) pin
def gamma(V, o1, so1, o2, so2, i1, si1, i2, si2):
    """Antisymmetrised spinful vertex Gamma(out o1, o2; in i1, i2) of the
    SU(2)-reduced V(k1, k2, k3) (spin of k1 goes to k3, spin of k2 to k4):
    V(i1, i2, o1) d(s_i1, s_o1) d(s_i2, s_o2) - V(i2, i1, o1) d(s_i2, s_o1) d(s_i1, s_o2)."""
    g = 0.0
    if si1 == so1 and si2 == so2:
        g += V[i1, i2, o1]
    if si2 == so1 and si1 == so2:
        g -= V[i2, i1, o1]
    return g


def spinful_rhs(m, Bpp, Bph, V, o1, so1, o2, so2, i1, si1, i2, si2):
    """dGamma/dT of the generic one-loop equation for an antisymmetrised vertex,

        c_pp/2 sum PP(o1 o2; i1 i2) + c_ph [D(o1 o2; i1 i2) - D(o1 o2; i2 i1)],

    with explicit sums over the loop patches and the spins of both loop lines.
    PP: the two lines leave the (i1, i2) vertex and enter the (o1, o2) vertex;
    their total momentum is k_i1 + k_i2, the fine-grid line in patch a, the
    other in patch b, weighted by the pp bubble row of that momentum.
    D(o1 o2; i1 i2): the particle-hole loop whose transfer is k_o1 - k_i1; one
    vertex carries (i1 -> o1), the other (i2 -> o2); the line leaving the o1
    vertex is on the fine grid (patch a) and the line entering it is that line
    plus the transfer (patch b), weighted by the ph bubble row of the transfer.
    The minus sign of the exchanged term (i1 <-> i2) is antisymmetry.  The bubble
    rows are L-dot >= 0 as defined by the oracle's integrands; with them the
    textbook second order for an on-site U fixes c_pp = c_ph = -1 (checked
    below against the constant-vertex limit)."""
    N = m.N
    c_pp = c_ph = -1.0

    def pp():
        B = Bpp[m.row_pp(i1, i2)]
        s = 0.0
        for a in range(N):
            for b in range(N):
                w = B[a, b]
                if w == 0.0:
                    continue
                for sa in (UP, DN):
                    for sb in (UP, DN):
                        s += w * gamma(V, o1, so1, o2, so2, a, sa, b, sb) * \
                            gamma(V, a, sa, b, sb, i1, si1, i2, si2)
        return s

    def d(j_in, s_in, k_in, t_in):
        # loop attached to (j_in -> o1); the other vertex carries (k_in -> o2)
        B = Bph[m.row_ph(o1, j_in)]
        s = 0.0
        for a in range(N):
            for b in range(N):
                w = B[a, b]
                if w == 0.0:
                    continue
                for sx in (UP, DN):        # line b: into the o1 vertex
                    for sy in (UP, DN):    # line a: out of the o1 vertex
                        s += w * gamma(V, o1, so1, a, sy, j_in, s_in, b, sx) * \
                            gamma(V, b, sx, o2, so2, a, sy, k_in, t_in)
        return s

    return 0.5 * c_pp * pp() + c_ph * (d(i1, si1, i2, si2) - d(i2, si2, i1, si1))


def su2_form(F, o1, so1, o2, so2, i1, si1, i2, si2):
    """The SU(2) structure every spin component of dGamma/dT must have."""
    g = 0.0
    if si1 == so1 and si2 == so2:
        g += F[i1, i2, o1]
    if si2 == so1 and si1 == so2:
        g -= F[i2, i1, o1]
    return g


def test_su2_constant_vertex_gives_textbook_second_order():
    """V = U: the spinful equation gives -U^2 sum Bpp_q (Cooper screening) +
    U^2 sum Bph_{k3-k2} (spin-flip / RPA channel); the direct channel cancels."""
    m = O.Model(t=1, tp=-0.2, mu=-0.5, U=2.0, N=8, n_rad=4, n_ang=3)
    N, U, T = 8, 2.0, 0.13
    Bpp, Bph = m.bubbles(T)
    V = np.full((N, N, N), U)
    i4 = m.tables()["idx4"]
    for j1, j2, j3 in [(0, 1, 2), (3, 3, 5), (7, 2, 2), (4, 6, 1)]:
        got = spinful_rhs(m, Bpp, Bph, V, j3, UP, i4[j1, j2, j3], DN, j1, UP, j2, DN)
        ref = U * U * (-Bpp[m.row_pp(j1, j2)].sum() + Bph[m.row_ph(j3, j2)].sum())
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-15)


def test_su2_spinful_equation_exact_momentum_closure():
    """N = 4 at half filling: patch centres are (+-pi/2, +-pi/2), so k1 + k2 - k3
    folds exactly onto a centre and the crossing map (j1, j2, j3) -> (j2, j1, j4)
    is an exact involution.  For a crossing-symmetric random V the oracle's F
    is crossing symmetric too, and every spin component of the spinful one-loop
    equation equals the SU(2) form built from it (all three channels, general
    index arrangement)."""
    m = O.Model(t=1, tp=0.0, mu=0.0, U=2.0, N=4, n_rad=3, n_ang=2)
    N = 4
    i4 = m.tables()["idx4"]
    for j1, j2, j3 in itertools.product(range(N), repeat=3):
        assert i4[j2, j1, i4[j1, j2, j3]] == j3
    rng = np.random.default_rng(3)
    R = 2.0 * (1.0 + 0.5 * rng.uniform(-1.0, 1.0, (N, N, N)))
    V = np.empty_like(R)
    for j1, j2, j3 in itertools.product(range(N), repeat=3):
        V[j1, j2, j3] = 0.5 * (R[j1, j2, j3] + R[j2, j1, i4[j1, j2, j3]])
    T = 0.17
    F = m.rhs(T, V)
    Bpp, Bph = m.bubbles(T)
    scale = np.abs(F).max()
    # crossing of the result, V(k1,k2,k3) = V(k2,k1,k4), for a non-constant vertex
    for j1, j2, j3 in itertools.product(range(N), repeat=3):
        assert abs(F[j2, j1, i4[j1, j2, j3]] - F[j1, j2, j3]) <= 1e-13 * scale
    worst = 0.0
    for j1, j2, j3 in itertools.product(range(N), repeat=3):
        j4 = i4[j1, j2, j3]
        for s1, s2, s3, s4 in SPINS:
            got = spinful_rhs(m, Bpp, Bph, V, j3, s3, j4, s4, j1, s1, j2, s2)
            ref = su2_form(F, j3, s3, j4, s4, j1, s1, j2, s2)
            worst = max(worst, abs(got - ref))
    assert worst <= 1e-13 * scale


@pytest.mark.parametrize("cfg", [dict(N=8, n_rad=4, n_ang=3, tp=-0.2, mu=-0.5),
                                 dict(N=16, n_rad=4, n_ang=4, tp=-0.25, mu=-1.0)], ids=["N8", "N16"])
def test_su2_spinful_equation_general_geometry(cfg):
    """Any patch geometry: for V(k1, k2, k3) = f(k1, k2) with f symmetric (a
    vertex that depends on the incoming pair only, so that crossing holds
    exactly whatever idx4 is), the spinful equation equals the SU(2) form of the
    oracle's rhs in every spin component.  This fixes which loop line enters
    which vertex in the crossed and direct particle-hole channels."""
    m = O.Model(t=1, U=2.0, **cfg)
    N = m.N
    rng = np.random.default_rng(11 + N)
    f = rng.uniform(1.0, 3.0, (N, N))
    f = 0.5 * (f + f.T)
    V = np.ascontiguousarray(np.broadcast_to(f[:, :, None], (N, N, N)))
    T = 0.13
    F = m.rhs(T, V)
    Bpp, Bph = m.bubbles(T)
    i4 = m.tables()["idx4"]
    entries = list(itertools.product(range(N), repeat=3))
    spins = SPINS if N <= 8 else [(UP, DN, UP, DN), (UP, UP, UP, UP), (UP, DN, DN, UP)]
    if N > 8:
        entries = [entries[i] for i in rng.choice(len(entries), 48, replace=False)]
    scale = np.abs(F).max()
    worst = 0.0
    for j1, j2, j3 in entries:
        j4 = i4[j1, j2, j3]
        for s1, s2, s3, s4 in spins:
            got = spinful_rhs(m, Bpp, Bph, V, j3, s3, j4, s4, j1, s1, j2, s2)
            ref = su2_form(F, j3, s3, j4, s4, j1, s1, j2, s2)
            worst = max(worst, abs(got - ref))
    assert worst <= 1e-13 * scale


# ------------------------------------------------------- particle-hole pin
def ph_symmetric_vertex(kc, U=2.0):
    """A smooth vertex of the three transfers q = k1 + k2, k3 - k2, k3 - k1; each
    is unchanged (mod 2 pi) when every momentum is shifted by (pi, pi)."""
    K = kc
    q = K[:, None, :] + K[None, :, :]
    Qc = K[None, None, :, :] - K[None, :, None, :]
    Qd = K[None, None, :, :] - K[:, None, None, :]
    cq = (np.cos(q[..., 0]) + np.cos(q[..., 1]))[:, :, None]
    cc = np.cos(Qc[..., 0]) + np.cos(Qc[..., 1])
    cd = np.cos(Qd[..., 0]) + np.cos(Qd[..., 1])
    return np.ascontiguousarray(U + 0.4 * cq + 0.3 * cc + 0.2 * cd)


def ph_violation(N, n_rad, n_ang, T):
    m = O.Model(t=1, tp=0.0, mu=0.0, U=2.0, N=N, n_rad=n_rad, n_ang=n_ang)
    kc = m.tables(idx4=False)["kc"]
    P = np.array([m.project(O.fold(x + math.pi), O.fold(y + math.pi)) for x, y in kc])
    assert np.array_equal(P[P], np.arange(N))          # an involution on the patches
    V = ph_symmetric_vertex(kc)
    assert np.abs(V[np.ix_(P, P, P)] - V).max() <= 1e-14
    F = m.rhs(T, V)
    return np.abs(F[np.ix_(P, P, P)] - F).max() / np.abs(F).max()


def test_particle_hole_violation_shrinks_with_the_grid():
    """t' = 0, mu = 0: eps(k + (pi, pi)) = -eps(k) and both bubbles are even in
    (xi1, xi2) -> (-xi1, -xi2), so the continuum flow keeps a vertex that is
    invariant under shifting every momentum by (pi, pi).  On the patches the
    symmetry holds up to discretisation: loop lines are projected radially onto
    the Fermi surface, which commutes with the shift only on the Fermi surface.
    At low T (bubbles concentrated there) the violation shrinks as the patches
    and the fine grid are refined."""
    v = [ph_violation(N, nr, na, 0.03) for N, nr, na in ((16, 16, 16), (32, 32, 16), (32, 64, 32))]
    print("particle-hole violation at T = 0.03:", v)
    assert v[0] > v[1] > v[2]
    assert v[2] < 4e-3


# ------------------------------------------------------------ weights pin
@pytest.mark.parametrize("tp,mu", [(-0.25, -1.0), (0.0, 0.0)])
def test_weights_integrate_closed_forms(tp, mu):
    """Brillouin-zone averages with closed forms: <cos^2 kx> = 1/2,
    <cos kx cos ky> = 0, <cos^2 kx cos^2 ky> = 1/4, <eps> = -mu,
    <eps^2> = 4t^2 + 4t'^2 + mu^2, <kx^2 + ky^2> = 2 pi^2 / 3.  The polar
    midpoint rule (weight r dr dtheta / (2 pi)^2) converges at second order:
    doubling n_rad and n_ang cuts every error about fourfold."""
    exact = dict(c2=0.5, cc=0.0, c22=0.25, e1=-mu, e2=4.0 + 4.0 * tp * tp + mu * mu,
                 r2=2.0 * math.pi ** 2 / 3.0)
    errs = []
    for nr, na in ((4, 4), (8, 8), (16, 16)):
        tb = O.Model(t=1, tp=tp, mu=mu, U=2.0, N=16, n_rad=nr, n_ang=na).tables(idx4=False)
        w, px, py, xi = tb["w"], tb["px"], tb["py"], tb["xi"]
        cx, cy = np.cos(px), np.cos(py)
        got = dict(c2=(w * cx * cx).sum(), cc=(w * cx * cy).sum(), c22=(w * cx * cx * cy * cy).sum(),
                   e1=(w * xi).sum(), e2=(w * xi * xi).sum(), r2=(w * (px * px + py * py)).sum())
        errs.append({k: abs(got[k] - exact[k]) for k in exact})
    for k in exact:
        e = [x[k] for x in errs]
        if e[0] < 1e-15:
            continue
        assert 3.5 < e[0] / e[1] < 4.8 and 3.5 < e[1] / e[2] < 4.8, (k, e)
    assert errs[2]["c2"] < 1e-4 and errs[2]["r2"] < 2e-2
