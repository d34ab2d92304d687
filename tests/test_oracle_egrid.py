"""Pins of the oracle's energy-angle quadrature (no GPU).

The paper integrates over the Brillouin zone with an outer fixed midpoint grid
in energy and an inner locally adaptive midpoint rule along each energy (Sec. 4).
The oracle's version of it (one point list per patch sector, weights as the
quadrature gives them) is checked here against facts that do not come from the
oracle:

  * the density of states of the nearest-neighbour band at mu = 0 in closed form,
    K(1 - (E/4t)^2) / (2 pi^2 t) with K the complete elliptic integral (scipy);
  * for t' != 0, the density of states and the shell areas from an independent
    slicing of the zone at fixed kx (for |t'| < t/2 the band rises with |ky| at
    fixed kx, so each slice below energy E is one interval in closed form),
    integrated with scipy's adaptive quadrature;
  * the zone's normalised area (sum of the weights -> 1, error shrinking linearly
    with the energy spacing, which is what the midpoint rule gives across the
    logarithmic van Hove singularity) and the band moments <eps> = -mu and
    <eps^2> = 4t^2 + 4t'^2 + mu^2;
  * every point lies on its shell's energy; C4v images carry equal weights;
    a tighter target puts more points where the density of the contour varies.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import ellipk

import oracle as O


def grid(t=1.0, tp=0.0, mu=0.0, N=32, n_E=64, max_level=5, rtol=1e-4):
    m = O.Model(t=t, tp=tp, mu=mu, U=2.0, N=N, egrid=dict(n_E=n_E, max_level=max_level, rtol=rtol))
    tb = m.tables(idx4=False)
    Emin = -4.0 * t - 4.0 * tp - mu
    Emax = 4.0 * t - 4.0 * tp - mu
    return m, tb, Emin, (Emax - Emin) / n_E


def shells(tb, Emin, dE, n_E):
    """per-shell weight sums, grouped by the points' energies"""
    w, xi = tb["w"], tb["xi"]
    live = w > 0
    sh = np.floor((xi[live] - Emin) / dE).astype(int)
    assert sh.min() >= 0 and sh.max() < n_E
    return np.bincount(sh, weights=w[live], minlength=n_E)


def _slice_edges(E, t, tp, mu):
    """the kx in (0, pi) where u = +-1 (the slice's interval closes or fills the zone)"""
    out = []
    for c in ((-E - mu - 2.0 * t) / (2.0 * t + 4.0 * tp), (E + mu - 2.0 * t) / (4.0 * tp - 2.0 * t)):
        if -1.0 < c < 1.0:
            out.append(math.acos(c))
    return sorted(out)


def slice_dos(E, t, tp, mu):
    """rho(E) by slicing at fixed kx: at fixed kx, eps < E on |ky| < arccos(u),
    u = (-E - mu - 2t cos kx) / (2t + 4t' cos kx), so d(area)/dE integrates
    1 / (sqrt(1 - u^2) (2t + 4t' cos kx)) over the kx where |u| < 1 (inverse
    square-root ends, split there so that the adaptive rule sees them at ends)."""
    def f(kx):
        a = 2.0 * t + 4.0 * tp * math.cos(kx)
        u = (-E - mu - 2.0 * t * math.cos(kx)) / a
        return 0.0 if abs(u) >= 1.0 else 1.0 / (math.sqrt(1.0 - u * u) * a)
    cuts = [0.0] + _slice_edges(E, t, tp, mu) + [math.pi]
    v = sum(integrate.quad(f, a, b, limit=400, epsabs=1e-14, epsrel=1e-12)[0] for a, b in zip(cuts, cuts[1:]))
    return 2.0 * v * 2.0 / (4.0 * math.pi ** 2)


def slice_area(E, t, tp, mu):
    """normalised area of {eps < E} by the same slicing"""
    def f(kx):
        a = 2.0 * t + 4.0 * tp * math.cos(kx)
        u = (-E - mu - 2.0 * t * math.cos(kx)) / a
        return math.acos(max(-1.0, min(1.0, u)))
    cuts = [0.0] + _slice_edges(E, t, tp, mu) + [math.pi]
    v = sum(integrate.quad(f, a, b, limit=400, epsabs=1e-15, epsrel=1e-13)[0] for a, b in zip(cuts, cuts[1:]))
    return 2.0 * 2.0 * v / (4.0 * math.pi ** 2)


def test_points_lie_on_their_shells():
    n_E = 48
    for tp, mu in ((0.0, 0.0), (-0.3, -1.2), (0.2, 0.4)):
        m, tb, Emin, dE = grid(tp=tp, mu=mu, N=24, n_E=n_E, max_level=4, rtol=1e-3)
        live = tb["w"] > 0
        xi = tb["xi"][live]
        i = np.floor((xi - Emin) / dE)
        E = Emin + (i + 0.5) * dE
        assert np.abs(xi - E).max() <= 1e-12
        # every shell is populated (the contour exists at every energy inside the band)
        assert len(np.unique(i)) == n_E
        # padding: zero weight, after every live point of its patch
        w = tb["w"].reshape(24, m.nf)
        assert (w >= 0).all() and (w == 0).any()
        cnt = (w > 0).sum(1)
        for J in range(24):
            assert (w[J, :cnt[J]] > 0).all() and (w[J, cnt[J]:] == 0).all()


def test_dos_nearest_neighbour_band_is_the_elliptic_integral():
    n_E = 64
    m, tb, Emin, dE = grid(t=1.0, N=32, n_E=n_E, max_level=6, rtol=1e-5)
    dos = shells(tb, Emin, dE, n_E) / dE
    E = Emin + (np.arange(n_E) + 0.5) * dE
    ref = ellipk(1.0 - (E / 4.0) ** 2) / (2.0 * math.pi ** 2)
    rel = np.abs(dos - ref) / ref
    far = np.abs(E) > 0.5          # away from the van Hove energy E = 0
    print("DOS rel err away from vH: max %.2e; next to vH %.2e" % (rel[far].max(), rel[~far].max()))
    assert rel[far].max() <= 2e-5
    assert rel.max() <= 2e-3
    # with t = 2 the density halves and the band doubles
    m2, tb2, Emin2, dE2 = grid(t=2.0, N=32, n_E=n_E, max_level=6, rtol=1e-5)
    dos2 = shells(tb2, Emin2, dE2, n_E) / dE2
    E2 = Emin2 + (np.arange(n_E) + 0.5) * dE2
    ref2 = ellipk(1.0 - (E2 / 8.0) ** 2) / (4.0 * math.pi ** 2)
    assert (np.abs(dos2 - ref2) / ref2)[np.abs(E2) > 1.0].max() <= 2e-5


@pytest.mark.parametrize("tp,mu", [(-0.3, -1.2), (0.2, 0.4)])
def test_dos_and_shell_areas_against_slicing(tp, mu):
    n_E, t = 40, 1.0
    m, tb, Emin, dE = grid(t=t, tp=tp, mu=mu, N=24, n_E=n_E, max_level=6, rtol=1e-5)
    got = shells(tb, Emin, dE, n_E)
    E = Emin + (np.arange(n_E) + 0.5) * dE
    dos = np.array([slice_dos(e, t, tp, mu) for e in E])
    # van Hove energies eps(pi, 0) = 4t' - mu: keep a margin of two shells
    vh = 4.0 * tp - mu
    far = np.abs(E - vh) > 2.0 * dE
    rel = np.abs(got / dE - dos) / dos
    print("t'=%g mu=%g: DOS rel err max %.2e (away from vH)" % (tp, mu, rel[far].max()))
    assert rel[far].max() <= 2e-5
    # the shell's weight is the area between its edges up to the midpoint rule's
    # O(dE^3 rho'') term: compare with the slicing's areas
    edges = Emin + np.arange(n_E + 1) * dE
    area = np.diff([slice_area(e, t, tp, mu) for e in edges])
    rel_a = np.abs(got - area) / area
    print("shell areas: max rel err %.2e" % rel_a[far].max())
    assert rel_a[far].max() <= 1e-2


def test_total_weight_converges_linearly_in_the_energy_spacing():
    defs = []
    for n_E in (32, 64, 128):
        m, tb, Emin, dE = grid(tp=-0.25, mu=-0.8, N=16, n_E=n_E, max_level=6, rtol=1e-5)
        defs.append(1.0 - tb["w"].sum())
    print("1 - sum w:", defs)
    assert 0.0 < defs[2] < defs[1] < defs[0] < 0.02
    # each halving of dE roughly halves the deficit (log singularity of the DOS)
    for a, b in zip(defs, defs[1:]):
        assert 1.5 <= a / b <= 2.6


def test_band_moments():
    """<eps> = -mu and <eps^2> = 4t^2 + 4t'^2 + mu^2 over the zone.  At mu = 4t'
    the van Hove energy is 0, where the energy midpoint rule loses weight at
    first order, so the unnormalised moments converge at second order."""
    t, tp, mu = 1.0, -0.3, -1.2
    m, tb, Emin, dE = grid(t=t, tp=tp, mu=mu, N=24, n_E=200, max_level=6, rtol=1e-5)
    w, xi = tb["w"], tb["xi"]
    m1 = (w * xi).sum()
    m2 = (w * xi * xi).sum()
    print("moments", w.sum(), m1, m2)
    assert abs(m1 - (-mu)) <= 3e-4
    assert abs(m2 - (4 * t * t + 4 * tp * tp + mu * mu)) <= 3e-4


def test_c4v_images_carry_equal_weights():
    N = 32
    m, tb, Emin, dE = grid(tp=-0.3, mu=-1.2, N=N, n_E=24, max_level=4, rtol=1e-4)
    nf = m.nf
    w = tb["w"].reshape(N, nf)
    px, py = tb["px"].reshape(N, nf), tb["py"].reshape(N, nf)
    wdg = N // 8
    for J in range(N):
        o, r = divmod(J, wdg)
        src = r if o % 2 == 0 else wdg - 1 - r
        assert np.array_equal(np.sort(w[J]), np.sort(w[src]))
        # radii agree exactly up to the rotation's rounding
        rJ = np.sort(np.hypot(px[J], py[J]))
        rs = np.sort(np.hypot(px[src], py[src]))
        assert np.abs(rJ - rs).max() <= 1e-13


def test_a_tighter_target_refines_where_the_contour_density_varies():
    """On the shell next to the van Hove energy of the nearest-neighbour band the
    contour passes close to the saddle (pi, 0): the sector holding that direction
    takes more points than its neighbour, and the shell's density of states
    follows the target (error about rtol / 3)."""
    E = -4.0 + 15.5 * 0.25
    ref = ellipk(1.0 - (E / 4.0) ** 2) / (2.0 * math.pi ** 2)
    prev = None
    for rtol in (1e-3, 1e-4, 1e-5):
        m, tb, Emin, dE = grid(tp=0.0, mu=0.0, N=16, n_E=32, max_level=8, rtol=rtol)
        on = (np.abs(tb["xi"] - E) < 1e-9) & (tb["w"] > 0)
        cnt = on.reshape(16, -1).sum(1)
        err = abs(tb["w"][on].sum() / dE - ref) / ref
        print("rtol %g: points in sectors 0, 1: %s, DOS err %.2e" % (rtol, cnt[:2], err))
        assert cnt[0] > cnt[1]
        assert err <= rtol
        if prev is not None:
            assert cnt.sum() > prev
        prev = cnt.sum()


def test_arguments_checked():
    for bad in (dict(n_E=0, max_level=3, rtol=1e-3), dict(n_E=8, max_level=0, rtol=1e-3),
                dict(n_E=8, max_level=13, rtol=1e-3), dict(n_E=8, max_level=3, rtol=0.0)):
        with pytest.raises(ValueError):
            O.Model(N=16, egrid=bad)
    with pytest.raises(ValueError):
        O.Model(t=1.0, tp=0.5, N=16, egrid=dict(n_E=8, max_level=3, rtol=1e-3))
