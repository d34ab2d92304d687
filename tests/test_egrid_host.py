"""The library's host geometry of the energy-angle grid against the oracle's
(no device needed).

Both sides build the paper's quadrature (Sec. 4: outer midpoint energy grid,
inner adaptive trisection midpoint rule in the ray angle per patch sector) in
code written separately with the same floating-point operation order, so the
points, weights and energies agree bit for bit; the second-line patches the
device tabulates from them then agree as integers.  The library pads each
patch to a multiple of 512 points (its sweep's segment); the oracle pads to
the largest patch.  Both keep each patch's live points first.
"""
import numpy as np
import pytest

import oracle as O
from paper_1510_07799_amd import frg

CASES = [
    dict(t=1.0, tp=0.0, mu=0.0, U=2.0, N=16, egrid=dict(n_E=24, max_level=4, rtol=1e-3)),
    dict(t=1.0, tp=-0.3, mu=-1.2, U=3.0, N=24, egrid=dict(n_E=32, max_level=5, rtol=1e-4)),
    dict(t=1.0, tp=0.2, mu=0.4, U=2.0, N=12, egrid=dict(n_E=16, max_level=3, rtol=1e-3)),
    dict(t=1.0, tp=-0.25, mu=-1.0, U=3.0, N=32, egrid=dict(n_E=48, max_level=3, rtol=1e-4)),
]


@pytest.mark.parametrize("c", CASES, ids=[f"N{c['N']}" for c in CASES])
def test_host_tables_bit_exact(c):
    e = c["egrid"]
    m = O.Model(t=c["t"], tp=c["tp"], mu=c["mu"], U=c["U"], N=c["N"], egrid=e)
    ref = m.tables(idx4=True)
    got = frg.host_tables(t=c["t"], tp=c["tp"], mu=c["mu"], U=c["U"], N=c["N"], idx4=True, egrid=e)
    N, nf_o, nf_g = c["N"], m.nf, got["nf"]
    assert nf_g % 512 == 0 and nf_o <= nf_g < nf_o + 512
    for k in ("kc", "bnd", "qpp", "qph", "idx4"):
        assert np.array_equal(got[k], ref[k]), k
    w_o = ref["w"].reshape(N, nf_o)
    cnt_o = (w_o > 0).sum(1)
    assert np.array_equal(got["count"], cnt_o)
    for k in ("px", "py", "w", "xi"):
        a = got[k].reshape(N, nf_g)
        b = ref[k].reshape(N, nf_o)
        for J in range(N):
            n = cnt_o[J]
            assert np.array_equal(a[J, :n], b[J, :n]), (k, J)
    wg = got["w"].reshape(N, nf_g)
    for J in range(N):
        assert (wg[J, cnt_o[J]:] == 0).all()
        # the padding sits on a point of its own patch (its first live point)
        assert got["px"].reshape(N, nf_g)[J, -1] == got["px"].reshape(N, nf_g)[J, 0]


def test_weights_are_the_quadratures():
    c = CASES[1]
    got = frg.host_tables(t=c["t"], tp=c["tp"], mu=c["mu"], U=c["U"], N=c["N"], idx4=False, egrid=c["egrid"])
    s = got["w"].sum()
    # not normalised: the energy midpoint rule's error across the van Hove energy
    assert s != 1.0 and abs(s - 1.0) < 0.02


@pytest.mark.parametrize("bad", [dict(n_E=0), dict(max_level=0), dict(max_level=13), dict(rtol=0.0),
                                 dict(rtol=float("nan"))])
def test_bad_egrid_rejected(bad):
    e = dict(n_E=8, max_level=3, rtol=1e-3)
    e.update(bad)
    with pytest.raises(frg.FRGError) as x:
        frg.host_tables(N=16, egrid=e)
    assert x.value.status == frg.EINVAL


def test_next_nearest_hopping_limit():
    with pytest.raises(frg.FRGError) as x:
        frg.host_tables(t=1.0, tp=0.5, N=16, egrid=dict(n_E=8, max_level=3, rtol=1e-3))
    assert x.value.status == frg.EINVAL


def test_too_many_points_not_supported():
    with pytest.raises(frg.FRGError) as x:
        frg.host_tables(N=8, egrid=dict(n_E=4000, max_level=6, rtol=1e-9), idx4=False)
    assert x.value.status == frg.ENOTSUP


def test_paper_workload_host_tables_bit_exact():
    """The workload with the paper's quadrature (N = 96, 1600 energies, relative
    target 1e-4, 27 points per sector and shell at most) on both sides."""
    from paper_1510_07799_amd import inputs as I
    p = I.model_params("E1")
    m = O.Model(**p)
    ref = m.tables(idx4=False)
    got = frg.host_tables(**p, idx4=False)
    N, nf_o, nf_g = p["N"], m.nf, got["nf"]
    print(f"E1: n_f {nf_o} (oracle) / {nf_g} (library), live points {got['count'].sum()}")
    assert nf_g % 512 == 0 and nf_o <= nf_g < nf_o + 512
    cnt = (ref["w"].reshape(N, nf_o) > 0).sum(1)
    assert np.array_equal(got["count"], cnt)
    for k in ("kc", "bnd", "qpp", "qph"):
        assert np.array_equal(got[k], ref[k]), k
    for k in ("px", "py", "w", "xi"):
        a = got[k].reshape(N, nf_g)
        b = ref[k].reshape(N, nf_o)
        for J in range(N):
            assert np.array_equal(a[J, :cnt[J]], b[J, :cnt[J]]), (k, J)
