"""The paper's quadrature on the GPU against the oracle, through the C ABI.

The energy-angle grid (Sec. 4: outer midpoint energy grid, inner adaptive
midpoint rule along each energy) gives each patch hundreds to tens of
thousands of points; the sweep walks them in segments of 512 with the rows'
bins held in LDS across segments.  Compared with the oracle built on the same
quadrature:

  * the second-line patch table, bit for bit on every live point;
  * the bubble derivatives (every row, and the paired rows of the C4v
    reduction) at T = 1, 0.05 and 1e-3;
  * the rhs for constant, C4v-symmetric and unsymmetric random vertices, every
    column and one column per orbit, FP64 and split;
  * the full bubbles of the interaction flow and their rhs;
  * a DP5(4) FP64 temperature flow, step for step;
  * at the workload size (N = 96, 1600 energies, ~1.9 million points), the rhs
    on a seeded sample of entries against the oracle's brute-force sum.

Bars (normwise): FP64 1e-12 (bubbles) and 1e-10 (rhs); split 1e-5 and 2e-4.
"""
import numpy as np
import pytest

import oracle as O
from paper_1510_07799_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1510_07799_amd import frg  # noqa: E402

# several segments per patch, C4v reduction available (N % 8 == 0)
E24 = dict(t=1.0, tp=-0.3, mu=-1.2, U=3.0, N=24, n_rad=1, n_ang=1, egrid=dict(n_E=32, max_level=4, rtol=1e-4))
# no C4v octant construction (N % 8 != 0), t' > 0
E12 = dict(t=1.0, tp=0.2, mu=0.4, U=2.0, N=12, n_rad=1, n_ang=1, egrid=dict(n_E=24, max_level=3, rtol=1e-3))
CASES = {"E24": E24, "E12": E12}
TEMPS = [1.0, 0.05, 1e-3]
_cache = {}


def stats(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    return float(d.max() / np.abs(ref).max()), float(d.max())


def models(name):
    if name not in _cache:
        p = CASES[name]
        print(f"[egrid] create {name} {p}", flush=True)
        _cache[name] = (O.Model(**p), frg.Context(**p))
    return _cache[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_points_and_second_line_table(name):
    m, g = models(name)
    N = m.N
    cnt = g.counts()
    w_o = m.tables(idx4=False)["w"].reshape(N, m.nf)
    assert np.array_equal(cnt, (w_o > 0).sum(1))
    assert g.nf % 512 == 0 and g.nf >= m.nf
    print(f"[egrid] {name}: n_f {g.nf} (oracle {m.nf}), live {cnt.min()}..{cnt.max()}", flush=True)
    for kind in (O.PP, O.PH):
        got = g.bins(kind).cpu().numpy().reshape(-1, N, g.nf)
        ref = m.bins(kind).reshape(-1, N, m.nf)
        for a in range(N):
            assert np.array_equal(got[:, a, :cnt[a]], ref[:, a, :cnt[a]]), (kind, a)


@pytest.mark.parametrize("T", TEMPS)
@pytest.mark.parametrize("name", list(CASES))
def test_bubbles(name, T):
    m, g = models(name)
    Rpp, Rph = m.bubbles(T)
    for prec, tol in ((frg.PREC_FP64, 1e-12), (frg.PREC_SPLIT_BF16, 1e-5)):
        Bpp, Bph = g.bubbles(T, prec)
        e = [stats(Bpp.cpu().numpy(), Rpp), stats(Bph.cpu().numpy(), Rph)]
        if g.symmetry()[0]:
            pp_rows, ph_rows = g.bubble_reps()
            Spp, Sph = g.bubbles_reps(T, prec)
            e += [stats(Spp.cpu().numpy(), Rpp[pp_rows]), stats(Sph.cpu().numpy(), Rph[ph_rows])]
        print(f"[egrid bubbles] {name} T={T} prec={prec}: {e}", flush=True)
        for x in e:
            assert x[0] <= tol


@pytest.mark.parametrize("T", TEMPS)
@pytest.mark.parametrize("name", list(CASES))
def test_rhs(name, T):
    m, g = models(name)
    N, U = m.N, m.U
    Rpp, Rph = m.bubbles(T)
    vs = {"const": I.constant_vertex(N, U),
          "sym": I.random_vertex(N, U, seed=301, amp=0.3, symmetrise=True),
          "raw": I.random_vertex(N, U, seed=302, amp=0.3, symmetrise=False)}
    for vname, V in vs.items():
        ref = m.contract(Rpp, Rph, V)
        Vd = dev(V)
        modes = [False, True] if (vname != "raw" and N % 8 == 0) else [False]
        for vsym in modes:
            g.set_vsym(vsym)
            try:
                for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
                    e = stats(g.rhs(T, Vd, prec).cpu().numpy(), ref)
                    print(f"[egrid rhs] {name} T={T} V={vname} vsym={vsym} prec={prec}: {e[0]:.2e}", flush=True)
                    assert e[0] <= tol
            finally:
                g.set_vsym(False)


def test_full_bubbles_and_interaction_rhs():
    m, g = models("E24")
    T = 0.1
    Rpp, Rph = m.bubbles(T, deriv=0)
    for prec, tol in ((frg.PREC_FP64, 1e-12), (frg.PREC_SPLIT_BF16, 1e-5)):
        Bpp, Bph = g.bubbles_full(T, prec)
        e = [stats(Bpp.cpu().numpy(), Rpp), stats(Bph.cpu().numpy(), Rph)]
        print(f"[egrid full bubbles] prec={prec}: {e}", flush=True)
        assert max(x[0] for x in e) <= tol
    V = I.random_vertex(m.N, m.U, seed=303, amp=0.3, symmetrise=True)
    ref = m.contract(Rpp, Rph, V)
    for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
        e = stats(g.rhs_full(T, dev(V), prec).cpu().numpy(), ref)
        print(f"[egrid rhs_full] prec={prec}: {e[0]:.2e}", flush=True)
        assert e[0] <= tol


def test_fp64_flow_step_for_step():
    m, g = models("E12")
    f = dict(stepper="dp54", T0=1.0, T_min=0.01, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    V_o, r_o, log_o = m.flow(**f)
    V = torch.full((m.N,) * 3, m.U, dtype=torch.float64, device="cuda")
    r_g, log_g = g.flow(V, frg.flow_opts(prec=frg.PREC_FP64, **f))
    print(f"[egrid flow] oracle {r_o['accepted']}/{r_o['rejected']} reason {r_o['reason']}; "
          f"GPU {r_g['accepted']}/{r_g['rejected']} reason {r_g['reason']}", flush=True)
    assert (r_g["accepted"], r_g["rejected"], r_g["reason"]) == (r_o["accepted"], r_o["rejected"], r_o["reason"])
    assert np.allclose(log_g[:, 0], log_o[:, 0], rtol=0, atol=1e-9)
    assert stats(V.cpu().numpy(), V_o)[0] <= 1e-9


def test_workload_size_sampled_against_brute_force():
    """N = 96 with the paper's quadrature: 64 seeded entries of the rhs (every
    column and one column per orbit, FP64 and split) against the oracle's
    direct fine-grid sum at T = 0.05."""
    p = I.model_params("E1")
    T = 0.05
    print(f"[egrid E1] create {p}", flush=True)
    g = frg.Context(**p)
    m = O.Model(**p)
    try:
        N = p["N"]
        print(f"[egrid E1] n_f {g.nf}, live points {g.counts().sum()}, workspace {g.sizes()['workspace_bytes'] / 1e9:.1f} GB",
              flush=True)
        V = I.random_vertex(N, p["U"], seed=304, amp=0.3, symmetrise=True)
        idx = I.random_entries(N, 64, seed=305)
        ref = m.rhs_entries(T, V, idx)
        scale = np.abs(ref).max()
        Vd = dev(V)
        for vsym in (False, True):
            g.set_vsym(vsym)
            for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
                F = g.rhs(T, Vd, prec).cpu().numpy()
                got = F[idx[:, 0], idx[:, 1], idx[:, 2]]
                e = float(np.abs(got - ref).max() / scale)
                print(f"[egrid E1] vsym={vsym} prec={prec}: sampled normwise {e:.2e}", flush=True)
                assert e <= tol
    finally:
        g.close()


def test_captured_steps_equal_eager_steps():
    """Flow steps on the energy-angle grid replayed from the captured graph equal
    the eager launches bit for bit."""
    import os
    p = E24
    o = frg.flow_opts("dp54", frg.PREC_SPLIT_BF16, T0=1.0, T_min=0.1, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.02)

    def run(graph):
        if graph:
            os.environ.pop("FRG_NO_GRAPH", None)
        else:
            os.environ["FRG_NO_GRAPH"] = "1"
        g = frg.Context(**p)
        try:
            g.set_vsym(True)
            V = torch.full((p["N"],) * 3, p["U"], dtype=torch.float64, device="cuda")
            st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
            g.flow_init(o, V, st)
            for _ in range(4):
                g.flow_step(o, V, st)
            torch.cuda.synchronize()
            return V.cpu().numpy(), st.cpu().numpy()
        finally:
            os.environ.pop("FRG_NO_GRAPH", None)
            g.close()

    (Ve, se), (Vg, sg) = run(False), run(True)
    assert np.array_equal(Ve, Vg)
    assert np.array_equal(se, sg, equal_nan=True)
