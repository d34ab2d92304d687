"""GPU path vs the CPU oracle, element by element, through the C ABI.

Bars (from the arithmetic of each path):
  - integer maps (second-line patch of every (row, point)): bit-exact;
  - FP64 bubbles and rhs: normwise relative error <= 1e-10 (rounding-order only);
  - split path (FP32 compensated bubbles, split-BF16 MFMA contraction with FP32
    accumulation): normwise relative error <= 2e-4 on the rhs, 1e-5 on bubbles.
Normwise error = max|x - x_ref| / max|x_ref| over the whole tensor.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1510_07799_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1510_07799_amd import frg  # noqa: E402  (loads libfrg.so; fails loudly if missing)

RAGGED = dict(t=1.0, tp=-0.12, mu=-0.35, U=2.0, N=12, n_rad=5, n_ang=3)   # N%8 != 0, n_f = 15
TINY = dict(t=1.0, tp=-0.15, mu=-0.3, U=2.0, N=4, n_rad=3, n_ang=2)
SMALL_ODD = dict(t=1.0, tp=-0.2, mu=-0.6, U=2.5, N=24, n_rad=9, n_ang=10)  # n_f = 90 (ragged tiles)
# N % 32 == 0: the split contraction's buffer-load path
FAST32 = dict(t=1.0, tp=-0.25, mu=-0.9, U=2.5, N=32, n_rad=6, n_ang=4)
FAST64 = dict(t=1.0, tp=-0.3, mu=-1.1, U=3.0, N=64, n_rad=4, n_ang=3)


def nrel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


_models = {}


def pair(name_or_params):
    key = name_or_params if isinstance(name_or_params, str) else tuple(sorted(name_or_params.items()))
    if key not in _models:
        p = I.model_params(name_or_params) if isinstance(name_or_params, str) else name_or_params
        print(f"[gpu] create {p}", flush=True)
        _models[key] = (O.Model(**p), frg.Context(**p))
    return _models[key]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("cfg", ["C1", "C2", RAGGED, TINY, SMALL_ODD], ids=["C1", "C2", "ragged", "tiny", "odd"])
def test_second_line_patches_bit_exact(cfg):
    om, g = pair(cfg)
    for kind in (O.PP, O.PH):
        ref = om.bins(kind)
        got = g.bins(kind).cpu().numpy().astype(np.int32)
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), f"kind {kind}: {np.count_nonzero(got != ref)} mismatches"


def test_tables_bit_exact_through_context():
    om, g = pair("C2")
    a, b = g.tables(), om.tables()
    for k in b:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("T", [0.5, 0.05, 1e-3])
@pytest.mark.parametrize("cfg", ["C1", RAGGED, SMALL_ODD], ids=["C1", "ragged", "odd"])
def test_bubbles_fp64(cfg, T):
    om, g = pair(cfg)
    Rpp, Rph = om.bubbles(T)
    Bpp, Bph = g.bubbles(T, frg.PREC_FP64)
    torch.cuda.synchronize()
    assert nrel(Bpp.cpu().numpy(), Rpp) <= 1e-12
    assert nrel(Bph.cpu().numpy(), Rph) <= 1e-12


@pytest.mark.parametrize("T", [0.5, 0.05, 1e-3])
def test_bubbles_split(T):
    om, g = pair("C1")
    Rpp, Rph = om.bubbles(T)
    Bpp, Bph = g.bubbles(T, frg.PREC_SPLIT_BF16)
    torch.cuda.synchronize()
    assert nrel(Bpp.cpu().numpy(), Rpp) <= 1e-5
    assert nrel(Bph.cpu().numpy(), Rph) <= 1e-5


def test_bubbles_production_grid():
    om, g = pair("C2")
    for T in (0.07, 2e-3):
        Rpp, Rph = om.bubbles(T)
        Bpp, Bph = g.bubbles(T, frg.PREC_FP64)
        Spp, Sph = g.bubbles(T, frg.PREC_SPLIT_BF16)
        torch.cuda.synchronize()
        assert nrel(Bpp.cpu().numpy(), Rpp) <= 1e-12 and nrel(Bph.cpu().numpy(), Rph) <= 1e-12
        assert nrel(Spp.cpu().numpy(), Rpp) <= 1e-5 and nrel(Sph.cpu().numpy(), Rph) <= 1e-5


def _vertices(N, U):
    return {"const": I.constant_vertex(N, U),
            "sym": I.random_vertex(N, U, seed=21, symmetrise=True),
            "raw": I.random_vertex(N, U, seed=22, symmetrise=False)}


@pytest.mark.parametrize("cfg", ["C1", RAGGED, TINY, SMALL_ODD, "C2", FAST32, FAST64],
                         ids=["C1", "ragged", "tiny", "odd", "C2", "n32", "n64"])
def test_rhs_fp64(cfg):
    om, g = pair(cfg)
    N, U = om.N, om.U
    for T in (0.3, 0.02):
        for vname, V in _vertices(N, U).items():
            ref = om.rhs(T, V)
            got = g.rhs(T, dev(V), frg.PREC_FP64).cpu().numpy()
            err = nrel(got, ref)
            print(f"[fp64] N={N} T={T} {vname}: {err:.2e}", flush=True)
            assert err <= 1e-10


@pytest.mark.parametrize("cfg", ["C1", RAGGED, SMALL_ODD, "C2", FAST32, FAST64],
                         ids=["C1", "ragged", "odd", "C2", "n32", "n64"])
def test_rhs_split(cfg):
    om, g = pair(cfg)
    N, U = om.N, om.U
    for T in (0.3, 0.02):
        for vname, V in _vertices(N, U).items():
            ref = om.rhs(T, V)
            got = g.rhs(T, dev(V), frg.PREC_SPLIT_BF16).cpu().numpy()
            err = nrel(got, ref)
            print(f"[split] N={N} T={T} {vname}: {err:.2e}", flush=True)
            assert err <= 2e-4


def test_rhs_deterministic():
    om, g = pair("C2")
    V = dev(I.random_vertex(om.N, om.U, seed=5))
    a = g.rhs(0.05, V, frg.PREC_FP64).clone()
    b = g.rhs(0.05, V, frg.PREC_FP64).clone()
    assert torch.equal(a, b)
    a = g.rhs(0.05, V, frg.PREC_SPLIT_BF16).clone()
    b = g.rhs(0.05, V, frg.PREC_SPLIT_BF16).clone()
    assert torch.equal(a, b)


def test_rhs_full_size_sampled():
    """N = 96, n_f = 512 (the benchmark workload): sampled entries against the
    oracle's brute-force per-entry sum, plus a normwise bound from the sample."""
    om, g = pair("C3")
    N, U = om.N, om.U
    V = I.random_vertex(N, U, seed=31, amp=0.3)
    idx = I.random_entries(N, 24, seed=32)
    for T in (0.05,):
        ref = om.rhs_entries(T, V, idx)
        F64 = g.rhs(T, dev(V), frg.PREC_FP64).cpu().numpy()
        Fsp = g.rhs(T, dev(V), frg.PREC_SPLIT_BF16).cpu().numpy()
        scale = np.abs(F64).max()
        got64 = F64[idx[:, 0], idx[:, 1], idx[:, 2]]
        gotsp = Fsp[idx[:, 0], idx[:, 1], idx[:, 2]]
        e64 = np.abs(got64 - ref).max() / scale
        esp = np.abs(gotsp - ref).max() / scale
        print(f"[C3 sampled] fp64 {e64:.2e} split {esp:.2e} kskip {g.kskip()}", flush=True)
        assert e64 <= 1e-10
        assert esp <= 2e-4
        # whole-tensor agreement of the two GPU paths
        assert nrel(Fsp, F64) <= 2e-4


def test_rhs_largest_sampled_and_c4v_equivariant():
    """N = 192, n_f = 1024 (the largest workload: two m tiles, 16 points per lane):
    10^4 seeded entries against the oracle's brute-force per-entry sum, and, over
    the whole tensor, F(g j1, g j2, g j3) = F(j1, j2, j3) for a C4v symmetric V
    (a property that holds at any size)."""
    om, g = pair("C5")
    N, U = om.N, om.U
    V = I.random_vertex(N, U, seed=33, amp=0.3, symmetrise=True)
    idx = I.random_entries(N, 10000, seed=34)
    T = 0.05
    print("[C5] oracle brute force on 10^4 entries", flush=True)
    ref = om.rhs_entries(T, V, idx)
    F64 = g.rhs(T, dev(V), frg.PREC_FP64).cpu().numpy()
    Fsp = g.rhs(T, dev(V), frg.PREC_SPLIT_BF16).cpu().numpy()
    scale = np.abs(F64).max()
    e64 = np.abs(F64[idx[:, 0], idx[:, 1], idx[:, 2]] - ref).max() / scale
    esp = np.abs(Fsp[idx[:, 0], idx[:, 1], idx[:, 2]] - ref).max() / scale
    print(f"[C5 sampled] fp64 {e64:.2e} split {esp:.2e} (max-abs {e64 * scale:.2e} / {esp * scale:.2e}) "
          f"kskip {g.kskip()}", flush=True)
    assert e64 <= 1e-10
    assert esp <= 2e-4
    assert nrel(Fsp, F64) <= 2e-4
    # the same entries in symmetric-vertex mode (one column per C4v orbit)
    g.set_vsym(True)
    try:
        for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
            Fv = g.rhs(T, dev(V), prec).cpu().numpy()
            ev = np.abs(Fv[idx[:, 0], idx[:, 1], idx[:, 2]] - ref).max() / scale
            print(f"[C5 sampled, orbit columns] prec={prec}: {ev:.2e}", flush=True)
            assert ev <= tol
    finally:
        g.set_vsym(False)
    for o in range(1, 8):
        p = I.c4v_patch_perm(N, o)
        for F, tol in ((F64, 1e-12), (Fsp, 2e-4)):
            Fg = F[np.ix_(p, p, p)]
            assert nrel(Fg, F) <= tol, (o, nrel(Fg, F))


def test_rhs_argument_errors():
    om, g = pair("C1")
    N = om.N
    V = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(frg.FRGError) as e:
        g.rhs(0.0, V)
    assert e.value.status == frg.EINVAL
    with pytest.raises(frg.FRGError) as e:
        g.rhs(float("nan"), V)
    assert e.value.status == frg.EINVAL
    with pytest.raises(frg.FRGError) as e:
        g.rhs(0.1, V, out=V)
    assert e.value.status == frg.EINVAL
    with pytest.raises(frg.FRGError) as e:
        frg.Context(t=1, tp=0, mu=0, U=1, N=10, n_rad=2, n_ang=2)
    assert e.value.status == frg.EINVAL


def test_flow_c1_rk4_matches_oracle():
    om, g = pair("C1")
    N, U = om.N, om.U
    Vo, ro, _ = om.flow(stepper="rk4", fixed_steps=40, T_min=0.05, vmax=20.0)
    V = dev(np.full((N, N, N), U))
    res, log = g.flow(V, frg.flow_opts("rk4", frg.PREC_FP64, T0=1.0, T_min=0.05, fixed_steps=40, vmax=20.0))
    print("[flow C1 rk4]", res, ro, flush=True)
    assert res["reason"] == ro["reason"] == O.STOP_DIVERGED
    assert res["accepted"] == ro["accepted"]
    assert math.log(res["T_c_interp"]) == pytest.approx(ro["s_c_interp"], abs=1e-9)
    assert nrel(V.cpu().numpy(), Vo) <= 1e-9


def test_flow_dp54_matches_oracle_and_first_step():
    om, g = pair("C1")
    N, U = om.N, om.U
    Vo, ro, lo = om.flow(stepper="dp54", T_min=0.05, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    V = dev(np.full((N, N, N), U))
    res, log = g.flow(V, frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.05, rtol=1e-6,
                                       atol=1e-10, vmax=20.0, h0=-0.01))
    print("[flow C1 dp54]", res, ro, flush=True)
    import json
    import os
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
    assert res["first_step_rhs"] == golden["rhs_evals_first_step"]["value"] == ro["first_step_rhs"]
    assert res["reason"] == ro["reason"]
    assert res["accepted"] == ro["accepted"] and res["rejected"] == ro["rejected"]
    assert np.allclose(log[:, 0], lo[:, 0], rtol=0, atol=1e-9)
    assert nrel(V.cpu().numpy(), Vo) <= 1e-8


def test_flow_step_api_and_tmin_stop():
    """frg_flow_step driven from the host to T_min without divergence (small U)."""
    p = dict(t=1.0, tp=-0.1, mu=-0.3, U=0.5, N=8, n_rad=4, n_ang=4)
    om, g = pair(p)
    N = om.N
    Vo, ro, _ = om.flow(stepper="dp54", T0=1.0, T_min=0.2, rtol=1e-7, atol=1e-12, vmax=20.0, h0=-0.05)
    V = dev(np.full((N, N, N), 0.5))
    state = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.2, rtol=1e-7, atol=1e-12, vmax=20.0, h0=-0.05)
    g.flow_init(o, V, state)
    for _ in range(500):
        g.flow_step(o, V, state)
        if state[frg.ST_REASON].item() != 0:
            break
    st = state.cpu().numpy()
    assert st[frg.ST_REASON] == O.STOP_TMIN == ro["reason"]
    assert st[frg.ST_S] == pytest.approx(math.log(0.2), abs=1e-15)
    assert int(st[frg.ST_ACCEPTED]) == ro["accepted"]
    assert nrel(V.cpu().numpy(), Vo) <= 1e-9


@pytest.mark.parametrize("cfg", ["C1", SMALL_ODD, "C2", FAST64], ids=["C1", "odd", "C2", "n64"])
def test_c4v_row_reduction_matches_full_rows(cfg):
    """Bubble rows computed for one transfer per C4v orbit and read through the
    patch permutation give the same rhs as computing every row."""
    om, g = pair(cfg)
    active, rows = g.symmetry()
    assert active and rows < (g.Tpp + g.Tph) / 6
    V = dev(I.random_vertex(om.N, om.U, seed=41, symmetrise=False))
    for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
        Fs = g.rhs(0.04, V, prec).cpu().numpy()
        g.set_symmetry(False)
        try:
            assert g.symmetry() == (False, g.Tpp + g.Tph)
            Ff = g.rhs(0.04, V, prec).cpu().numpy()
        finally:
            g.set_symmetry(True)
        ref = om.rhs(0.04, V.cpu().numpy())
        assert nrel(Fs, ref) <= tol and nrel(Ff, ref) <= tol
        if prec == frg.PREC_FP64:
            assert nrel(Fs, Ff) <= 1e-12


def test_c4v_reduction_unavailable_for_n_not_multiple_of_8():
    om, g = pair(RAGGED)
    assert g.symmetry() == (False, g.Tpp + g.Tph)
    with pytest.raises(frg.FRGError) as e:
        g.set_symmetry(True)
    assert e.value.status == frg.ENOTSUP


@pytest.mark.parametrize("cfg", ["C1", RAGGED, SMALL_ODD, "C2", FAST64], ids=["C1", "ragged", "odd", "C2", "n64"])
def test_zero_block_skipping_matches_dense(cfg):
    """Visiting only the k chunks where some bubble row of a column tile has a
    fine point gives the dense contraction's rhs (skipped terms are exact
    zeros; only the summation order differs)."""
    om, g = pair(cfg)
    on, frac = g.kskip()
    assert on and 0.0 < frac <= 1.0
    print(f"[kskip] N={om.N}: executed share {frac:.3f}", flush=True)
    if om.N >= 48:
        assert frac < 0.8
    V = dev(I.random_vertex(om.N, om.U, seed=43, symmetrise=False))
    ref = om.rhs(0.03, V.cpu().numpy())
    for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
        Fs = g.rhs(0.03, V, prec).cpu().numpy()
        g.set_kskip(False)
        try:
            assert g.kskip() == (False, 1.0)
            Fd = g.rhs(0.03, V, prec).cpu().numpy()
        finally:
            g.set_kskip(True)
        assert nrel(Fs, ref) <= tol and nrel(Fd, ref) <= tol
        if prec == frg.PREC_FP64:
            assert nrel(Fs, Fd) <= 1e-12


@pytest.mark.parametrize("cfg", [FAST32, FAST64, "C3"], ids=["n32", "n64", "C3"])
def test_split_buffer_path_matches_general_path(cfg, monkeypatch):
    """For N % 32 == 0 the split contraction reads its operands with buffer
    loads (out-of-range offsets read zero); FRG_NO_FAST forces the general
    loads.  Both paths do the same arithmetic in the same order."""
    om, g = pair(cfg)
    V = dev(I.random_vertex(om.N, om.U, seed=47, symmetrise=False))
    Ff = g.rhs(0.03, V, frg.PREC_SPLIT_BF16).cpu().numpy()
    monkeypatch.setenv("FRG_NO_FAST", "1")
    Fg = g.rhs(0.03, V, frg.PREC_SPLIT_BF16).cpu().numpy()
    monkeypatch.delenv("FRG_NO_FAST")
    print(f"[fast/general] N={om.N}: {nrel(Ff, Fg):.2e}", flush=True)
    assert np.array_equal(Ff, Fg)


BATCH = [dict(t=1.0, tp=-0.1, mu=-0.3, U=2.0, N=16, n_rad=4, n_ang=4),
         dict(t=1.0, tp=-0.3, mu=-0.9, U=2.5, N=24, n_rad=4, n_ang=4),
         dict(t=1.0, tp=0.0, mu=0.0, U=1.5, N=32, n_rad=4, n_ang=4),
         dict(t=1.0, tp=-0.2, mu=-0.5, U=3.0, N=12, n_rad=4, n_ang=4)]


def test_batch_rhs_matches_single_flows_and_oracle():
    b = frg.Batch(BATCH)
    Vs = [dev(I.random_vertex(p["N"], p["U"], seed=50 + i, symmetrise=False)) for i, p in enumerate(BATCH)]
    Ts = [0.3, 0.05, 0.1, 0.02]
    for prec, tol in ((frg.PREC_FP64, 1e-12), (frg.PREC_SPLIT_BF16, 2e-4)):
        Fs = b.rhs(Ts, Vs, prec)
        for i, p in enumerate(BATCH):
            om, g = pair(p)
            single = g.rhs(Ts[i], Vs[i], prec).cpu().numpy()
            got = Fs[i].cpu().numpy()
            assert nrel(got, single) <= (1e-12 if prec == frg.PREC_FP64 else 1e-5), (i, prec)
            if i in (0, 3):
                assert nrel(got, om.rhs(Ts[i], Vs[i].cpu().numpy())) <= (1e-10 if prec == frg.PREC_FP64 else tol)
    b.close()


def test_batch_flow_matches_single_flows():
    b = frg.Batch(BATCH)
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.02, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    Vs = [torch.full((p["N"],) * 3, p["U"], dtype=torch.float64, device="cuda") for p in BATCH]
    res, log = b.flow(Vs, o, log_cap=256)
    for i, p in enumerate(BATCH):
        om, g = pair(p)
        V1 = torch.full((p["N"],) * 3, p["U"], dtype=torch.float64, device="cuda")
        r1, l1 = g.flow(V1, o)
        print("[batch flow]", i, res[i], r1, flush=True)
        assert res[i]["reason"] == r1["reason"]
        assert res[i]["accepted"] == r1["accepted"] and res[i]["rejected"] == r1["rejected"]
        assert res[i]["first_step_rhs"] == 7
        assert np.allclose(log[i, :res[i]["accepted"], 0], l1[:, 0], rtol=0, atol=1e-9)
        assert nrel(Vs[i].cpu().numpy(), V1.cpu().numpy()) <= 1e-9
    b.close()


@pytest.mark.parametrize("cfg", ["C1", FAST64, "C3"], ids=["C1", "n64", "C3"])
def test_symmetric_vertex_mode_matches_full_rhs(cfg):
    """For a C4v-invariant V the rhs from one column per C4v orbit equals the
    rhs from every column, and F is exactly invariant."""
    om, g = pair(cfg)
    N = om.N
    V = dev(I.random_vertex(N, om.U, seed=51, amp=0.3, symmetrise=True))
    assert g.check_vsym(V) <= 1e-15
    ref = om.rhs(0.04, V.cpu().numpy()) if N <= 64 else None
    for prec, tol in ((frg.PREC_FP64, 1e-12), (frg.PREC_SPLIT_BF16, 2e-4)):
        Ff = g.rhs(0.04, V, prec).cpu().numpy()
        g.set_vsym(True)
        try:
            active, cols = g.vsym()
            assert active and N * N <= 8 * cols <= N * N + 8 * N
            Fs = g.rhs(0.04, V, prec).cpu().numpy()
        finally:
            g.set_vsym(False)
        print(f"[vsym] N={N} prec={prec} cols={cols}: {nrel(Fs, Ff):.2e}", flush=True)
        assert nrel(Fs, Ff) <= tol
        if ref is not None:
            assert nrel(Fs, ref) <= (1e-10 if prec == frg.PREC_FP64 else 2e-4)
        for o in range(1, 8):
            p = I.c4v_patch_perm(N, o)
            assert np.array_equal(Fs[np.ix_(p, p, p)], Fs)


@pytest.mark.parametrize("cfg", ["C3", FAST64], ids=["C3", "n64"])
def test_orbit_column_tiles_stay_as_dense_as_every_column_tiles(cfg):
    """The representative of each column orbit is the member whose transfer lies
    in one C4v wedge, so the orbit columns' transfers fill that wedge densely
    and a 64-column tile visits about the same share of the k chunks as the
    every-column tiles do (0.45 at N = 96; the orbit's smallest natural index
    as representative scattered the transfers and gave 0.59)."""
    _, g = pair(cfg)
    _, full = g.kskip()
    g.set_vsym(True)
    try:
        _, cols = g.vsym()
        _, orb = g.kskip()
    finally:
        g.set_vsym(False)
    N = g.N
    per_col = orb * N * N / cols   # chunk share per computed orbit column
    print(f"[tiles] N={N}: every column {full:.3f}, orbit columns {per_col:.3f}", flush=True)
    assert per_col <= 1.06 * full


def test_symmetric_vertex_orbit_count_and_checks():
    """About N^3/8 independent entries (the paper's count at N = 32 is 4072,
    which also uses spin and time-reversal symmetry); the mode refuses a grid
    without exact covariance and a flow from a non-invariant vertex."""
    om, g = pair(FAST32)
    N = om.N
    g.set_vsym(True)
    try:
        _, cols = g.vsym()
        assert abs(cols * N - N ** 3 / 8) / (N ** 3 / 8) < 0.05
        V = dev(I.random_vertex(N, om.U, seed=52, symmetrise=False))
        assert g.check_vsym(V) > 1e-3
        state = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
        opts = frg.flow_opts("rk4", frg.PREC_FP64, T0=1.0, T_min=0.5, fixed_steps=2, vmax=1e9)
        with pytest.raises(frg.FRGError) as e:
            g.flow_init(opts, V, state)
        assert e.value.status == frg.EINVAL
    finally:
        g.set_vsym(False)
    _, gr = pair(RAGGED)
    with pytest.raises(frg.FRGError) as e:
        gr.set_vsym(True)
    assert e.value.status == frg.ENOTSUP


def test_symmetric_vertex_flows_single_and_batched():
    """A DP5(4) flow from V = U (invariant) in symmetric-vertex mode follows the
    full-vertex flow step for step, alone and in a batch."""
    cfgs = [p for p in BATCH if p["N"] % 8 == 0]
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.02, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    ref = []
    for p in cfgs:
        om, g = pair(p)
        V1 = torch.full((p["N"],) * 3, p["U"], dtype=torch.float64, device="cuda")
        r1, _ = g.flow(V1, o)
        ref.append((r1, V1.cpu().numpy()))
        g.set_vsym(True)
        try:
            V2 = torch.full((p["N"],) * 3, p["U"], dtype=torch.float64, device="cuda")
            r2, _ = g.flow(V2, o)
        finally:
            g.set_vsym(False)
        assert (r2["reason"], r2["accepted"], r2["rejected"]) == (r1["reason"], r1["accepted"], r1["rejected"])
        assert nrel(V2.cpu().numpy(), ref[-1][1]) <= 1e-9
    b = frg.Batch(cfgs)
    b.set_vsym(True)
    Vs = [torch.full((p["N"],) * 3, p["U"], dtype=torch.float64, device="cuda") for p in cfgs]
    res, _ = b.flow(Vs, o, log_cap=256)
    for i, (r1, v1) in enumerate(ref):
        assert res[i]["accepted"] == r1["accepted"] and res[i]["reason"] == r1["reason"]
        assert nrel(Vs[i].cpu().numpy(), v1) <= 1e-9
    b.close()


def test_symmetric_vertex_flow_from_random_invariant_vertex():
    """Flows in symmetric-vertex mode keep one entry per orbit column and free
    index and expand it for every rhs input and for V: from a random C4v-invariant
    vertex (so a wrong gather or expansion index shows at once), fixed RK4 and
    DP5(4) steps follow the every-column flow, and V stays exactly invariant.  In
    the split path the two modes round differently, so both are held to the FP64
    flow instead, the symmetric one within three times the other's error."""
    om, g = pair(FAST32)
    N = om.N
    V0 = I.random_vertex(N, om.U, seed=53, amp=0.3, symmetrise=True)

    def run(stepper, prec, vs):
        kw = dict(fixed_steps=4) if stepper == "rk4" else dict(rtol=1e-6, atol=1e-10, h0=-0.05)
        o = frg.flow_opts(stepper, prec, T0=1.0, T_min=0.3, vmax=1e6, **kw)
        g.set_vsym(vs)
        try:
            V = dev(V0)
            st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
            g.flow_init(o, V, st)
            for _ in range(4):
                g.flow_step(o, V, st)
            torch.cuda.synchronize()
            return V.cpu().numpy(), st.cpu().numpy()
        finally:
            g.set_vsym(False)

    for stepper in ("rk4", "dp54"):
        (Vf, sf), (Vs, ss) = run(stepper, frg.PREC_FP64, False), run(stepper, frg.PREC_FP64, True)
        print(f"[vsym flow] {stepper} FP64: {nrel(Vs, Vf):.2e}", flush=True)
        # the error norm differs in its rounding (other K-part sums), so the
        # DP5(4) step sizes differ slightly
        assert ss[frg.ST_S] == pytest.approx(sf[frg.ST_S], abs=1e-10)
        assert nrel(Vs, Vf) <= 1e-10
        assert nrel(Vs, V0) > 1e-3   # the flow moved
        for o_ in range(1, 8):
            pm = I.c4v_patch_perm(N, o_)
            assert np.array_equal(Vs[np.ix_(pm, pm, pm)], Vs)
        if stepper == "rk4":
            (Vfs, _), (Vss, _) = (run(stepper, frg.PREC_SPLIT_BF16, False),
                                  run(stepper, frg.PREC_SPLIT_BF16, True))
            ef, es = nrel(Vfs, Vf), nrel(Vss, Vf)
            print(f"[vsym flow] rk4 split against FP64: every column {ef:.2e}, symmetric {es:.2e}", flush=True)
            assert es <= max(3.0 * ef, 1e-5)
            for o_ in range(1, 8):
                pm = I.c4v_patch_perm(N, o_)
                assert np.array_equal(Vss[np.ix_(pm, pm, pm)], Vss)


def test_batched_split_symmetric_flows_follow_every_column_flows():
    """Batched split-BF16 steps in symmetric-vertex mode (reduced stage vectors,
    the layout reading them directly, the reduced combine) follow the same
    batch computing every column, from random C4v-invariant vertices."""
    cfgs = [p for p in BATCH if p["N"] % 8 == 0]
    V0 = [I.random_vertex(p["N"], p["U"], seed=60 + i, amp=0.3, symmetrise=True) for i, p in enumerate(cfgs)]
    # a tolerance the truncation error dominates, so that the split rounding of the
    # two modes does not steer the step sizes apart
    o = frg.flow_opts("dp54", frg.PREC_SPLIT_BF16, T0=1.0, T_min=0.2, rtol=1e-3, atol=1e-6, vmax=1e6,
                      h0=-0.05)
    out = []
    for vs in (False, True):
        b = frg.Batch(cfgs)
        try:
            b.set_vsym(vs)
            Vs = [dev(v) for v in V0]
            b.flow_init(Vs, o)
            for _ in range(4):
                b.flow_step()
            res, _ = b.results()
            torch.cuda.synchronize()
            out.append((res, [v.cpu().numpy() for v in Vs]))
        finally:
            b.close()
    (rf, Vf), (rs, Vs) = out
    for i, p in enumerate(cfgs):
        err = nrel(Vs[i], Vf[i])
        print(f"[batch vsym split] N={p['N']}: T {rs[i]['T_end']:.9f} / {rf[i]['T_end']:.9f}, V {err:.2e}",
              flush=True)
        assert rs[i]["accepted"] == rf[i]["accepted"]
        assert rs[i]["T_end"] == pytest.approx(rf[i]["T_end"], rel=1e-4)
        assert err <= 1e-3
        assert nrel(Vs[i], V0[i]) > 1e-3
        for o_ in range(1, 8):
            pm = I.c4v_patch_perm(p["N"], o_)
            assert np.array_equal(Vs[i][np.ix_(pm, pm, pm)], Vs[i])


def test_batched_symmetric_split_step_at_benchmark_size():
    """The benchmark's batched path at its full size (N = 96, n_f = 512: split,
    symmetric-vertex mode, reduced stage vectors read by the layout, evened-out
    sweep chunks, batch K parts) against the same flows stepped one at a time,
    whose symmetric rhs is checked against the every-column rhs and that one
    against the oracle's sampled entries above."""
    p0 = I.model_params("C3")
    cfgs = [p0, dict(p0, mu=-0.9, tp=-0.2, U=2.5)]
    V0 = [I.random_vertex(p["N"], p["U"], seed=70 + i, amp=0.3, symmetrise=True) for i, p in enumerate(cfgs)]
    o = frg.flow_opts("dp54", frg.PREC_SPLIT_BF16, T0=1.0, T_min=0.05, rtol=1e-3, atol=1e-6, vmax=1e6,
                      h0=-0.05)
    single = []
    for p, v in zip(cfgs, V0):
        g = frg.Context(**p)
        g.set_vsym(True)
        V = dev(v)
        st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
        g.flow_init(o, V, st)
        g.flow_step(o, V, st)
        torch.cuda.synchronize()
        single.append((V.cpu().numpy(), st.cpu().numpy()))
        del g
    b = frg.Batch(cfgs)
    try:
        b.set_vsym(True)
        Vs = [dev(v) for v in V0]
        b.flow_init(Vs, o)
        b.flow_step()
        res, _ = b.results()
        torch.cuda.synchronize()
        for i, (Vsg, ssg) in enumerate(single):
            Vb = Vs[i].cpu().numpy()
            err = nrel(Vb, Vsg)
            print(f"[C3 batch step] flow {i}: T {res[i]['T_end']:.9f} / {np.exp(ssg[frg.ST_S]):.9f}, V {err:.2e}",
                  flush=True)
            assert res[i]["T_end"] == pytest.approx(np.exp(ssg[frg.ST_S]), rel=1e-9)
            assert err <= 1e-4
            assert nrel(Vb, V0[i]) > 1e-4
    finally:
        b.close()


def test_symmetric_vertex_toggled_mid_flow():
    """Switching the mode between steps converts the rhs a DP5(4) flow carries to
    its next step (first same as last) to the new form: a flow switched on after
    two steps and off after two more follows the every-column flow."""
    om, g = pair(FAST32)
    N = om.N
    V0 = I.random_vertex(N, om.U, seed=54, amp=0.3, symmetrise=True)
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.2, rtol=1e-6, atol=1e-10, vmax=1e6, h0=-0.05)
    runs = []
    for pattern in ((False,) * 6, (False, False, True, True, False, False)):
        V = dev(V0)
        st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
        g.set_vsym(False)
        g.flow_init(o, V, st)
        try:
            for vs in pattern:
                g.set_vsym(vs)
                g.flow_step(o, V, st)
            torch.cuda.synchronize()
        finally:
            g.set_vsym(False)
        runs.append((V.cpu().numpy(), st.cpu().numpy()))
    (Va, sa), (Vb, sb) = runs
    print(f"[vsym toggle] {nrel(Vb, Va):.2e}", flush=True)
    assert sb[frg.ST_S] == pytest.approx(sa[frg.ST_S], abs=1e-10)
    assert nrel(Vb, Va) <= 1e-10


def test_flow_step_graph_replay_matches_eager():
    """Single-flow steps replay one captured graph; with eager rhs work on the
    same context between the replays they give bit for bit the state of the
    eager launches (FRG_NO_GRAPH, read per call)."""
    import os
    om, g = pair("C1")
    N, U = om.N, om.U
    o = frg.flow_opts("dp54", frg.PREC_SPLIT_BF16, T0=1.0, T_min=0.05, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.02)

    def run(graph):
        if graph:
            os.environ.pop("FRG_NO_GRAPH", None)
        else:
            os.environ["FRG_NO_GRAPH"] = "1"
        try:
            V = dev(np.full((N, N, N), U))
            st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
            g.flow_init(o, V, st)
            other = dev(I.random_vertex(N, U, seed=7))
            for _ in range(6):
                g.flow_step(o, V, st)
                g.rhs(0.3, other, frg.PREC_FP64)
                torch.cuda.synchronize()
            return V.cpu().numpy(), st.cpu().numpy()
        finally:
            os.environ.pop("FRG_NO_GRAPH", None)

    Ve, se = run(False)
    Vg, sg = run(True)
    diff = [(i, se[i], sg[i]) for i in range(len(se)) if not (se[i] == sg[i] or (se[i] != se[i] and sg[i] != sg[i]))]
    print("[flow graph] state differences:", diff, flush=True)
    assert np.array_equal(Ve, Vg)
    assert not diff


def test_flow_step_graph_after_workspace_reallocation():
    """A captured step holds the address of the channel buffer; an eager rhs in
    symmetric-vertex mode needs more K parts (16 against 8 at N = 32) and
    reallocates that buffer.  Toggling the mode back must not replay the old
    graph: the steps equal the eager launches (FRG_NO_GRAPH) bit for bit."""
    import os
    om, g = pair(FAST32)
    N, U = om.N, om.U
    V0 = I.random_vertex(N, U, seed=55, amp=0.3, symmetrise=True)
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.2, rtol=1e-6, atol=1e-10, vmax=1e6, h0=-0.05)

    def run(graph):
        if graph:
            os.environ.pop("FRG_NO_GRAPH", None)
        else:
            os.environ["FRG_NO_GRAPH"] = "1"
        # a fresh context each time, so that the channel buffer starts at the
        # every-column size
        c = frg.Context(**FAST32)
        try:
            V = dev(V0)
            st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
            c.flow_init(o, V, st)
            c.flow_step(o, V, st)                        # captured with 8 K parts
            c.set_vsym(True)
            F = c.rhs(0.3, dev(V0), frg.PREC_FP64)       # 16 K parts: the buffer moves
            c.set_vsym(False)
            for _ in range(3):
                c.flow_step(o, V, st)                    # same key as the first capture
            torch.cuda.synchronize()
            return V.cpu().numpy(), st.cpu().numpy(), F.cpu().numpy()
        finally:
            os.environ.pop("FRG_NO_GRAPH", None)
            c.close()

    Ve, se, Fe = run(False)
    Vg, sg, Fg = run(True)
    print(f"[graph realloc] V {nrel(Vg, Ve):.2e} F {nrel(Fg, Fe):.2e}", flush=True)
    assert np.array_equal(Ve, Vg)
    assert np.array_equal(Fe, Fg)
    assert np.array_equal(se, sg, equal_nan=True)
