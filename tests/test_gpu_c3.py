"""The benchmark workload against the oracle over whole tensors, through the C ABI.

N = 96 patches with 512 fine points each (32 radial x 16 angular), t' = -0.3,
mu = -1.2, U = 3: the size the benchmark times.  The oracle computes the
binned bubbles once per temperature and contracts them with each vertex; the
GPU paths are compared element by element:

  * bubble rows: every row (the unpaired sweep with 8 points per lane) and the
    paired representative rows the rhs sweeps under the C4v reduction;
  * the rhs at T = 1, 0.05 and 1e-3 for a constant, a C4v-symmetric random and
    an unsymmetric random vertex, FP64 and split, every column and (for the
    symmetric vertices) one column per C4v orbit;
  * two of the benchmark's drawn flows through the batched rhs (symmetric
    vertex mode, both precisions).

Bars (normwise, max|x - ref| / max|ref| over the tensor): FP64 1e-10 (rhs) and
1e-12 (bubbles); split 2e-4 (rhs) and 1e-5 (bubbles).  Each case also prints
the max-abs error and the largest relative error over the entries with
|ref| >= 1e-3 max|ref|.
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

C3 = I.model_params("C3")
_state = {}


def stats(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    scale = np.abs(ref).max()
    big = np.abs(ref) >= 1e-3 * scale
    rel = float((d[big] / np.abs(ref[big])).max()) if big.any() else 0.0
    return float(d.max() / scale), float(d.max()), rel


def models():
    if "m" not in _state:
        print(f"[C3] create {C3}", flush=True)
        _state["m"] = O.Model(**C3)
        _state["g"] = frg.Context(**C3)
    return _state["m"], _state["g"]


def oracle_bubbles(T):
    """Oracle dL/dT bubble tensors at T (one temperature cached: about 1 GB)."""
    if _state.get("T") != T:
        _state.pop("B", None)
        m, _ = models()
        print(f"[C3] oracle bubbles at T={T}", flush=True)
        _state["B"] = m.bubbles(T)
        _state["T"] = T
    return _state["B"]


def vertices(N, U):
    return {"const": I.constant_vertex(N, U),
            "sym": I.random_vertex(N, U, seed=81, amp=0.3, symmetrise=True),
            "raw": I.random_vertex(N, U, seed=82, amp=0.3, symmetrise=False)}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


TEMPS = [1.0, 0.05, 1e-3]


@pytest.mark.parametrize("T", TEMPS)
def test_c3_bubbles_every_row_and_paired_rows(T):
    m, g = models()
    Rpp, Rph = oracle_bubbles(T)
    for prec, tol in ((frg.PREC_FP64, 1e-12), (frg.PREC_SPLIT_BF16, 1e-5)):
        Bpp, Bph = g.bubbles(T, prec)
        e = [stats(Bpp.cpu().numpy(), Rpp), stats(Bph.cpu().numpy(), Rph)]
        del Bpp, Bph
        pp_rows, ph_rows = g.bubble_reps()
        Spp, Sph = g.bubbles_reps(T, prec)
        e += [stats(Spp.cpu().numpy(), Rpp[pp_rows]), stats(Sph.cpu().numpy(), Rph[ph_rows])]
        del Spp, Sph
        torch.cuda.empty_cache()
        print(f"[C3 bubbles] T={T} prec={prec} every row pp/ph, paired pp/ph (normwise, maxabs, rel): {e}",
              flush=True)
        assert len(pp_rows) == 612
        for x in e:
            assert x[0] <= tol


@pytest.mark.parametrize("T", TEMPS)
def test_c3_rhs_whole_tensor(T):
    m, g = models()
    N, U = m.N, m.U
    Rpp, Rph = oracle_bubbles(T)
    for vname, V in vertices(N, U).items():
        ref = m.contract(Rpp, Rph, V)
        Vd = dev(V)
        modes = [False, True] if vname != "raw" else [False]
        for vs in modes:
            g.set_vsym(vs)
            try:
                for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
                    got = g.rhs(T, Vd, prec).cpu().numpy()
                    e = stats(got, ref)
                    print(f"[C3 rhs] T={T} V={vname} {'orbit columns' if vs else 'every column'} "
                          f"prec={prec}: normwise {e[0]:.2e} maxabs {e[1]:.2e} rel {e[2]:.2e}", flush=True)
                    assert e[0] <= tol
            finally:
                g.set_vsym(False)
        if vname == "raw" and T == 0.05:
            # every bubble row swept (no C4v row reduction, the unpaired sweep)
            g.set_symmetry(False)
            try:
                for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
                    e = stats(g.rhs(T, Vd, prec).cpu().numpy(), ref)
                    print(f"[C3 rhs] T={T} V=raw every row prec={prec}: {e}", flush=True)
                    assert e[0] <= tol
            finally:
                g.set_symmetry(True)
        del Vd
    torch.cuda.empty_cache()


def test_c3_batched_drawn_flows_against_oracle():
    """The benchmark's batched leg draws (mu, t', U) as in the batched
    configuration at N = 96, 512 points per patch; its first two flows through
    the batched rhs in symmetric-vertex mode, against the oracle."""
    draws = I.c4_flows(n_per_N=16, Ns=(96,), n_rad=C3["n_rad"], n_ang=C3["n_ang"])[:2]
    Ts = [0.05, 1e-3]
    Vs = [I.random_vertex(96, d["U"], seed=90 + i, amp=0.3, symmetrise=True) for i, d in enumerate(draws)]
    refs = []
    for d, T, V in zip(draws, Ts, Vs):
        m = O.Model(**d)
        print(f"[C3 batch] oracle rhs {d} at T={T}", flush=True)
        refs.append(m.rhs(T, V))
        del m
    b = frg.Batch(draws)
    try:
        b.set_vsym(True)
        Vd = [dev(v) for v in Vs]
        for prec, tol in ((frg.PREC_SPLIT_BF16, 2e-4), (frg.PREC_FP64, 1e-10)):
            Fs = b.rhs(Ts, Vd, prec)
            for i, (F, ref) in enumerate(zip(Fs, refs)):
                e = stats(F.cpu().numpy(), ref)
                print(f"[C3 batch] flow {i} T={Ts[i]} prec={prec}: normwise {e[0]:.2e} maxabs {e[1]:.2e} "
                      f"rel {e[2]:.2e}", flush=True)
                assert e[0] <= tol
    finally:
        b.close()
