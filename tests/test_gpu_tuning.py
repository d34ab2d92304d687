"""The autotuner and its launch parameters, through the C ABI.

Every tuning only changes launch shapes (K parts, sweep rows per block,
contraction block rows): the rhs must stay within the parity bars against the
oracle, a captured step must be re-captured after a change, and a batch must
follow its single flows under a tuning.
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

P32 = dict(t=1.0, tp=-0.25, mu=-0.9, U=2.5, N=32, n_rad=6, n_ang=4)
P48 = dict(t=1.0, tp=-0.2, mu=-0.7, U=2.0, N=48, n_rad=5, n_ang=5)   # n_f = 25: ragged lanes


def nrel(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("p", [P32, P48], ids=["n32", "n48"])
def test_every_launch_shape_keeps_parity(p):
    m, g = O.Model(**p), frg.Context(**p)
    N = p["N"]
    V = I.random_vertex(N, p["U"], seed=121, amp=0.3, symmetrise=True)
    ref = m.rhs(0.07, V)
    Vd = dev(V)
    for vs in (False, True):
        g.set_vsym(vs)
        for kparts, rows, bm in ((1, 16, 32), (3, 256, 64), (12, 32, 96), (48, 128, 32)):
            g.set_tuning(kparts=kparts, sweep_rows=rows, block_rows=bm)
            assert g.tuning() == dict(kparts=kparts, sweep_rows=rows, block_rows=bm)
            for prec, tol in ((frg.PREC_FP64, 1e-10), (frg.PREC_SPLIT_BF16, 2e-4)):
                e = nrel(g.rhs(0.07, Vd, prec).cpu().numpy(), ref)
                print(f"[tuning] N={N} vsym={vs} {kparts}/{rows}/{bm} prec={prec}: {e:.2e}", flush=True)
                assert e <= tol
    g.set_vsym(False)


def test_tuning_arguments_checked():
    g = frg.Context(**P32)
    for bad in (dict(kparts=65), dict(sweep_rows=6), dict(sweep_rows=260), dict(block_rows=48), dict(kparts=-1)):
        with pytest.raises(frg.FRGError) as e:
            g.set_tuning(**bad)
        assert e.value.status == frg.EINVAL


def test_tuner_returns_a_measured_best_and_keeps_it():
    p = P32
    g = frg.Context(**p)
    g.set_vsym(True)
    V = dev(I.random_vertex(p["N"], p["U"], seed=122, amp=0.3, symmetrise=True))
    best, ms, log = g.tune(0.3, V, frg.PREC_SPLIT_BF16, reps=2)
    print(f"[tune] {best} {ms:.4f} ms, {len(log)} candidates", flush=True)
    assert g.tuning() == best
    assert ms > 0 and len(log) >= 6
    # the chosen contraction shape is the fastest contraction candidate measured
    con = log[6:]
    row = con[np.argmin(con[:, 4])]
    assert (int(row[0]), int(row[2])) == (best["kparts"], best["block_rows"])
    assert best["sweep_rows"] == int(log[:6][np.argmin(log[:6, 3]), 1])


def test_captured_step_after_a_tuning_change_matches_eager():
    """A step captured under one tuning, then a new tuning, then steps: the graph
    is made again (the offsets and launch shapes changed) and the steps equal the
    eager launches bit for bit."""
    import os
    p = P32
    V0 = I.random_vertex(p["N"], p["U"], seed=123, amp=0.3, symmetrise=True)
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.2, rtol=1e-6, atol=1e-10, vmax=1e6, h0=-0.05)

    def run(graph):
        if graph:
            os.environ.pop("FRG_NO_GRAPH", None)
        else:
            os.environ["FRG_NO_GRAPH"] = "1"
        g = frg.Context(**p)
        try:
            V = dev(V0)
            st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
            g.flow_init(o, V, st)
            g.flow_step(o, V, st)
            g.set_tuning(kparts=5, sweep_rows=32, block_rows=64)
            for _ in range(3):
                g.flow_step(o, V, st)
            torch.cuda.synchronize()
            return V.cpu().numpy(), st.cpu().numpy()
        finally:
            os.environ.pop("FRG_NO_GRAPH", None)
            g.close()

    (Ve, se), (Vg, sg) = run(False), run(True)
    assert np.array_equal(Ve, Vg)
    assert np.array_equal(se, sg, equal_nan=True)


def test_batch_under_a_tuning_follows_single_flows():
    cfgs = [dict(P32), dict(P32, tp=-0.1, mu=-0.4, U=2.0), dict(t=1.0, tp=-0.3, mu=-1.0, U=3.0, N=24,
                                                               n_rad=6, n_ang=4)]
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=0.1, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    b = frg.Batch(cfgs)
    try:
        Ts = [0.3, 0.1, 0.05]
        Vs = [dev(I.random_vertex(c["N"], c["U"], seed=130 + i, amp=0.3, symmetrise=False))
              for i, c in enumerate(cfgs)]
        best, ms, log = b.tune(Ts, Vs, frg.PREC_FP64, reps=2)
        print(f"[batch tune] {best} {ms:.4f} ms, {len(log)} candidates", flush=True)
        b.set_tuning(kparts=3, sweep_rows=48, block_rows=32)
        Fs = b.rhs(Ts, Vs, frg.PREC_FP64)
        for i, c in enumerate(cfgs):
            ref = O.Model(**c).rhs(Ts[i], Vs[i].cpu().numpy())
            assert nrel(Fs[i].cpu().numpy(), ref) <= 1e-10
        Vb = [torch.full((c["N"],) * 3, c["U"], dtype=torch.float64, device="cuda") for c in cfgs]
        res, _ = b.flow(Vb, o)
    finally:
        b.close()
    for i, c in enumerate(cfgs):
        g = frg.Context(**c)
        V1 = torch.full((c["N"],) * 3, c["U"], dtype=torch.float64, device="cuda")
        r1, _ = g.flow(V1, o)
        assert res[i]["accepted"] == r1["accepted"] and res[i]["reason"] == r1["reason"]
        assert nrel(Vb[i].cpu().numpy(), V1.cpu().numpy()) <= 1e-9
        g.close()
