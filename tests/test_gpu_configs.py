"""The workloads' flows on the GPU, with their errors stated (through the C ABI).

Eq. (1) of the paper is integrated by an explicit stepper whose rhs is
evaluated with V frozen (Sec. 2); Sec. 4 times the seven rhs evaluations of the
first step.  Each test runs one workload's flow and prints its error table:

  * production FP64 (N = 48): the GPU's adaptive DP5(4) flow against the
    oracle's own flow (step log and final vertex stored by
    tests/golden/make_c2_flow.py), and the GPU rhs against the oracle's at
    every accepted state;
  * precision form (N = 96): the split rhs and the FP64 rhs against the oracle
    on identical FP64 flow states along the flow, and the divergence
    temperature of the split flow against the FP64 flow's;
  * batched form: 256 flows (64 each of N = 32, 48, 64, 96, 256 points per
    patch, parameters drawn from the seed) batched in split precision against
    the same flows run one at a time in FP64;
  * large (N = 192): 30 accepted DP5(4) steps, split against FP64.
"""
import json
import math
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_1510_07799_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1510_07799_amd import frg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ST_SC, ST_SC_INTERP = 8, 9


def nrel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def opts_of(cfg, prec, **over):
    f = dict(I.CONFIGS[cfg]["flow"])
    f.update(over)
    return frg.flow_opts(f.pop("stepper"), prec, **f)


def step_through(g, o, V, on_accept=None, cap=2000):
    """Drive a flow with frg_flow_step, calling on_accept(state) after every
    accepted step; returns the final state."""
    st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
    g.flow_init(o, V, st)
    acc = 0
    for _ in range(cap):
        g.flow_step(o, V, st)
        s = st.cpu().numpy()
        if s[frg.ST_ACCEPTED] > acc:
            acc = int(s[frg.ST_ACCEPTED])
            if on_accept:
                on_accept(s)
        if s[frg.ST_REASON] != 0:
            return s
    raise AssertionError("flow did not stop")


def test_c2_flow_matches_the_oracle_flow_and_rhs_at_every_accepted_state():
    gold = json.load(open(os.path.join(HERE, "golden", "c2_flow_oracle.json")))
    p = gold["params"]
    m, g = O.Model(**p), frg.Context(**p)
    N, U = p["N"], p["U"]
    o = opts_of("C2", frg.PREC_FP64)
    V = torch.full((N, N, N), float(U), dtype=torch.float64, device="cuda")
    rows, errs = [], []

    def check(s):
        T = math.exp(s[frg.ST_S])
        rows.append([s[frg.ST_S], s[frg.ST_VMAX], s[frg.ST_RHS], s[frg.ST_REJECTED]])
        Vh = V.cpu().numpy()
        ref = m.rhs(T, Vh)
        e64 = nrel(g.rhs(T, V, frg.PREC_FP64).cpu().numpy(), ref)
        esp = nrel(g.rhs(T, V, frg.PREC_SPLIT_BF16).cpu().numpy(), ref)
        errs.append((T, e64, esp))

    s = step_through(g, o, V, check)
    log = np.array(gold["log"])
    res = gold["result"]
    print(f"[C2] accepted {int(s[frg.ST_ACCEPTED])} / oracle {res['accepted']}, rejected "
          f"{int(s[frg.ST_REJECTED])} / {res['rejected']}, reason {int(s[frg.ST_REASON])} / {res['reason']}",
          flush=True)
    e64 = max(e[1] for e in errs)
    esp = max(e[2] for e in errs)
    print(f"[C2] rhs at {len(errs)} accepted states: FP64 worst {e64:.2e}, split worst {esp:.2e}; "
          f"T from {errs[0][0]:.4g} to {errs[-1][0]:.4g}", flush=True)
    for T, a, b in errs[:: max(1, len(errs) // 8)] + errs[-1:]:
        print(f"[C2]   T={T:.5g}: FP64 {a:.2e} split {b:.2e}", flush=True)
    assert int(s[frg.ST_REASON]) == res["reason"]
    assert int(s[frg.ST_ACCEPTED]) == res["accepted"] and int(s[frg.ST_REJECTED]) == res["rejected"]
    got = np.array(rows)
    assert np.abs(got[:, 0] - log[:, 0]).max() <= 1e-9
    assert np.abs(got[:, 1] - log[:, 3]).max() <= 1e-8 * np.abs(log[:, 3]).max()
    if res["s_c"] is not None:
        print(f"[C2] T_c {math.exp(s[ST_SC]):.9g} / oracle {math.exp(res['s_c']):.9g}; interpolated "
              f"{math.exp(s[ST_SC_INTERP]):.9g} / {math.exp(res['s_c_interp']):.9g}", flush=True)
        assert abs(s[ST_SC] - res["s_c"]) <= 1e-9
        assert abs(s[ST_SC_INTERP] - res["s_c_interp"]) <= 1e-9
    idx = np.array(gold["sample_entries"])
    Vf = V.cpu().numpy()[idx[:, 0], idx[:, 1], idx[:, 2]]
    ev = np.abs(Vf - np.array(gold["sample_values"])).max() / gold["final_max_abs_V"]
    print(f"[C2] final V on {len(idx)} seeded entries: {ev:.2e} of max|V|", flush=True)
    assert ev <= 1e-8
    assert e64 <= 1e-10 and esp <= 2e-4


def test_c3_split_against_oracle_on_fp64_flow_states_and_tc():
    p = I.model_params("C3")
    N, U = p["N"], p["U"]
    g = frg.Context(**p)
    g.set_vsym(True)
    o64 = opts_of("C3", frg.PREC_FP64)
    V = torch.full((N, N, N), float(U), dtype=torch.float64, device="cuda")
    states = []
    s64 = step_through(g, o64, V, lambda s: states.append((math.exp(s[frg.ST_S]), s[frg.ST_VMAX],
                                                            V.cpu().numpy())))
    n = len(states)
    print(f"[C3] FP64 flow: {n} accepted steps, reason {int(s64[frg.ST_REASON])}, "
          f"T_c {math.exp(s64[ST_SC]):.6g} (interpolated {math.exp(s64[ST_SC_INTERP]):.6g})", flush=True)
    # the split flow of the same workload: the same stop; the divergence
    # temperature if it diverges, else the vertex at T_min
    Vs = torch.full((N, N, N), float(U), dtype=torch.float64, device="cuda")
    ssp = step_through(g, opts_of("C3", frg.PREC_SPLIT_BF16), Vs)
    print(f"[C3] split flow: {int(ssp[frg.ST_ACCEPTED])} accepted steps, reason {int(ssp[frg.ST_REASON])}, "
          f"T_c {math.exp(ssp[ST_SC]):.6g} (interpolated {math.exp(ssp[ST_SC_INTERP]):.6g})", flush=True)
    assert int(ssp[frg.ST_REASON]) == int(s64[frg.ST_REASON])
    if int(s64[frg.ST_REASON]) == frg.STOP_DIVERGED:
        dtc = abs(math.exp(ssp[ST_SC_INTERP]) - math.exp(s64[ST_SC_INTERP])) / math.exp(s64[ST_SC_INTERP])
        print(f"[C3] relative T_c difference split / FP64: {dtc:.2e}", flush=True)
        assert dtc <= 1e-3
    else:
        ev = nrel(Vs.cpu().numpy(), V.cpu().numpy())
        print(f"[C3] no divergence above T_min = {math.exp(s64[frg.ST_S]):.3g}: max|V| {s64[frg.ST_VMAX]:.4g} "
              f"(FP64) / {ssp[frg.ST_VMAX]:.4g} (split); split final V normwise {ev:.2e}", flush=True)
        assert ev <= 1e-3
    # split and FP64 rhs against the oracle on identical FP64 states along the flow
    m = O.Model(**p)
    picks = sorted(set([0, n // 3, (2 * n) // 3, n - 2, n - 1]))
    worst = [0.0, 0.0]
    for k in picks:
        T, vmax, Vh = states[k]
        ref = m.rhs(T, Vh)
        Vd = torch.from_numpy(Vh).cuda()
        scale = np.abs(ref).max()
        row = []
        for prec in (frg.PREC_FP64, frg.PREC_SPLIT_BF16):
            got = g.rhs(T, Vd, prec).cpu().numpy()
            d = np.abs(got - ref)
            big = np.abs(ref) >= 1e-3 * scale
            row.append((d.max() / scale, d.max(), (d[big] / np.abs(ref[big])).max()))
        print(f"[C3] step {k + 1}/{n} T={T:.5g} max|V|={vmax:.3g}: FP64 normwise {row[0][0]:.2e} "
              f"max-abs {row[0][1]:.2e} rel {row[0][2]:.2e}; split normwise {row[1][0]:.2e} "
              f"max-abs {row[1][1]:.2e} rel {row[1][2]:.2e}", flush=True)
        worst = [max(worst[0], row[0][0]), max(worst[1], row[1][0])]
    assert worst[0] <= 1e-10
    assert worst[1] <= 2e-4


@pytest.mark.timeout(900)
def test_c4_batched_split_flows_against_single_fp64_flows():
    draws = I.c4_flows()
    assert len(draws) == 256
    o_sp = frg.flow_opts("dp54", frg.PREC_SPLIT_BF16, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10, vmax=20.0,
                         h0=-0.01)
    o_64 = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10, vmax=20.0,
                         h0=-0.01)
    eqv = [(d["N"] / 96.0) ** 5 for d in draws]   # N = 96-equivalent work per rhs (the contraction's N^5)
    t0 = time.perf_counter()
    b = frg.Batch(draws)
    t_setup = time.perf_counter() - t0
    try:
        b.set_vsym(True)
        Vb = [torch.full((d["N"],) * 3, float(d["U"]), dtype=torch.float64, device="cuda") for d in draws]
        t0 = time.perf_counter()
        rb, _ = b.flow(Vb, o_sp)
        t_batch = time.perf_counter() - t0
    finally:
        b.close()
    Vbh = [v.cpu().numpy() for v in Vb]
    del Vb
    torch.cuda.empty_cache()
    # the same batch in FP64: follows the single FP64 flows to rounding
    b = frg.Batch(draws)
    try:
        b.set_vsym(True)
        Vb = [torch.full((d["N"],) * 3, float(d["U"]), dtype=torch.float64, device="cuda") for d in draws]
        t0 = time.perf_counter()
        rb64, _ = b.flow(Vb, o_64)
        t_batch64 = time.perf_counter() - t0
    finally:
        b.close()
    Vb64h = [v.cpu().numpy() for v in Vb]
    del Vb
    torch.cuda.empty_cache()
    rs, t_single, dtc, dv, d64 = [], 0.0, [], [], []
    for i, d in enumerate(draws):
        g = frg.Context(**d)
        g.set_vsym(True)
        V = torch.full((d["N"],) * 3, float(d["U"]), dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        r, _ = g.flow(V, o_64)
        t_single += time.perf_counter() - t0
        rs.append(r)
        g.close()
        Vh = V.cpu().numpy()
        if rb64[i]["reason"] == r["reason"] and rb64[i]["accepted"] == r["accepted"]:
            d64.append(nrel(Vb64h[i], Vh))
        else:
            d64.append(float("inf"))
        if rb[i]["reason"] != r["reason"]:
            # only a flow whose divergence sits at T_min itself may stop differently
            tc = r["T_c_interp"] if r["reason"] == frg.STOP_DIVERGED else rb[i]["T_c_interp"]
            assert abs(math.log(tc / 1e-3)) < 0.01, (i, d, rb[i], r)
            continue
        if r["reason"] == frg.STOP_DIVERGED:
            dtc.append(abs(rb[i]["T_c_interp"] - r["T_c_interp"]) / r["T_c_interp"])
        else:
            dv.append(nrel(Vbh[i], Vh))
    eq_b = sum(e * r["rhs_evals"] for e, r in zip(eqv, rb))
    eq_b64 = sum(e * r["rhs_evals"] for e, r in zip(eqv, rb64))
    eq_s = sum(e * r["rhs_evals"] for e, r in zip(eqv, rs))
    ndiv = sum(1 for r in rs if r["reason"] == frg.STOP_DIVERGED)
    print(f"[C4] 256 flows: {ndiv} diverge, {256 - ndiv} reach T_min; batch set-up {t_setup:.1f} s", flush=True)
    print(f"[C4] batched split: {t_batch:.2f} s, {eq_b / t_batch:.0f} N=96-equivalent rhs/s; batched FP64: "
          f"{t_batch64:.2f} s, {eq_b64 / t_batch64:.0f}; one at a time FP64: {t_single:.2f} s, "
          f"{eq_s / t_single:.0f} N=96-equivalent rhs/s", flush=True)
    n_same = sum(1 for x in d64 if x != float("inf"))
    print(f"[C4] batched FP64 vs one at a time FP64: {n_same}/256 flows with the same steps, final V max "
          f"normwise difference {max(x for x in d64 if x != float('inf')):.2e}", flush=True)
    assert n_same >= 254
    assert max(x for x in d64 if x != float("inf")) <= 1e-8
    if dtc:
        # the split rhs rounding (~1e-6 relative) is of the size of rtol = 1e-6, so the
        # two precisions take different step sequences; the interpolated crossing
        # carries the interpolation error of each run's own steps
        print(f"[C4] relative T_c difference (interpolated), split batch vs FP64 single: max {max(dtc):.2e} "
              f"median {float(np.median(dtc)):.2e}", flush=True)
        assert float(np.median(dtc)) <= 1e-3 and max(dtc) <= 1e-2
    if dv:
        print(f"[C4] final V of flows reaching T_min: max normwise difference {max(dv):.2e}", flush=True)
        assert max(dv) <= 1e-3


def test_c5_thirty_steps_split_against_fp64():
    """30 accepted DP5(4) steps of the FP64 flow; the split flow of the same
    workload is then run to the temperature the FP64 flow reached (its last step
    clipped onto it) and the two vertices are compared there.  The step
    sequences themselves differ: the split rounding is of the size of rtol."""
    p = I.model_params("C5")
    N, U = p["N"], p["U"]
    g = frg.Context(**p)
    g.set_vsym(True)
    V64 = torch.full((N, N, N), float(U), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    r64, l64 = g.flow(V64, opts_of("C5", frg.PREC_FP64))
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    assert r64["accepted"] == 30 or r64["reason"] == frg.STOP_DIVERGED
    Vsp = torch.full((N, N, N), float(U), dtype=torch.float64, device="cuda")
    T_end = r64["T_end"]
    t0 = time.perf_counter()
    rsp, lsp = g.flow(Vsp, opts_of("C5", frg.PREC_SPLIT_BF16, T_min=T_end, max_steps=0))
    torch.cuda.synchronize()
    tsp = time.perf_counter() - t0
    Va, Vb = V64.cpu().numpy(), Vsp.cpu().numpy()
    ev = nrel(Vb, Va)
    print(f"[C5] FP64: {r64['accepted']} accepted steps to T = {T_end:.6g} in {t64:.1f} s; split to the same T: "
          f"{rsp['accepted']} accepted, {tsp:.1f} s; max|V| {np.abs(Va).max():.4g}; split V normwise {ev:.2e}",
          flush=True)
    if r64["reason"] != frg.STOP_DIVERGED:
        assert rsp["reason"] == frg.STOP_TMIN and rsp["T_end"] == pytest.approx(T_end, rel=1e-12)
        assert ev <= 1e-3
