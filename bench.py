#!/usr/bin/env python3
"""Benchmark: fRG rhs evaluations per second at N = 96 on one MI355X.

Workload: 2D Hubbard model, N = 96 patches, 512 fine points per patch
(32 radial x 16 angular), t' = -0.3, mu = -1.2 (van Hove filling), U = 3.
One timed step is one Dormand-Prince 5(4) step of the temperature flow run
entirely on the device: six rhs evaluations (bubble sweep, operand layout,
the fused channel contraction, combine) plus the FP64 stage sums, error norm
and step control.  The split-BF16 and FP64 paths of one flow, and batches of
16 flows in either precision, are timed in regions of their own; `value` is the
batched leg's split-BF16 rhs evaluations per second (16 flows at N = 96 stepped
together).  `ratios` holds the like-for-like speed-ups (both sides computing one
contraction column per C4v orbit); `symmetric_vertex_gain` the speed-up of that
reduction itself over computing every column.  `roofline` describes the
dominant kernel of the batched leg.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per process).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

RHS_PER_STEP = 6   # DP5(4) with first-same-as-last: six new stages per step
PEAK = {"hbm_GBs": 8000.0, "bf16_TFLOPs": 2500.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3,
        "valu_TFLOPs": 78.6}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def progress(msg: str) -> None:
    """one line per finished leg on stderr (stdout carries the single JSON line)"""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    # the kernels and the host code that builds their work lists and launch shapes
    for f in ("k_contract.hip", "k_bubbles.hip", "abi.cpp"):
        with open(os.path.join(ROOT, "paper_1510_07799_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PROFILE_STEPS = 3   # extra steps timed per kernel class (eager launches, events between kernels)


def timed_flow_steps(frg, torch, ctx, prec, V0, steps, warmup):
    """DP5(4) steps of the temperature flow: `steps` timed as the library runs
    them (one captured graph replayed per step), then PROFILE_STEPS more with
    per-kernel-class HIP events (launched eagerly) for the breakdown."""
    opts = frg.flow_opts("dp54", prec, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    V = V0.clone()
    state = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
    ctx.flow_init(opts, V, state)
    for _ in range(warmup):
        ctx.flow_step(opts, V, state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.flow_step(opts, V, state)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile_begin()
    for _ in range(PROFILE_STEPS):
        ctx.flow_step(opts, V, state)
    torch.cuda.synchronize()
    prof = ctx.profile_end()
    st = state.cpu().numpy()
    return t1 - t0, prof, st


def timed_iflow_steps(frg, torch, ctx, prec, V0, T, steps, warmup):
    """DP5(4) steps of the interaction flow (bubbles once at T, contraction-only
    rhs), timed as timed_flow_steps does."""
    opts = frg.iflow_opts("dp54", prec, T=T, rtol=1e-6, atol=1e-10, vmax=20.0, h0=0.01)
    V = V0.clone()
    state = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
    ctx.iflow_init(opts, V, state)
    for _ in range(warmup):
        ctx.iflow_step(opts, V, state)
    torch.cuda.synchronize()
    rhs0 = float(state[frg.ST_RHS].item())
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.iflow_step(opts, V, state)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rhs1 = float(state[frg.ST_RHS].item())
    ctx.profile_begin()
    for _ in range(PROFILE_STEPS):
        ctx.iflow_step(opts, V, state)
    torch.cuda.synchronize()
    prof = ctx.profile_end()
    rhs2 = float(state[frg.ST_RHS].item())
    st = state.cpu().numpy()
    return t1 - t0, prof, rhs1 - rhs0, rhs2 - rhs1, st


def load_profiles():
    try:
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
    except (OSError, ValueError):
        return None
    return tr if tr.get("source_hash") == kernel_source_hash() else None


def rhs_micro(frg, torch, ctx, p, entry64, entry32, runs=50, warm=5):
    """frg_rhs alone at the benchmark workload, symmetric-vertex mode: HIP events
    recorded on the launch stream around each call, `warm` untimed and `runs`
    timed calls, median and 90th percentile.  State classes: (i) V = U; (ii)
    states of an FP64 DP5(4) flow from V = U at T = 1, the first past
    max|V| = 5 and 10 and the last one before the flow stops above 20 (the flow
    starts at max|V| = U = 3); (iii) a seeded
    C4v-symmetric V = U (1 + 0.5 eta), eta uniform on [-1, 1].  Each at
    T = 0.05 and 1e-3, FP64 and split; the split result is compared with the
    FP64 one on the same state (cost does not depend on V, the error does)."""
    from paper_1510_07799_amd import inputs as I
    from paper_1510_07799_amd import tuning as TU
    N, U = p["N"], float(p["U"])
    ctx.set_vsym(True)
    states = {"V=U": torch.full((N, N, N), U, dtype=torch.float64, device="cuda")}
    # (ii) flow states
    TU.apply(ctx, entry64)
    V = states["V=U"].clone()
    st = torch.zeros(frg.STATE_LEN, dtype=torch.float64, device="cuda")
    o = frg.flow_opts("dp54", frg.PREC_FP64, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
    ctx.flow_init(o, V, st)
    targets = [5.0, 10.0]
    last = None
    for _ in range(4000):
        ctx.flow_step(o, V, st)
        sh = st.cpu().numpy()
        if sh[frg.ST_REASON] != 0:
            break
        m = float(V.abs().max())
        last = (V.clone(), m, math.exp(sh[frg.ST_S]))
        while targets and m >= targets[0]:
            states[f"flow state past max|V|={targets[0]:g}"] = V.clone()
            targets.pop(0)
    if last is not None:
        states["last flow state before the stop at max|V| > 20"] = last[0]
    # (iii) random symmetric state
    states["U(1+0.5 eta)"] = torch.from_numpy(I.random_vertex(N, U, seed=151007799, amp=0.5,
                                                              symmetrise=True)).cuda()
    stream = torch.cuda.current_stream()
    out = {"protocol": f"frg_rhs alone, HIP events on the launch stream around each call, {warm} untimed "
                       f"+ {runs} timed calls; N=96, 512 points/patch, symmetric-vertex mode, tuned "
                       "parameters of one flow",
           "flow_T_at_last_state": round(last[2], 6) if last else None, "states": {}}
    F = {prec: torch.empty_like(states["V=U"]) for prec in (frg.PREC_FP64, frg.PREC_SPLIT_BF16)}
    for name, Vs in states.items():
        rec = {"max_abs_V": round(float(Vs.abs().max()), 4)}
        for T in (0.05, 1e-3):
            rt = {}
            for prec, nm, entry in ((frg.PREC_FP64, "fp64", entry64), (frg.PREC_SPLIT_BF16, "split", entry32)):
                TU.apply(ctx, entry)
                for _ in range(warm):
                    ctx.rhs(T, Vs, prec, out=F[prec])
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(runs)]
                for a, b in ev:
                    a.record(stream)
                    ctx.rhs(T, Vs, prec, out=F[prec])
                    b.record(stream)
                torch.cuda.synchronize()
                ms = sorted(a.elapsed_time(b) for a, b in ev)
                med, p90 = ms[len(ms) // 2], ms[min(len(ms) - 1, int(0.9 * len(ms)))]
                rt[nm] = {"median_ms": round(med, 4), "p90_ms": round(p90, 4), "rhs_per_s": round(1e3 / med, 1)}
            d = (F[frg.PREC_SPLIT_BF16] - F[frg.PREC_FP64]).abs()
            ref = float(F[frg.PREC_FP64].abs().max())
            rt["split_vs_fp64"] = {"max_abs": float(d.max()), "rel": float(d.max()) / ref if ref > 0 else None}
            rec[f"T={T:g}"] = rt
        out["states"][name] = rec
        progress(f"rhs micro {name}: max|V| {rec['max_abs_V']}, T=0.05 split "
                 f"{rec['T=0.05']['split']['median_ms']} ms, fp64 {rec['T=0.05']['fp64']['median_ms']} ms")
    return out


def bubble_roofline(avg_s, terms, energies, leg, kernel):
    """The sweep is bound by plain vector ALU work.  Algorithmic unit: 50 FP32
    operation-equivalents per dL/dT term (two cosines, two exponential-class
    operations, one division, ~30 flops, a projection and a compensated add),
    against the FP32 vector peak 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed)
    x 2.4 GHz = 157.3 TFLOP/s.  The build disables packed FP32, so 78.6 TFLOP/s is
    the rate its instructions can reach; frac_nonpacked states that view."""
    achieved = 50.0 * terms / avg_s / 1e12
    roof = {"kernel": kernel, "bound": "alu", "achieved": round(achieved, 4), "peak": PEAK["fp32_TFLOPs"],
            "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp32_TFLOPs"], 6),
            "frac_nonpacked": round(achieved / PEAK["valu_TFLOPs"], 6),
            "work": {"terms_per_launch": int(terms), "energies_per_launch": int(energies),
                     "op_equivalents_per_term": 50},
            "avg_launch_ms": round(avg_s * 1e3, 4)}
    tr = load_profiles()
    roof["traffic"] = None
    roof["valu_issue_frac"] = None
    if tr:
        k = tr.get("kernels", {}).get(leg, {}).get("bubbles")
        if k:
            roof["traffic"] = k["bytes_per_launch"]
        vb = tr.get("valu", {}).get(leg, {}).get("bubbles")
        if vb:
            # hardware view: VALU issue cycles (4 per wave64 instruction on a 16-lane
            # SIMD, 16 for a quarter-rate transcendental) over the 1024 SIMDs' cycles
            cyc = 4.0 * vb["insts_valu"] + 12.0 * vb["insts_trans_f32"]
            roof["valu_issue_frac"] = round(cyc / (1024 * avg_s * 2.4e9), 4)
    return roof


def contract_roofline(avg_s, algo_flops, dense_flops, exec_share, split, leg, kernel):
    """The contraction is a dense product on the matrix cores: algorithmic flops (N
    multiply-adds per structurally nonzero bubble entry per computed column)
    against the dense MFMA peak of its precision."""
    peak = PEAK["bf16_TFLOPs"] if split else PEAK["fp64_TFLOPs"]
    achieved = algo_flops / avg_s / 1e12
    passes = 3.0 if split else 1.0
    roof = {"kernel": kernel, "bound": "mfma", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 6),
            "executed_frac": round(passes * dense_flops * exec_share / avg_s / 1e12 / peak, 6),
            "kskip_executed_share": round(exec_share, 4), "avg_launch_ms": round(avg_s * 1e3, 4),
            "traffic": None}
    tr = load_profiles()
    if tr:
        k = tr.get("kernels", {}).get(leg, {}).get("contract")
        if k:
            roof["traffic"] = k["bytes_per_launch"]
    return roof


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU-baseline leg (default: every host core)")
    ap.add_argument("--cpu-only", action="store_true", help="run only the CPU-baseline leg")
    ap.add_argument("--legs", default="split,fp64,batch,batch_fp64,batch64,split_full,fp64_full,rhs,c4,iflow,egrid,se",
                    help="comma list of split, fp64 (one flow), batch, batch_fp64 (16 flows, split / FP64), "
                         "batch64 (64 flows, split), all in symmetric-vertex mode; split_full, fp64_full "
                         "(one flow, every column computed); iflow (the interaction flow of the paper's "
                         "working example, N=32); egrid (one flow at N=96 on the paper's quadrature: "
                         "1600 energies, adaptive inner rule); se (one flow at N=96 with the self-energy "
                         "flowing along: every bubble row, every column); rhs (frg_rhs alone, event-timed, "
                         "over V = U, FP64 flow states past max|V| 5, 10 and before the stop at 20, and "
                         "a random symmetric V, at "
                         "T = 0.05 and 1e-3); c4 (the mixed batch of 256 flows, N = 32..96, in N = 96-"
                         "equivalent rhs/s)")
    ap.add_argument("--batch-flows", type=int, default=16,
                    help="flows in the batched legs (N=96, 512 points/patch, drawn parameters)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (calibrates "
                         "the HBM byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        n = args.copy_calib // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "layout is a design note only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_1510_07799_amd import inputs as I

    p = I.model_params("C3")
    N = p["N"]
    if args.cpu_only:
        print(json.dumps({"cpu_baseline": cpu_baseline(args, p)}))
        return

    import torch
    from paper_1510_07799_amd import frg

    nf = p["n_rad"] * p["n_ang"]
    ctx = frg.Context(**p)
    V0 = torch.full((N, N, N), float(p["U"]), dtype=torch.float64, device="cuda")

    # algorithmic work per launch (T independent): bubble-row occupancy, i.e. the
    # (a, b) pairs of row t for which some fine point of patch a has its second
    # line in patch b (the structurally nonzero entries), counted from the
    # second-line tables so that no extra bubble sweep enters the profile
    def occupancy(kind):
        bins = ctx.bins(kind).to(torch.int64)
        rows = bins.shape[0]
        patch = torch.arange(N * nf, device="cuda") // nf
        key = (torch.arange(rows, device="cuda")[:, None] * N + patch[None, :]) * N + bins
        hit = torch.zeros(rows * N * N, dtype=torch.bool, device="cuda")
        hit[key.reshape(-1)] = True
        return hit.reshape(rows, N * N).sum(dim=1).to(torch.float64)
    nnz_pp, nnz_ph = occupancy(1), occupancy(0)
    rows_pp = torch.tensor([[min(i, j) * N - min(i, j) * (min(i, j) - 1) // 2 + abs(i - j)
                             for j in range(N)] for i in range(N)], device="cuda").reshape(-1)
    colsum_pp = float(nnz_pp[rows_pp].sum())
    # ph column (y, x) uses row of Q = k_x - k_y; every ordered pair occurs once, x == y uses row 0
    colsum_ph = float(nnz_ph[1:].sum() + N * nnz_ph[0])
    # pp: one product per column, phc: one, phd: two (N output rows each); with a
    # C4v-invariant vertex only one column per orbit is needed (every column of an
    # orbit has the same bubble-row occupancy)
    ctx.set_vsym(True)
    vsym_cols = ctx.vsym()[1]
    ctx.set_vsym(False)
    algo_full = 2.0 * N * colsum_pp + 2.0 * N * colsum_ph + 4.0 * N * colsum_ph
    algo_vsym = algo_full * vsym_cols / (N * N)
    dense_flops = 8.0 * N ** 5   # what the dense formulation executes (x3 passes in split mode)
    ctx.set_vsym(True)
    _, exec_share = ctx.kskip()   # share of the dense k chunks (all columns) the contraction visits
    # bubble terms one rhs evaluates (C4v-reduced rows) and second-line energies
    # (a pp row and the ph row of the opposite transfer share one energy)
    sym_rows = ctx.symmetry()[1]
    terms_per_rhs, energies_per_rhs = sym_rows * N * nf, sym_rows // 2 * N * nf

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    from paper_1510_07799_amd import tuning as TU
    table = TU.load()
    tuned = {}
    results = {}
    for leg in legs:
        if leg.startswith("batch") or leg in ("rhs", "c4", "iflow", "egrid", "se"):
            continue
        prec = frg.PREC_FP64 if leg.startswith("fp64") else frg.PREC_SPLIT_BF16
        orbit = not leg.endswith("_full")
        ctx.set_vsym(orbit)   # the flows start from V = U: C4v invariant
        entry = TU.lookup(N, nf, prec == frg.PREC_SPLIT_BF16, orbit, 1, table)
        TU.apply(ctx, entry)
        tuned[leg] = ctx.tuning()
        dt, prof, st = timed_flow_steps(frg, torch, ctx, prec, V0, args.steps, args.warmup)
        results[leg] = dict(seconds=dt, prof=prof, state=st)
        progress(f"leg {leg}: {RHS_PER_STEP * args.steps / dt:.1f} rhs/s")
    ctx.set_vsym(True)
    micro = None
    if "rhs" in legs:
        micro = rhs_micro(frg, torch, ctx, p, TU.lookup(N, nf, False, True, 1, table),
                          TU.lookup(N, nf, True, True, 1, table))
        ctx.set_vsym(True)

    def run_batch(nflows, prec):
        # batched workload at N = 96: (mu, t', U) from the seeded draws of the batched configuration
        draws = I.c4_flows(n_per_N=nflows, Ns=(96,), n_rad=p["n_rad"], n_ang=p["n_ang"])
        b = frg.Batch(draws)
        b.set_vsym(True)
        if TU.apply(b, TU.lookup(N, nf, prec == frg.PREC_SPLIT_BF16, True, nflows, table)):
            tuned[f"batch of {nflows} {'split' if prec == frg.PREC_SPLIT_BF16 else 'fp64'}"] = \
                TU.lookup(N, nf, prec == frg.PREC_SPLIT_BF16, True, nflows, table)
        sym = b.symmetry()
        Vs = [torch.full((N, N, N), float(d["U"]), dtype=torch.float64, device="cuda") for d in draws]
        o = frg.flow_opts("dp54", prec, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
        b.flow_init(Vs, o)
        for _ in range(args.warmup):
            b.flow_step()
        res0, _ = b.results()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.flow_step()
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        res1, _ = b.results()
        # per kernel class: a few more steps launched eagerly with events between the classes
        b.profile_begin()
        for _ in range(PROFILE_STEPS):
            b.flow_step()
        prof = b.profile_end()
        res2, _ = b.results()
        rhs_done = sum(r1["rhs_evals"] - r0["rhs_evals"] for r0, r1 in zip(res0, res1))
        rhs_prof = sum(r2["rhs_evals"] - r1["rhs_evals"] for r1, r2 in zip(res1, res2))
        out_b = dict(seconds=tb, rhs=rhs_done, flows=len(draws), prof=prof, rhs_prof=rhs_prof,
                     still_running=sum(1 for r in res1 if r["reason"] == 0),
                     mean_active=rhs_done / (RHS_PER_STEP * args.steps),
                     mean_active_prof=rhs_prof / (RHS_PER_STEP * PROFILE_STEPS),
                     reduced=sum(1 for a, _ in sym if a))
        b.close()
        del Vs
        torch.cuda.empty_cache()
        return out_b

    batches = {}
    for leg, nfl, prec in (("batch", args.batch_flows, frg.PREC_SPLIT_BF16),
                           ("batch_fp64", args.batch_flows, frg.PREC_FP64),
                           ("batch64", 64, frg.PREC_SPLIT_BF16)):
        if leg in legs:
            batches[leg] = run_batch(nfl, prec)
            progress(f"leg {leg}: {batches[leg]['rhs'] / batches[leg]['seconds']:.1f} rhs/s")

    c4 = None
    if "c4" in legs:
        # the mixed batch: 256 flows, 64 each of N = 32, 48, 64, 96 (16 x 16 points
        # per patch, drawn mu, t', U), symmetric-vertex mode, in N = 96-equivalent
        # work (the contraction's N^5)
        draws = I.c4_flows()
        eqv = [(d["N"] / 96.0) ** 5 for d in draws]
        t_c = time.perf_counter()
        b4 = frg.Batch(draws)
        t_c = time.perf_counter() - t_c
        b4.set_vsym(True)
        c4 = {"workload": "256 flows, 64 each of N=32,48,64,96, 16x16 points/patch, (mu, t', U) drawn as in "
                          "the batched configuration; DP5(4) steps from V=U at T=1, symmetric-vertex mode; "
                          "default launch parameters", "batch_create_s": round(t_c, 2)}
        for prec, nm in ((frg.PREC_SPLIT_BF16, "split"), (frg.PREC_FP64, "fp64")):
            Vs4 = [torch.full((d["N"],) * 3, float(d["U"]), dtype=torch.float64, device="cuda") for d in draws]
            o4 = frg.flow_opts("dp54", prec, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10, vmax=20.0, h0=-0.01)
            b4.flow_init(Vs4, o4)
            for _ in range(args.warmup):
                b4.flow_step()
            r0, _ = b4.results()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                b4.flow_step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            r1, _ = b4.results()
            d_rhs = [y["rhs_evals"] - x["rhs_evals"] for x, y in zip(r0, r1)]
            c4[nm] = {"n96_equivalent_rhs_per_s": round(sum(e * k for e, k in zip(eqv, d_rhs)) / dt, 1),
                      "rhs_per_s": round(sum(d_rhs) / dt, 1),
                      "mean_active_flows": round(sum(d_rhs) / (RHS_PER_STEP * args.steps), 2)}
            progress(f"leg c4 {nm}: {c4[nm]['n96_equivalent_rhs_per_s']:.1f} N=96-equivalent rhs/s")
            del Vs4
        b4.close()
        torch.cuda.empty_cache()

    iflow = None
    if "iflow" in legs:
        # the paper's working example: interaction flow at T = 0.1, t' = -0.01,
        # mu = -0.02, 32 patches (16 x 16 points each), from V = U; each rhs is
        # the contraction alone (the bubbles are computed once per flow)
        pi = I.model_params("P1")
        Ni = pi["N"]
        ci = frg.Context(**pi)
        ci.set_vsym(True)
        Vi = torch.full((Ni, Ni, Ni), float(pi["U"]), dtype=torch.float64, device="cuda")
        iflow = {}
        for prec, nm in ((frg.PREC_SPLIT_BF16, "split"), (frg.PREC_FP64, "fp64")):
            t_i, prof_i, rhs_i, rhs_p, st_i = timed_iflow_steps(frg, torch, ci, prec, Vi, 0.1, args.steps,
                                                                args.warmup)
            iflow[nm] = {"rhs_per_s": round(rhs_i / t_i, 3), "rhs_evaluated": int(rhs_i),
                         "g_reached": round(float(st_i[frg.ST_S]), 6),
                         "kernel_ms_per_rhs": {k: round(ms / max(1.0, rhs_p), 4) for k, (ms, c) in prof_i.items()
                                               if c}}
        ci.close()

    egrid = None
    if "egrid" in legs:
        # the paper's quadrature on the N = 96 model (split and FP64 single flows,
        # symmetric-vertex mode); the sweep walks each patch's live points
        pe = I.model_params("E1")
        Ne = pe["N"]
        t_c = time.perf_counter()
        ce = frg.Context(**pe)
        t_c = time.perf_counter() - t_c
        ce.set_vsym(True)
        live = int(ce.counts().sum())
        rows_e = ce.symmetry()[1]
        terms_e, energies_e = rows_e * live, rows_e // 2 * live
        Ve = torch.full((Ne, Ne, Ne), float(pe["U"]), dtype=torch.float64, device="cuda")
        egrid = {"workload": "N=96, t'=-0.3 mu=-1.2 U=3; paper's quadrature: 1600 midpoint energies across the "
                             "band, inner adaptive trisection midpoint rule in the ray angle per patch sector "
                             "(rtol 1e-4, at most 27 points per sector and shell); DP5(4) steps from V=U at T=1, "
                             "symmetric-vertex mode",
                 "points_per_patch_stride": ce.nf, "live_points": live, "context_create_s": round(t_c, 2)}
        for prec, nm in ((frg.PREC_SPLIT_BF16, "split"), (frg.PREC_FP64, "fp64")):
            dt, prof, st = timed_flow_steps(frg, torch, ce, prec, Ve, args.steps, args.warmup)
            ms, cnt = prof["bubbles"]
            progress(f"leg egrid {nm}: {RHS_PER_STEP * args.steps / dt:.1f} rhs/s")
            egrid[nm] = {"rhs_per_s": round(RHS_PER_STEP * args.steps / dt, 3),
                         "kernel_ms_per_rhs": {k: round(v / (PROFILE_STEPS * RHS_PER_STEP), 4)
                                               for k, (v, c) in prof.items()},
                         "bubble_roofline": bubble_roofline(ms / max(cnt, 1) * 1e-3, terms_e, energies_e,
                                                            "egrid_" + nm, "bubble_seg_kernel")}
        ce.close()
        del Ve
        torch.cuda.empty_cache()

    se_leg = None
    if "se" in legs:
        # the vertex and a self-energy per patch flowing together (N = 96, 512
        # points per patch): with the self-energy announced C4v invariant (the
        # flow from V = U, S = 0 keeps it so) as without one (bubble rows per C4v
        # orbit, paired; one contraction column per orbit; reduced flow state);
        # in the general mode every row and every column
        cs_ = frg.Context(**p)
        Vse = torch.cat([torch.full((N ** 3,), float(p["U"]), dtype=torch.float64, device="cuda"),
                         torch.zeros(N, dtype=torch.float64, device="cuda")]).contiguous()
        se_leg = {"workload": "N=96, 512 points/patch, t'=-0.3 mu=-1.2 U=3; vertex and self-energy per patch "
                              "flowing together (DP5(4) steps from V=U, S=0 at T=1); c4v_invariant_S: bubble "
                              "rows per C4v orbit, paired, one contraction column per orbit, reduced flow state; "
                              "general_S: every bubble row, every column"}
        for symmetric, mode in ((True, "c4v_invariant_S"), (False, "general_S")):
            cs_.set_self_energy(False)
            cs_.set_vsym(symmetric)
            cs_.set_self_energy(True, symmetric=symmetric)
            se_leg[mode] = {}
            for prec, nm in ((frg.PREC_SPLIT_BF16, "split"), (frg.PREC_FP64, "fp64")):
                TU.apply(cs_, TU.lookup(N, nf, prec == frg.PREC_SPLIT_BF16, symmetric, 1, table))
                dt, prof, st = timed_flow_steps(frg, torch, cs_, prec, Vse, args.steps, args.warmup)
                progress(f"leg se {mode} {nm}: {RHS_PER_STEP * args.steps / dt:.1f} rhs/s")
                se_leg[mode][nm] = {"rhs_per_s": round(RHS_PER_STEP * args.steps / dt, 3),
                                    "kernel_ms_per_rhs": {k: round(v / (PROFILE_STEPS * RHS_PER_STEP), 4)
                                                          for k, (v, c) in prof.items()}}
        cs_.close()
        del Vse
        torch.cuda.empty_cache()

    head = batches.get("batch")
    if head is None and not results:
        print(json.dumps({"rhs_micro": micro, "c4": c4, "iflow_p1": iflow, "egrid": egrid, "se": se_leg}))
        return
    rate = {leg: RHS_PER_STEP * args.steps / r["seconds"] for leg, r in results.items()}
    rate.update({leg: bb["rhs"] / bb["seconds"] for leg, bb in batches.items()})
    if head is not None:
        value, ms_step = rate["batch"], 1e3 * head["seconds"] / args.steps
    else:
        leg0 = next(iter(results))
        value, ms_step = rate[leg0], 1e3 * results[leg0]["seconds"] / args.steps
    out = {
        "metric": "fRG rhs evals/sec at N=96 (split-BF16 vs FP64, same GPU); % MFMA/HBM roofline",
        "value": round(value, 3),
        "unit": "rhs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-fp32",
        "data": "synthetic",
        "config": {"workload": "hubbard-2d N=96 patches, 512 fine points/patch (32x16), DP5(4) temperature "
                               "flow steps (6 rhs each) from V=U at T=1; value = batched split-BF16 rhs/s of "
                               f"{args.batch_flows} flows at N=96 with (mu, t', U) drawn as in the batched "
                               "configuration; single-flow legs at t'=-0.3 mu=-1.2 U=3",
                   "N": N, "n_f": nf, "rhs_per_step": RHS_PER_STEP, "parallelism": "1 GPU",
                   "symmetry": f"C4v: bubble rows per transfer orbit; vertex C4v invariant, {vsym_cols} of "
                               f"{N * N} columns per channel computed ({vsym_cols * N} independent entries); "
                               "the *_every_column legs compute all columns"},
    }
    out["config"]["tuning"] = {"table": "paper_1510_07799_amd/tuning.json" if table else None, "applied": tuned}
    names = {"split_full": "split_every_column", "fp64_full": "fp64_every_column"}
    for leg, r in results.items():
        nm = names.get(leg, leg)
        out[f"{nm}_rhs_per_s"] = round(rate[leg], 3)
        out[f"{nm}_kernel_ms_per_rhs"] = {
            k: round(ms / (PROFILE_STEPS * RHS_PER_STEP), 4) for k, (ms, c) in r["prof"].items()}
    for leg, bb in batches.items():
        out[f"{leg}_rhs_per_s"] = round(rate[leg], 3)
        out[leg] = {"flows": bb["flows"], "rhs_evaluated": bb["rhs"], "seconds": round(bb["seconds"], 4),
                    "mean_active_flows": round(bb["mean_active"], 3), "flows_running_at_end": bb["still_running"],
                    "flows_with_c4v_reduction": bb["reduced"],
                    "kernel_ms_per_flow_rhs": {k: round(ms / max(1, bb["rhs_prof"]), 4)
                                               for k, (ms, c) in bb["prof"].items()}}
    # like-for-like ratios (both sides in the same symmetric-vertex mode); the target
    # reading is batched split over one FP64 flow
    ratios = {}
    if "fp64" in rate:
        if "split" in rate:
            ratios["split_over_fp64"] = round(rate["split"] / rate["fp64"], 3)
        if "batch" in rate:
            ratios["batch_split_over_fp64"] = round(rate["batch"] / rate["fp64"], 3)
        if "batch64" in rate:
            ratios["batch64_split_over_fp64"] = round(rate["batch64"] / rate["fp64"], 3)
    if "batch" in rate and "batch_fp64" in rate:
        ratios["batch_split_over_batch_fp64"] = round(rate["batch"] / rate["batch_fp64"], 3)
    if ratios:
        ratios["target"] = "batch_split_over_fp64 >= 10"
        out["ratios"] = ratios
    # what the triple-orbit reduction (one contraction column per C4v orbit) gains,
    # apart from precision
    gain = {}
    for a, b_ in (("split", "split_full"), ("fp64", "fp64_full")):
        if a in rate and b_ in rate:
            gain[a] = round(rate[a] / rate[b_], 3)
    if gain:
        out["symmetric_vertex_gain"] = gain

    if iflow is not None:
        out["iflow_p1"] = dict(iflow, workload="interaction flow at T=0.1, N=32, 16x16 points/patch, "
                                               "t'=-0.01 mu=-0.02, bare U(g=1)=2, DP5(4) steps from V=U, "
                                               "symmetric-vertex mode; bubbles once per flow")

    if micro is not None:
        out["rhs_micro"] = micro
    if c4 is not None:
        out["c4_mixed_batch"] = c4
    if egrid is not None:
        out["egrid_e1"] = egrid
    if se_leg is not None:
        out["self_energy"] = se_leg

    # roofline of the dominant kernel of the value leg (the batched sweep), from the
    # event-timed steps: one launch covers every active flow
    if head is not None:
        ms, cnt = head["prof"]["bubbles"]
        act = head["mean_active_prof"]
        out["roofline"] = bubble_roofline(ms / max(cnt, 1) * 1e-3, act * terms_per_rhs, act * energies_per_rhs,
                                          "batch", "bubble_kernel_batched")
        ms, cnt = head["prof"]["contract"]
        out["contract_roofline"] = contract_roofline(ms / max(cnt, 1) * 1e-3, act * algo_vsym, act * dense_flops,
                                                     exec_share, True, "batch", "contract_items")
    single = {}
    for leg in ("split", "fp64"):
        if leg in results:
            pr = results[leg]["prof"]
            ms, cnt = pr["bubbles"]
            single[f"{leg}_bubbles"] = bubble_roofline(ms / max(cnt, 1) * 1e-3, terms_per_rhs, energies_per_rhs,
                                                       leg, "bubble_kernel")
            ms, cnt = pr["contract"]
            single[f"{leg}_contract"] = contract_roofline(ms / max(cnt, 1) * 1e-3, algo_vsym, dense_flops,
                                                          exec_share, leg == "split", leg, "contract_fused")
    if single:
        out["single_flow_rooflines"] = single
    if head is None and single:
        out["roofline"] = single.get("split_bubbles") or next(iter(single.values()))

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, p)
    print(json.dumps(out))


def cpu_baseline(args, p):
    """The oracle as it stands: one full FP64 rhs (bubbles and contraction) at the
    benchmark workload on the host's cores."""
    import numpy as np
    import oracle as O
    O.build(force=False)
    cores = os.cpu_count() or 1
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    if args.cpu_threads > 0:
        cores = args.cpu_threads
    O.set_threads(cores)
    m = O.Model(**p)
    N = p["N"]
    Vh = np.full((N, N, N), float(p["U"]))
    # the oracle's rhs is its bubbles then its contraction: timed as the two calls
    t0 = time.perf_counter()
    Bpp, Bph = m.bubbles(0.05)
    t1 = time.perf_counter()
    progress(f"cpu baseline: oracle bubbles {t1 - t0:.1f} s on {cores} threads")
    m.contract(Bpp, Bph, Vh)
    t_cpu = time.perf_counter() - t0
    progress(f"cpu baseline: oracle contraction {t_cpu - (t1 - t0):.1f} s")
    out = {"value": round(1.0 / t_cpu, 6), "unit": "rhs/s", "cores": cores, "kind": "oracle",
           "sample": "one full FP64 oracle rhs at the benchmark workload (N=96, 512 points/patch, T=0.05): "
                     "bubbles + contraction", "cpu_model": cpu_model(), "seconds": round(t_cpu, 3),
           "bubbles_seconds": round(t1 - t0, 3)}
    one = os.path.join(ROOT, "profiles", "cpu_oracle_n96.json")
    if args.cpu_threads == 0 and os.path.exists(one):
        with open(one) as fh:
            rec = json.load(fh)
        out["one_thread"] = {"value": rec["cpu_baseline"]["value"], "cpu_model": rec["cpu_baseline"]["cpu_model"],
                             "source": "profiles/cpu_oracle_n96.json (bench.py --cpu-only --cpu-threads 1)"}
    return out


if __name__ == "__main__":
    main()
