#!/usr/bin/env python3
"""Benchmark: fRG rhs evaluations per second at N = 96 on one MI355X.

Workload: 2D Hubbard model, N = 96 patches, 512 fine points per patch
(32 radial x 16 angular), t' = -0.3, mu = -1.2 (van Hove filling), U = 3.
One timed step is one Dormand-Prince 5(4) step of the temperature flow run
entirely on the device: six rhs evaluations (bubble sweep, operand layout,
the fused channel contraction, combine) plus the FP64 stage sums, error norm
and step control.  The split-BF16 and FP64 paths of one flow are timed in
regions of their own; `value` is the batched leg's split-BF16 rhs evaluations
per second (16 flows at N = 96 stepped together), the single-flow rates are
reported beside it.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per process).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

RHS_PER_STEP = 6   # DP5(4) with first-same-as-last: six new stages per step
PEAK = {"hbm_GBs": 8000.0, "bf16_TFLOPs": 2500.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3,
        "valu_TFLOPs": 78.6}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_contract.hip", "k_bubbles.hip"):
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


def roofline(head, results, algo_flops, dense_flops, exec_share, evals_per_rhs, kernel=None):
    prof = head["prof"]
    dom = kernel or max(prof, key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    avg_s = ms / max(cnt, 1) * 1e-3
    leg_name = "split" if "split" in results else [k for k in results][0]
    if dom.startswith("contract"):
        peak = PEAK["bf16_TFLOPs"] if leg_name == "split" else PEAK["fp64_TFLOPs"]
        achieved = algo_flops[dom] / avg_s / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 4), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 6)}
        passes = 3.0 if leg_name == "split" else 1.0
        roof["executed_frac"] = round(passes * dense_flops * exec_share / avg_s / 1e12 / peak, 6)
        roof["kskip_executed_share"] = round(exec_share, 4)
    elif dom == "bubbles":
        # plain ALU bound: vector FMA issue without packed FP32 (the build disables it),
        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s for FP32 and FP64.
        # Algorithmic work (flop-equivalents: FMA 2, a transcendental 4): per second-line
        # energy 12 (FP64 eps) + 9 (exp(-2|b|) and the terms a pair shares), per bubble
        # term 10 (its divided difference's own division and the run add); the
        # unshared Taylor branch is not counted
        peak = PEAK["valu_TFLOPs"]
        energies, terms = evals_per_rhs
        achieved = (21.0 * energies + 10.0 * terms) / avg_s / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 4), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 6),
                "work": {"energies_per_launch": energies, "terms_per_launch": terms}}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK["hbm_GBs"],
                "unit": "GB/s", "frac": None}
    roof["avg_launch_ms"] = round(avg_s * 1e3, 4)
    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        per_leg = tr.get("kernels", {}).get(leg_name, {})
        if tr.get("source_hash") == kernel_source_hash() and dom in per_leg:
            traffic = per_leg[dom]["bytes_per_launch"]
    except (OSError, ValueError):
        traffic = None
    roof["traffic"] = traffic
    if dom == "bubbles":
        # hardware view from the profiler's instruction counts (same kernel sources):
        # VALU issue cycles (4 per wave64 instruction on a 16-lane SIMD, 16 for a
        # quarter-rate transcendental) over the 1024 SIMDs' cycles at 2.4 GHz
        roof["valu_issue_frac"] = None
        try:
            with open(TRAFFIC_FILE) as fh:
                tr = json.load(fh)
            vb = tr.get("valu", {}).get(leg_name, {}).get("bubbles")
            if tr.get("source_hash") == kernel_source_hash() and vb:
                cyc = 4.0 * vb["insts_valu"] + 12.0 * vb["insts_trans_f32"]
                roof["valu_issue_frac"] = round(cyc / (1024 * avg_s * 2.4e9), 4)
        except (OSError, ValueError, KeyError):
            pass
    return roof


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="split,fp64,batch,batch64,split_full,fp64_full,iflow",
                    help="comma list of split, fp64, batch (16 flows), batch64 (64 flows) in "
                         "symmetric-vertex mode; split_full, fp64_full (every column computed); "
                         "iflow (the interaction flow of the paper's working example, N=32)")
    ap.add_argument("--batch-flows", type=int, default=16,
                    help="flows in the batched leg (N=96, 512 points/patch, drawn parameters)")
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
    import torch
    from paper_1510_07799_amd import frg, inputs as I

    p = I.model_params("C3")
    N = p["N"]
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
    algo_flops = {"contract": algo_full * vsym_cols / (N * N)}
    dense_flops = 8.0 * N ** 5   # what the dense formulation executes (x3 passes in split mode)
    ctx.set_vsym(True)
    _, exec_share = ctx.kskip()   # share of the dense k chunks (all columns) the contraction visits
    # bubble terms one rhs evaluates (C4v-reduced rows) and second-line energies
    # (a pp row and the ph row of the opposite transfer share one energy)
    sym_rows = ctx.symmetry()[1]
    evals_per_rhs = (sym_rows // 2 * N * nf, sym_rows * N * nf)

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    results = {}
    for leg in legs:
        if leg in ("batch", "batch64", "iflow"):
            continue
        prec = frg.PREC_FP64 if leg.startswith("fp64") else frg.PREC_SPLIT_BF16
        ctx.set_vsym(not leg.endswith("_full"))   # the flows start from V = U: C4v invariant
        dt, prof, st = timed_flow_steps(frg, torch, ctx, prec, V0, args.steps, args.warmup)
        results[leg] = dict(seconds=dt, prof=prof, state=st)
    ctx.set_vsym(True)
    batch = None
    def run_batch(nflows):
        # batched workload at N = 96: (mu, t', U) from the seeded draws of the batched configuration
        draws = I.c4_flows(n_per_N=nflows, Ns=(96,), n_rad=p["n_rad"], n_ang=p["n_ang"])
        b = frg.Batch(draws)
        b.set_vsym(True)
        sym = b.symmetry()
        Vs = [torch.full((N, N, N), float(d["U"]), dtype=torch.float64, device="cuda") for d in draws]
        o = frg.flow_opts("dp54", frg.PREC_SPLIT_BF16, T0=1.0, T_min=1e-3, rtol=1e-6, atol=1e-10,
                          vmax=20.0, h0=-0.01)
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
        active_steps = sum(1 for r in res1 if r["reason"] == 0)
        rhs_done = sum(r1["rhs_evals"] - r0["rhs_evals"] for r0, r1 in zip(res0, res1))
        out_b = dict(seconds=tb, rhs=rhs_done, flows=len(draws), still_running=active_steps,
                     reduced=sum(1 for a, _ in sym if a))
        b.close()
        del Vs
        torch.cuda.empty_cache()
        return out_b

    batch = run_batch(args.batch_flows) if "batch" in legs else None
    batch64 = run_batch(64) if "batch64" in legs else None

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

    head = results.get("split") or (results[next(iter(results))] if results else None)
    if head is None and batch is None:
        print(json.dumps({"iflow_p1": iflow}))
        return
    dt = head["seconds"] if head else batch["seconds"]
    value = RHS_PER_STEP * args.steps / dt
    if batch is not None:
        value = batch["rhs"] / batch["seconds"]
    out = {
        "metric": "fRG rhs evals/sec at N=96 (split-BF16 vs FP64, same GPU); % MFMA/HBM roofline",
        "value": round(value, 3),
        "unit": "rhs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-fp32" if "split" in results else "f64",
        "data": "synthetic",
        "config": {"workload": "hubbard-2d N=96 patches, 512 fine points/patch (32x16), "
                               "t'=-0.3 mu=-1.2 U=3, DP5(4) temperature flow step (6 rhs) from V=U",
                   "N": N, "n_f": nf, "rhs_per_step": RHS_PER_STEP, "parallelism": "1 GPU",
                   "symmetry": f"C4v: bubble rows per transfer orbit; vertex C4v invariant, "
                               f"{vsym_cols} of {N * N} columns per channel computed "
                               f"({vsym_cols * N} independent entries; split_full and fp64_full compute all)"},
    }
    for leg, r in results.items():
        rps = RHS_PER_STEP * args.steps / r["seconds"]
        out[f"{leg}_rhs_per_s"] = round(rps, 3)
        out[f"{leg}_kernel_ms_per_rhs"] = {
            k: round(ms / (PROFILE_STEPS * RHS_PER_STEP), 4) for k, (ms, c) in r["prof"].items()}
    if "split" in results and "fp64" in results:
        out["split_over_fp64"] = round(out["split_rhs_per_s"] / out["fp64_rhs_per_s"], 3)
    if batch is not None:
        out["batch_split_rhs_per_s"] = round(batch["rhs"] / batch["seconds"], 3)
        out["batch"] = {"flows": batch["flows"], "rhs_evaluated": batch["rhs"],
                        "seconds": round(batch["seconds"], 4),
                        "flows_running_at_end": batch["still_running"],
                        "flows_with_c4v_reduction": batch["reduced"]}
        if "fp64" in results:
            out["batch_split_over_fp64"] = round(out["batch_split_rhs_per_s"] / out["fp64_rhs_per_s"], 3)
        if "fp64_full" in results:
            out["batch_split_over_fp64_full"] = round(out["batch_split_rhs_per_s"] / out["fp64_full_rhs_per_s"], 3)
        out["config"]["workload"] += (f"; value = batched split-BF16 rhs/s of {batch['flows']} flows "
                                      "at N=96 with (mu, t', U) drawn as in the batched configuration")
    if batch64 is not None:
        out["batch64_split_rhs_per_s"] = round(batch64["rhs"] / batch64["seconds"], 3)
        out["batch64"] = {"flows": batch64["flows"], "rhs_evaluated": batch64["rhs"],
                          "seconds": round(batch64["seconds"], 4),
                          "flows_running_at_end": batch64["still_running"]}
        for ref in ("fp64", "fp64_full"):
            if ref in results:
                out[f"batch64_split_over_{ref}"] = round(out["batch64_split_rhs_per_s"] / out[f"{ref}_rhs_per_s"], 3)

    if iflow is not None:
        out["iflow_p1"] = dict(iflow, workload="interaction flow at T=0.1, N=32, 16x16 points/patch, "
                                               "t'=-0.01 mu=-0.02, bare U(g=1)=2, DP5(4) steps from V=U, "
                                               "symmetric-vertex mode; bubbles once per flow")

    # roofline of the dominant kernel of the headline leg (a single-flow leg)
    if head is None:
        out["roofline"] = {"kernel": None, "bound": None, "achieved": None, "peak": None, "unit": None,
                           "frac": None, "traffic": None, "note": "needs a single-flow leg"}
    else:
        out["roofline"] = roofline(head, results, algo_flops, dense_flops, exec_share, evals_per_rhs)
        if out["roofline"]["kernel"] != "contract":
            out["contract_roofline"] = roofline(head, results, algo_flops, dense_flops, exec_share,
                                                evals_per_rhs, kernel="contract")

    if not args.no_cpu_baseline:
        import oracle as O
        O.build(force=False)
        cores = os.cpu_count() or 1
        cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
        O.set_threads(cores)
        m = O.Model(**p)
        Vh = np.full((N, N, N), float(p["U"]))
        t0 = time.perf_counter()
        m.rhs(0.05, Vh)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1.0 / t_cpu, 6), "unit": "rhs/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "one full FP64 oracle rhs at the benchmark workload "
                                         "(N=96, 512 points/patch, T=0.05): bubbles + contraction"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
