"""Autotune the benchmark workloads and write the tuning table (needs a GPU).

    python -m paper_1510_07799_amd.tune [--out PATH] [--reps R]

Workloads: N = 96 patches with 512 fine points each; one flow in split and FP64
precision, with one contraction column per C4v orbit and with every column;
batches of 16 flows (split and FP64) and of 64 flows (split) with the
parameters drawn as in the batched configuration.  Each search runs in the
library (frg_tune / frg_batch_tune: event-timed rhs evaluations per candidate)
from a C4v-symmetric random vertex at T = 0.5, the temperature range of the
benchmark's timed steps.  The table records the best parameters, their
per-rhs kernel time and every candidate's times.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1510_07799_amd import inputs as I, tuning as TU  # noqa: E402

T_TUNE = 0.5
LOG_COLUMNS = ["kparts", "sweep_rows", "block_rows", "ms_bubbles", "ms_contract_and_sums", "ms_all"]


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=TU.TABLE_PATH)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--only", default="", help="comma list of keys to tune (default: all)")
    args = ap.parse_args()
    import torch
    from paper_1510_07799_amd import frg

    p = I.model_params("C3")
    N, nf = p["N"], p["n_rad"] * p["n_ang"]
    only = {x for x in args.only.split(",") if x}
    entries = {}

    def record(k, tun, ms, log, extra=None):
        entries[k] = dict(tun, ms_per_rhs=round(ms, 5), log_columns=LOG_COLUMNS,
                          log=[[round(float(v), 5) for v in row] for row in log], **(extra or {}))
        print(f"[tune] {k}: {tun} {ms:.4f} ms", flush=True)

    ctx = frg.Context(**p)
    V = torch.from_numpy(I.random_vertex(N, p["U"], seed=7, amp=0.3, symmetrise=True)).cuda()
    for split in (True, False):
        for orbit in (True, False):
            k = TU.key(N, nf, split, orbit)
            if only and k not in only:
                continue
            ctx.set_vsym(orbit)
            prec = frg.PREC_SPLIT_BF16 if split else frg.PREC_FP64
            tun, ms, log = ctx.tune(T_TUNE, V, prec, reps=args.reps)
            record(k, tun, ms, log)
    ctx.set_vsym(False)
    ctx.close()
    del V
    torch.cuda.empty_cache()
    for flows, split in ((16, True), (16, False), (64, True)):
        k = TU.key(N, nf, split, True, flows)
        if only and k not in only:
            continue
        draws = I.c4_flows(n_per_N=flows, Ns=(N,), n_rad=p["n_rad"], n_ang=p["n_ang"])
        b = frg.Batch(draws)
        b.set_vsym(True)
        Vs = [torch.from_numpy(I.random_vertex(N, d["U"], seed=11 + i, amp=0.3, symmetrise=True)).cuda()
              for i, d in enumerate(draws)]
        prec = frg.PREC_SPLIT_BF16 if split else frg.PREC_FP64
        tun, ms, log = b.tune([T_TUNE] * flows, Vs, prec, reps=max(2, args.reps // 2))
        record(k, tun, ms / flows, log, {"note": "ms per flow and rhs (the batched rhs of all flows / flows)"})
        b.close()
        del Vs
        torch.cuda.empty_cache()
    old = {}
    if os.path.exists(args.out):
        with open(args.out) as fh:
            old = json.load(fh).get("entries", {})
    old.update(entries)
    out = {"what": "tuned launch parameters per workload (kparts, sweep_rows, block_rows); log rows: " +
                   ", ".join(LOG_COLUMNS),
           "written_by": "python -m paper_1510_07799_amd.tune", "T": T_TUNE, "entries": old}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"[tune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
