"""Write c2_flow_oracle.json: the oracle's own adaptive flow of the production
FP64 workload (N = 48 patches, 16 x 16 fine points, t' = -0.25, mu = 4t' (van
Hove), U = 3; Dormand-Prince 5(4) in s = ln T from T = 1, rtol 1e-6,
atol 1e-10, h0 = -0.01, stopped when max|V| exceeds 20 or T reaches 1e-3).

Calls only the oracle (plain FP64 C, one output entry per thread, so the result
does not depend on the thread count).  The GPU flow test replays the same
configuration and compares its step log, its stop and a seeded sample of the
final vertex with what is stored here.  Run from the repository root:

    python tests/golden/make_c2_flow.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1510_07799_amd import inputs as I  # noqa: E402

SAMPLE_SEED = 4848
N_SAMPLE = 256


def main():
    O.build(force=False)
    c = I.CONFIGS["C2"]
    p = I.model_params("C2")
    f = c["flow"]
    m = O.Model(**p)
    V, res, log = m.flow(stepper="dp54", T0=f["T0"], T_min=f["T_min"], rtol=f["rtol"], atol=f["atol"],
                         vmax=f["vmax"], h0=f["h0"])
    idx = I.random_entries(m.N, N_SAMPLE, seed=SAMPLE_SEED)
    out = {
        "what": "oracle DP5(4) temperature flow of the production FP64 workload (N=48, 16x16 points/patch, "
                "t'=-0.25, mu=-1, U=3) from V=U at T=1; rtol 1e-6, atol 1e-10, h0=-0.01, vmax 20, T_min 1e-3",
        "written_by": "tests/golden/make_c2_flow.py (calls only oracle/)",
        "params": p,
        "flow": f,
        "result": {k: (None if isinstance(v, float) and math.isnan(v) else v) for k, v in res.items()},
        "log_columns": ["s", "h", "err", "max|V|", "rhs_evals", "rejected"],
        "log": log.tolist(),
        "final_max_abs_V": float(np.abs(V).max()),
        "sample_seed": SAMPLE_SEED,
        "sample_entries": idx.tolist(),
        "sample_values": V[idx[:, 0], idx[:, 1], idx[:, 2]].tolist(),
    }
    with open(os.path.join(HERE, "c2_flow_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"accepted {res['accepted']} rejected {res['rejected']} reason {res['reason']} "
          f"T_c {math.exp(res['s_c']) if res['s_c'] == res['s_c'] else None}")


if __name__ == "__main__":
    main()
