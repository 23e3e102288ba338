"""Writes the stored inputs and expected values for the benchmark-shaped case
(about 1.04e7 compounds, 256 -> 512 -> 512 (SiLU) -> 15 decoder).

1. c1_query.json: query thresholds. The seeded choices (objective head, bounded
   heads, sides, quantiles in [0.6, 0.9]) come from the input generator; the
   threshold values are the FP64 oracle's head quantiles over 2^16 seeded
   compounds. A "stringent" variant uses quantiles in [0.2, 0.4].
2. c1_oracle_<variant>.json: the FP64 oracle's exhaustive top-k (k = 1000, plus
   one extra entry for the k-th gap) with its boundary margins.
3. c1_heads_sample.json: FP64 heads of 1024 seeded compounds (per-head error of
   the low-precision paths).

Only the oracle computes anything here. Run: python tests/golden/make_c1_golden.py
(about 8 minutes per variant on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads.gen as g  # noqa: E402
from workloads.gen import Constraint, Query  # noqa: E402

K = 1000
SEED = 1


def f32(x):
    return float(np.float32(x))


def make_queries(lib, dec):
    obj, heads, sides, quant = g.seeded_query_c1(SEED, dec.n_heads)
    ids = g.sample_ids(SEED, "c1_calibration", lib.n_compounds, 1 << 16)
    H = oracle.heads(lib, dec, ids)
    out = {}
    for variant, qs in (("standard", quant), ("stringent", [q - 0.4 for q in quant])):
        cons = []
        for h, side, q in zip(heads, sides, qs):
            if side == "hi":  # head <= its q-quantile
                cons.append({"head": h, "lo": None, "hi": f32(np.quantile(H[:, h], q))})
            else:  # head >= its (1-q)-quantile
                cons.append({"head": h, "lo": f32(np.quantile(H[:, h], 1.0 - q)), "hi": None})
        w = [0.0] * dec.n_heads
        w[obj] = -1.0
        out[variant] = {"w": w, "constraints": cons, "k": K, "quantiles": [float(x) for x in qs]}
    return out


def to_query(spec):
    cons = [Constraint(c["head"], -np.inf if c["lo"] is None else c["lo"],
                       np.inf if c["hi"] is None else c["hi"]) for c in spec["constraints"]]
    return Query(w=np.array(spec["w"], np.float32), constraints=cons, k=spec["k"])


def main():
    lib, dec = g.config_c1(SEED)
    qpath = os.path.join(HERE, "c1_query.json")
    if os.path.exists(qpath):
        queries = json.load(open(qpath))["queries"]
    else:
        queries = make_queries(lib, dec)
        json.dump({"source": "tests/golden/make_c1_golden.py (FP64 oracle head quantiles, 2^16 seeded compounds)",
                   "seed": SEED, "n_compounds": lib.n_compounds, "queries": queries},
                  open(qpath, "w"), indent=1)
    hpath = os.path.join(HERE, "c1_heads_sample.json")
    if not os.path.exists(hpath):
        ids = g.sample_ids(SEED, "c1_head_error_sample", lib.n_compounds, 1024)
        H = oracle.heads(lib, dec, ids)
        json.dump({"source": "FP64 oracle heads of 1024 seeded compounds, tests/golden/make_c1_golden.py",
                   "ids": [int(x) for x in ids], "heads": [[float(v) for v in row] for row in H]},
                  open(hpath, "w"))
    only = sys.argv[1:] or [v for v in queries if not os.path.exists(os.path.join(HERE, f"c1_oracle_{v}.json"))]
    for variant in only:
        q = to_query(queries[variant])
        t0 = time.time()
        r = oracle.topk(lib, dec, q, extra=1, near_tol=1e-3)
        dt = time.time() - t0
        json.dump({
            "source": "FP64 oracle, exhaustive, tests/golden/make_c1_golden.py",
            "variant": variant, "k": q.k, "n_compounds": lib.n_compounds,
            "n_feasible": r.n_feasible, "seconds": dt,
            "ids": [int(x) for x in r.ids], "objective": [float(x) for x in r.objective],
            "gap_k": r.gap_k, "min_slack_selected": r.min_slack_selected,
            "min_violation_near": r.min_violation_near, "n_near": r.n_near,
        }, open(os.path.join(HERE, f"c1_oracle_{variant}.json"), "w"))
        print(variant, "n_feasible", r.n_feasible, "seconds", round(dt, 1), flush=True)


if __name__ == "__main__":
    main()
