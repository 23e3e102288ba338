"""Writes stored inputs and expected values for the large streamed case
(2,000 reactions, about 2.9e10 compounds, d = 256, 256 -> 512 -> 512 (SiLU) -> 15).

1. c3_query.json: objective = weighted sum of 3 seeded heads, 6 seeded one-sided
   bounds at quantiles in [0.6, 0.9] of 4096 seeded compounds' FP64 heads
   (the oracle), k = 10,000.
2. c3_oracle_subset.json: the FP64 oracle's exhaustive top-k of that query on a
   seeded reaction subset of about 1e7 compounds (the whole library is far beyond
   the oracle's reach: about 2.4e16 FP64 FLOP).
3. c3_heads_sample.json: FP64 heads of 512 seeded compounds of the full library.

Only the oracle computes anything here. The tables (5.4 GB of float32) are
generated with the bulk generator. Run: python tests/golden/make_c3_golden.py
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads.gen as g  # noqa: E402
from workloads.gen import Constraint, Query  # noqa: E402

SEED = 2
K = 10_000
SUBSET_TARGET = 10_000_000


def main():
    t0 = time.time()
    lib, dec = g.config_c3(SEED)
    print("library", lib.n_compounds, "rows", lib.n_rows, f"{time.time() - t0:.1f}s", flush=True)
    ids = g.sample_ids(SEED, "c3_calibration", lib.n_compounds, 4096)
    H = oracle.heads(lib, dec, ids)
    u = g.uniform_f64(SEED, "query_c3", 32)
    perm = np.argsort(g.uniform_f64(SEED, "query_c3_heads", 15), kind="stable")
    obj_heads = [int(h) for h in perm[:3]]
    con_heads = [int(h) for h in perm[3:9]]
    w = [0.0] * 15
    for i, h in enumerate(obj_heads):
        w[h] = float(np.float32(-1.0 + 2.0 * u[i]))
    cons = []
    for i, h in enumerate(con_heads):
        q = 0.6 + 0.3 * float(u[3 + i])
        if u[9 + i] < 0.5:
            cons.append({"head": h, "lo": None, "hi": float(np.float32(np.quantile(H[:, h], q)))})
        else:
            cons.append({"head": h, "lo": float(np.float32(np.quantile(H[:, h], 1.0 - q))), "hi": None})
    counts = lib.reaction_counts()
    order = np.argsort(g.uniform_f64(SEED, "c3_subset", lib.n_reactions), kind="stable")
    subset, tot = [], 0
    for t in order:
        if counts[int(t)] > SUBSET_TARGET // 4:
            continue
        subset.append(int(t))
        tot += counts[int(t)]
        if tot >= SUBSET_TARGET:
            break
    subset.sort()
    spec = {"w": w, "constraints": cons, "k": K, "subset": subset, "subset_compounds": tot}
    json.dump({"source": "tests/golden/make_c3_golden.py (FP64 oracle head quantiles, 4096 seeded compounds)",
               "seed": SEED, "n_compounds": lib.n_compounds, "query": spec},
              open(os.path.join(HERE, "c3_query.json"), "w"), indent=1)
    hs_ids = g.sample_ids(SEED, "c3_head_error_sample", lib.n_compounds, 512)
    HS = oracle.heads(lib, dec, hs_ids)
    json.dump({"source": "FP64 oracle heads of 512 seeded compounds, tests/golden/make_c3_golden.py",
               "ids": [int(x) for x in hs_ids], "heads": [[float(v) for v in row] for row in HS]},
              open(os.path.join(HERE, "c3_heads_sample.json"), "w"))
    q = Query(w=np.array(w, np.float32),
              constraints=[Constraint(c["head"], -math.inf if c["lo"] is None else c["lo"],
                                      math.inf if c["hi"] is None else c["hi"]) for c in cons],
              k=K, reactions=subset)
    t1 = time.time()
    r = oracle.topk(lib, dec, q, extra=1, near_tol=1e-3)
    json.dump({"source": "FP64 oracle, exhaustive over the subset, tests/golden/make_c3_golden.py",
               "k": K, "subset_compounds": tot, "n_feasible": r.n_feasible, "seconds": time.time() - t1,
               "ids": [int(x) for x in r.ids], "objective": [float(x) for x in r.objective],
               "gap_k": r.gap_k, "min_slack_selected": r.min_slack_selected,
               "min_violation_near": r.min_violation_near},
              open(os.path.join(HERE, "c3_oracle_subset.json"), "w"))
    print("subset", tot, "feasible", r.n_feasible, f"{time.time() - t1:.1f}s", flush=True)


if __name__ == "__main__":
    main()
