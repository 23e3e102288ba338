"""Benchmark: exhaustive constrained top-k over the benchmark-shaped synthetic
library (10,373,770 compounds in 40 reactions, 28 two-slot and 12 three-slot;
d = 256; decoder 256 -> 512 -> 512 (SiLU) -> 15; one objective, four bounds,
k = 1000).

One step is one complete search through the C ABI: threshold warm start, every
compound of the library gathered, combined and decoded on MFMA, masked and
filtered, candidates selected, the pool rescored in FP32 (BF16/FP8), the answer
sorted and decoded. Inputs (tables, weights) are resident in HBM before timing.

Prints one JSON line. `value` is the headline precision's compounds/s; the other
precisions, recall@k against the FP64 oracle's stored answer, the roofline of
the fused kernel and the CPU oracle's rate are reported beside it. The default
run adds the other measured workloads as legs of the same line:
  - "c3": the 2.9e10-compound library streamed, one search each in BF16 and FP8;
  - "serving_c4": a Poisson query stream over reaction subsets of that library
    (1e6 to 1e9 compounds each), shortened to what one GPU serves;
  - "probe_runtime_table": the paper's own configuration (a 28-head linear
    probe, d = 64) on libraries shaped like its 12M, 10B and 70B ones, at the
    k values and constraint sets of its runtime table, beside its T4 times;
  - "cpu_baseline": the FP64 oracle on the host (CPU model, threads, a
    single-thread rate, the tiny case in full).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")
PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}  # dense MFMA, MI355X
METRIC = "compounds/s scored+top-k, BF16/FP8 vs FP32 @ recall@k>=0.99; p99 query latency"
# vector ALU: 256 CUs x 64 lanes x 2.4 GHz (one FP32 operation per lane and clock, unpacked)
VALU_PEAK = 256 * 64 * 2.4e9

# The paper's runtime table (Table tab:runtime): end-to-end seconds on one NVIDIA
# Tesla T4 with its linear probe, averaged over five docking targets; the
# parenthesised CPU times of the table are "cpu".
PAPER_T4 = {
    "hardware": "one NVIDIA Tesla T4 (CPU model not stated); times include building an output table with "
                "SMILES, which this engine does not do",
    "none": {"12M": {10**4: (0.3, 0.4), 10**5: (1.2, 1.2), 10**6: (10.9, 12.7)},
             "10B": {10**4: (10.9, 130.7), 10**5: (11.6, 131.4), 10**6: (21.2, 147.6)},
             "70B": {10**4: (168.4, 838.5), 10**5: (169.3, 847.2), 10**6: (184.0, 858.9)}},
    "lipinski": {"12M": {10**4: (0.3, 0.7), 10**5: (0.9, 1.7), 10**6: (10.8, 12.9)},
                 "10B": {10**4: (13.9, 437.7), 10**5: (14.6, 443.7), 10**6: (24.3, 462.2)},
                 "70B": {10**4: (186.1, 3163.2), 10**5: (187.5, 3184.6), 10**6: (202.4, 3142.5)}},
}
PROFILES = os.path.join(ROOT, "profiles")
CSRC = "paper_2510_24380_amd/csrc/"


def fused_kernel(prec):
    """Name and defining sources of the fused kernel of one precision: FP32 runs
    the 16x16 MFMA kernel, BF16/FP8 the 32x32 one."""
    name, header = ("k_enum", "enum_kernel.h") if prec == "fp32" else ("k_enum32", "enum32_kernel.h")
    return name, [CSRC + header, CSRC + "enum_common.h", CSRC + "apex_internal.h", CSRC + f"enum_{prec}.hip"]


def log(msg):
    """Progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_sha256(prec):
    """Hash of the sources that define the fused kernel of one precision."""
    import hashlib
    h = hashlib.sha256()
    for rel in fused_kernel(prec)[1]:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def measured_traffic(prec, workload="c1"):
    """HBM bytes per launch of the fused kernel from the committed hardware-counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or
    None when there is none or the kernel sources changed since it was taken."""
    v = profile_values("counters", prec, workload)
    try:
        return float(v["hbm_bytes_per_launch"]) if v else None
    except (KeyError, ValueError):
        return None


def profile_values(name, prec, workload="c1"):
    """`- key: value` lines of a committed profile summary, or None when there is
    none or the kernel sources changed since it was taken."""
    path = os.path.join(PROFILES, f"{fused_kernel(prec)[0]}_{prec}_{workload}_{name}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip("` ")] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256(prec):
        return None
    return vals


def valu_estimate(prec, flops_per_compound, compounds_per_launch, avg_launch_ms):
    """Issue time of one launch's vector work beside its MFMA time, from the
    committed issue-level counters and the per-SIMD issue costs measured by
    throughput probes on gfx950: 4 cycles per VALU wave instruction, 8 per
    transcendental (exp2, rcp: half rate), and 8 cycles of VALU issue taken by
    each 32x32 MFMA (a VALU-only wave beside a saturated MFMA chain loses a
    quarter of its rate; measured for the BF16 shape, assumed for FP8). The
    1024 SIMDs issue at 2.4 GHz, the clock the peaks are quoted at."""
    v = profile_values("sq_counters", prec)
    if v is None or "mfma_insts_per_compound" not in v:
        return None
    simd_hz = 1024 * 2.4e9
    insts = float(v["valu_insts_per_compound"])  # MFMA included
    trans = float(v["trans_insts_per_compound"])
    mfma = float(v["mfma_insts_per_compound"])
    cycles = 4 * (insts - trans - mfma) + 8 * trans + 8 * mfma
    t_issue = cycles * compounds_per_launch / simd_hz
    t_mfma = flops_per_compound * compounds_per_launch / PEAK[prec]
    clock = float(v["clock_ghz_under_load"])
    return {"valu_insts_per_compound": insts, "trans_insts_per_compound": trans, "mfma_insts_per_compound": mfma,
            "issue_cycles_per_compound": cycles,
            "issue_model": "4 cycles per VALU instruction, 8 per transcendental, 8 per 32x32 MFMA (per SIMD)",
            "t_issue_ms": t_issue * 1e3, "t_mfma_ms_at_peak": t_mfma * 1e3, "t_launch_ms": avg_launch_ms,
            "issue_bound_at_peak": t_issue > t_mfma,
            "issue_frac_at_measured_clock": t_issue * 2.4 / clock / (avg_launch_ms * 1e-3) if avg_launch_ms else None,
            "measured_mfma_busy": float(v["mfma_busy"]), "measured_valu_active": float(v["valu_active"]),
            "measured_clock_ghz": clock}


def reference_gemm(precs, n=8192, iters=40):
    """Dense square GEMM rate of the vendor library (hipBLASLt through torch) on this
    GPU, in TFLOP/s per precision: a measured ceiling for MFMA work under the same
    clock and power limits, reported beside the published peak."""
    import torch
    dev = torch.device("cuda:0")
    out = {}
    for p in precs:
        if p == "fp8":
            a = torch.randn(n, n, device=dev).to(torch.float8_e4m3fn)
            b = torch.randn(n, n, device=dev).to(torch.float8_e4m3fn).t()
            one = torch.tensor(1.0, device=dev)
            f = lambda: torch._scaled_mm(a, b, scale_a=one, scale_b=one, out_dtype=torch.bfloat16)
        else:
            dt = torch.bfloat16 if p == "bf16" else torch.float32
            a = torch.randn(n, n, device=dev, dtype=dt)
            b = torch.randn(n, n, device=dev, dtype=dt)
            f = lambda: torch.matmul(a, b)
        its = iters if p != "fp32" else max(4, iters // 8)
        for _ in range(3):
            f()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(its):
            f()
        e1.record()
        torch.cuda.synchronize()
        tf = 2.0 * n ** 3 * its / (e0.elapsed_time(e1) * 1e-3) / 1e12
        out[p] = {"tflops": tf, "frac_of_peak": tf * 1e12 / PEAK[p]}
        del a, b, f
    torch.cuda.empty_cache()
    return out


def algorithmic_flops_per_compound(dims):
    """MFMA-class FLOPs per compound once the first layer is hoisted into the
    per-synthon tables: 2 * sum over the remaining layers of in * out."""
    return 2 * sum(dims[l] * dims[l + 1] for l in range(1, len(dims) - 1))


def load_query(variant="standard"):
    from workloads.gen import Constraint, Query
    spec = json.load(open(os.path.join(GOLDEN, "c1_query.json")))["queries"][variant]
    cons = [Constraint(c["head"], -math.inf if c["lo"] is None else c["lo"],
                       math.inf if c["hi"] is None else c["hi"]) for c in spec["constraints"]]
    return Query(w=np.array(spec["w"], np.float32), constraints=cons, k=spec["k"])


def golden_ids(variant="standard"):
    """The FP64 oracle's exhaustive top-k (stored by tests/golden/make_c1_golden.py)."""
    g = json.load(open(os.path.join(GOLDEN, f"c1_oracle_{variant}.json")))
    return g["ids"][:g["k"]]


def cpu_baseline(lib_h, dec_h, q, target_s=15.0):
    """The FP64 oracle (as it is) on a subset of reactions of the same library."""
    import oracle
    counts = lib_h.reaction_counts()
    order = sorted(range(len(counts)), key=lambda t: counts[t])
    # calibrate the rate on a small subset, then size the timed subset
    small = []
    tot = 0
    for t in order:
        if tot + counts[t] > 60_000:
            break
        small.append(t)
        tot += counts[t]
    if not small:
        small = [order[0]]
    qs = type(q)(w=q.w, constraints=q.constraints, k=q.k, reactions=small)
    t0 = time.perf_counter()
    oracle.topk(lib_h, dec_h, qs)
    rate = sum(counts[t] for t in small) / max(time.perf_counter() - t0, 1e-6)
    want = rate * target_s
    subset, tot = [], 0
    for t in order:
        if tot + counts[t] > want and subset:
            continue
        subset.append(t)
        tot += counts[t]
        if tot >= want:
            break
    qs = type(q)(w=q.w, constraints=q.constraints, k=q.k, reactions=subset)
    t0 = time.perf_counter()
    oracle.topk(lib_h, dec_h, qs)
    dt = time.perf_counter() - t0
    return {"value": tot / dt, "unit": "compounds/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, exhaustive top-k over a subset of {len(subset)} reactions "
                      f"({tot} compounds) of the same library and query, {dt:.1f} s"}


def serve_bench(eng, counts, head_sample, n_queries, qps, size_lo, size_hi, prec="bf16", chunk_compounds=1 << 20,
                seed=4, n_seq=None, capacity=True):
    """Continuous-batching server on a seeded Poisson stream of queries over
    reaction subsets of the library (sizes log-uniform in [size_lo, size_hi]
    compounds, thresholds at quantiles of `head_sample`, FP64 heads of seeded
    compounds), against one-query-at-a-time FP32 searches on the same arrivals
    (the first n_seq of them when given)."""
    import paper_2510_24380_amd as apex
    import workloads.gen as gen
    stream = gen.serving_stream(seed, n_queries, qps, counts, size_lo, size_hi,
                                lambda h, qq: np.quantile(head_sample[:, h], qq))
    sizes = [sum(counts[r] for r in q.reactions) for _, q in stream]

    def pct(v, p):
        return float(np.percentile(np.array(v), p)) if v else 0.0

    # 1. served, Poisson arrivals
    srv = apex.Server(eng, pool_bytes=4 << 30, max_active=16, chunk_compounds=chunk_compounds)
    t0 = time.perf_counter()
    tickets = []
    for i, (t, q) in enumerate(stream):
        dt = t0 + t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(q, precision=prec))
        if (i + 1) % 100 == 0:
            log(f"serving: {i + 1}/{len(stream)} submitted")
    served = []
    for i, tk in enumerate(tickets):
        served.append(srv.poll(tk, timeout_ms=600000))
        if (i + 1) % 20 == 0:
            log(f"serving: {i + 1}/{len(tickets)} completed")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out = {"queries": n_queries, "qps": qps, "precision": prec, "chunk_compounds": chunk_compounds,
           "library_sizes": [min(sizes), float(np.median(sizes)), max(sizes)],
           "served": {"p50_latency_ms": st["p50_latency_ms"], "p99_latency_ms": st["p99_latency_ms"],
                      "max_latency_ms": st["max_latency_ms"], "wall_s": wall,
                      "device_compounds_per_s": st["compounds_per_s"]}}
    # 2. served, all submitted at once (capacity)
    if capacity:
        srv = apex.Server(eng, pool_bytes=4 << 30, max_active=16, chunk_compounds=chunk_compounds)
        t1 = time.perf_counter()
        tk2 = [srv.submit(q, precision=prec) for _, q in stream]
        for tk in tk2:
            srv.poll(tk, timeout_ms=600000)
        out["served"]["saturated_query_compounds_per_s"] = sum(sizes) / (time.perf_counter() - t1)
        srv.close()
    # 3. sequential FP32 on the same arrivals
    seq_stream = stream if n_seq is None else stream[:n_seq]
    lat, seq = [], []
    t2 = time.perf_counter()
    busy = 0.0
    for t, q in seq_stream:
        dt = t2 + t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        a = time.perf_counter()
        seq.append(eng.search(q, precision="fp32"))
        busy += time.perf_counter() - a
        lat.append((time.perf_counter() - t2 - t) * 1e3)
        if len(seq) % 10 == 0:
            log(f"sequential FP32: {len(seq)}/{len(seq_stream)} done")
    recalls = [len(set(a.ids.tolist()) & set(b.ids.tolist())) / max(1, len(b.ids)) for a, b in zip(served, seq)]
    out["sequential_fp32"] = {"queries": len(seq_stream), "p50_latency_ms": pct(lat, 50),
                              "p99_latency_ms": pct(lat, 99), "max_latency_ms": max(lat),
                              "query_compounds_per_s": sum(sizes[:len(seq_stream)]) / busy}
    out["recall_vs_sequential_fp32"] = {"mean": float(np.mean(recalls)), "min": float(np.min(recalls))}
    return out


def build_c3(precisions):
    """The streamed 2.9e10-compound library and its engine (tables generated on the host)."""
    import torch
    import paper_2510_24380_amd as apex
    import workloads.gen as gen
    lib_h, dec_h = gen.config_c3()
    counts = lib_h.reaction_counts()
    tables = torch.from_numpy(lib_h.tables).cuda()
    del lib_h.tables
    lib = apex.Library(lib_h.n_slots, lib_h.slot_sizes, tables)
    dec = apex.Decoder(dec_h.dims, "silu", [torch.from_numpy(w).cuda() for w in dec_h.W],
                       [torch.from_numpy(b).cuda() for b in dec_h.b])
    return lib_h, dec_h, counts, lib, apex.Engine(lib, dec, precisions=precisions)


def main_c4(args):
    """Serving at the large scale: a Poisson stream (5 queries/s) of queries over
    reaction subsets of the 2.9e10-compound library, 1e6 to 1e9 compounds each."""
    t0 = time.perf_counter()
    lib_h, dec_h, counts, lib, eng = build_c3(("fp32", args.precision))
    log(f"engine ready ({lib.num_compounds} compounds, {time.perf_counter() - t0:.0f} s)")
    H = np.array(json.load(open(os.path.join(GOLDEN, "c3_heads_sample.json")))["heads"])
    sv = serve_bench(eng, counts, H, args.serve_queries, args.serve_qps, 1e6, 1e9, prec=args.precision,
                     chunk_compounds=1 << 26, seed=5, n_seq=args.seq_queries, capacity=False)
    out = {
        "metric": "served query compounds/s and latency (continuous batching) vs sequential FP32",
        "value": sv["served"]["device_compounds_per_s"], "unit": "compounds/s", "n_gpus": 1,
        "steps": args.serve_queries, "warmup": 0, "ms_per_step": sv["served"]["wall_s"] * 1e3 / args.serve_queries,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (seeded N(0,1) synthon embeddings, Xavier-uniform decoder)",
        "config": {"workload": f"serving: {args.serve_queries} queries, Poisson {args.serve_qps}/s, reaction "
                               "subsets of the 2.9e10-compound synthetic CSL with 1e6-1e9 compounds each, "
                               "random objectives over 15 heads, 2-6 bounds, k in {100, 1000, 10000}",
                   "precision": args.precision},
        "p99_latency_ms": sv["served"]["p99_latency_ms"],
        "serving": sv,
    }
    print(json.dumps(out), flush=True)


def main_c3(args):
    """The streamed 2.9e10-compound library: one step is one search over all of it."""
    import torch
    from workloads.gen import Constraint, Query
    t0 = time.perf_counter()
    lib_h, dec_h, counts, lib, eng = build_c3(("fp32", args.precision))
    spec = json.load(open(os.path.join(GOLDEN, "c3_query.json")))["query"]
    cons = [Constraint(c["head"], -math.inf if c["lo"] is None else c["lo"],
                       math.inf if c["hi"] is None else c["hi"]) for c in spec["constraints"]]
    q = Query(w=np.array(spec["w"], np.float32), constraints=cons, k=spec["k"])
    setup_s = time.perf_counter() - t0
    n = lib.num_compounds
    log(f"engine ready ({n} compounds, {setup_s:.0f} s)")
    flops_c = algorithmic_flops_per_compound(dec_h.dims)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        del a
    for _ in range(args.warmup):
        eng.search(q, precision=args.precision)
        log("warm-up search done")
    eng.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        r = eng.search(q, precision=args.precision)
        torch.cuda.synchronize()
        log(f"search {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / args.steps
    ms, launches, comps = eng.profile(False)
    achieved = flops_c * comps / (ms * 1e-3) if ms > 0 else 0.0
    out = {
        "metric": METRIC, "value": n / dt, "unit": "compounds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (seeded N(0,1) synthon embeddings, Xavier-uniform decoder)",
        "config": {"workload": "2.9e10-compound synthetic CSL streamed (2000 reactions, lognormal slot sizes median "
                               "800 up to 10000), d=256, decoder 256->512->512 (SiLU)->15, objective = weighted sum "
                               "of 3 heads, 6 one-sided bounds, k=10000, 4k pool rescored in FP32",
                   "n_compounds": n, "k": q.k, "precision": args.precision},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[args.precision] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[args.precision], "traffic": None,
                     "kernel": f"apex::{fused_kernel(args.precision)[0]} (fused)", "avg_launch_ms": ms / max(launches, 1),
                     "launches_per_step": launches / args.steps, "flops_per_compound": flops_c},
        "results": {"n_found": len(r.ids), "candidates": r.n_candidates, "reruns": r.n_reruns,
                    "best_ids": [int(x) for x in r.ids[:5]]},
        "setup_s": setup_s,
    }
    print(json.dumps(out), flush=True)


def c3_leg(precisions=("bf16", "fp8"), serve_queries=60, serve_qps=2.0, seq_queries=3):
    """The 2.9e10-compound library: one search per precision (the kernels are
    already loaded by the headline run), then a shortened serving stream over its
    reaction subsets. Returns (c3, serving) dicts; the engine is freed after."""
    import torch
    from workloads.gen import Constraint, Query
    t0 = time.perf_counter()
    lib_h, dec_h, counts, lib, eng = build_c3(("fp32",) + tuple(precisions))
    spec = json.load(open(os.path.join(GOLDEN, "c3_query.json")))["query"]
    cons = [Constraint(c["head"], -math.inf if c["lo"] is None else c["lo"],
                       math.inf if c["hi"] is None else c["hi"]) for c in spec["constraints"]]
    q = Query(w=np.array(spec["w"], np.float32), constraints=cons, k=spec["k"])
    n = lib.num_compounds
    setup_s = time.perf_counter() - t0
    log(f"c3: engine ready ({n} compounds, {setup_s:.0f} s)")
    flops_c = algorithmic_flops_per_compound(dec_h.dims)
    c3 = {"workload": "2.9e10-compound synthetic CSL streamed (2000 reactions, lognormal slot sizes median 800 up "
                      "to 10000), d=256, decoder 256->512->512 (SiLU)->15, objective = weighted sum of 3 heads, "
                      "6 one-sided bounds, k=10000, 4k pool rescored in FP32; one search per precision",
          "n_compounds": n, "setup_s": setup_s}
    top = {}
    for prec in precisions:
        eng.profile(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = eng.search(q, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ms, launches, comps = eng.profile(False)
        achieved = flops_c * comps / (ms * 1e-3) if ms > 0 else 0.0
        top[prec] = [int(x) for x in r.ids[:100]]
        c3[prec] = {"seconds": dt, "compounds_per_s": n / dt, "n_found": len(r.ids), "candidates": r.n_candidates,
                    "reruns": r.n_reruns,
                    "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12,
                                 "unit": "TFLOP/s", "frac": achieved / PEAK[prec],
                                 "traffic": measured_traffic(prec, "c3"), "traffic_unit": "bytes/launch",
                                 "kernel": f"apex::{fused_kernel(prec)[0]} (fused)",
                                 "avg_launch_ms": ms / max(launches, 1), "launches": launches}}
        log(f"c3 {prec}: {n / dt:.4g} compounds/s ({dt:.1f} s)")
    if len(top) == 2:
        a, b = list(top.values())
        c3["top100_overlap_between_precisions"] = len(set(a) & set(b)) / max(1, len(a))
    serving = None
    if serve_queries:
        H = np.array(json.load(open(os.path.join(GOLDEN, "c3_heads_sample.json")))["heads"])
        serving = serve_bench(eng, counts, H, serve_queries, serve_qps, 1e6, 1e9, prec=precisions[0],
                              chunk_compounds=1 << 26, seed=5, n_seq=seq_queries, capacity=False)
        serving["stream"] = (f"{serve_queries} queries, Poisson {serve_qps}/s, reaction subsets of the "
                             "2.9e10-compound library with 1e6-1e9 compounds each, random objectives over 15 heads, "
                             "2-6 bounds, k in {100, 1000, 10000}; shortened from 2,000 queries at 5/s, which offer "
                             "about 3e9 compounds/s, more than one GPU evaluates")
        log("c4 serving stream done")
    del eng, lib
    torch.cuda.empty_cache()
    return c3, serving


def probe_leg(targets=5, libraries=("12M", "10B", "70B")):
    """The paper's own configuration: a 28-head linear probe on d = 64 embeddings,
    libraries shaped like its BRICS 12M, BRICS 10B and Enamine REAL 70B ones, the
    runtime table's k values with no constraints and with the four Lipinski
    bounds, each time averaged over five docking-head objectives. Seconds are
    end to end through the C ABI (query tables, enumeration, selection, answer
    sort, heads, decode, readback into host arrays). The host arrays are the
    caller's, reused across searches as a C caller would (pinned:
    apex.ResultBuffers), so no search pays for first-touch host memory."""
    import torch
    import paper_2510_24380_amd as apex
    import workloads.gen as gen
    shapes = [("12M", 11, lambda: gen.library_shapes_probe(11, 12_450_000)),
              ("10B", 21, lambda: gen.config_c3_shape(21, 1e10)),
              ("70B", 22, lambda: gen.config_c3_shape(22, 7e10))]
    out = {"decoder": "linear probe, 28 heads, d=64 (Section 5.1, Appendix A.8)",
           "query": "minimise one docking head (heads 0-4, one per run) with no bounds or with four one-sided "
                    "Lipinski-style bounds on seeded property heads at seeded quantiles in [0.6, 0.9]",
           "paper_t4": PAPER_T4["hardware"],
           "result_arrays": "caller-owned pinned host arrays of capacity 1e6, reused across searches",
           "libraries": []}
    for name, seed, shape in shapes:
        if name not in libraries:
            continue
        t0 = time.perf_counter()
        n_slots, sizes = shape()
        lib_h, dec_h = gen.config_probe(seed, n_slots, sizes)
        tables = torch.from_numpy(lib_h.tables).cuda()
        del lib_h.tables
        lib = apex.Library(lib_h.n_slots, lib_h.slot_sizes, tables)
        dec = apex.Decoder(dec_h.dims, "none", [torch.from_numpy(w).cuda() for w in dec_h.W],
                           [torch.from_numpy(b).cuda() for b in dec_h.b])
        eng = apex.Engine(lib, dec, precisions=("fp32",))
        n = lib.num_compounds
        # bounds at quantiles of the engine's own FP32 heads of seeded compounds
        hs = eng.heads(gen.sample_ids(seed, "probe_sample", n, 1 << 14))
        quant = lambda h, p: float(np.quantile(hs[:, h], p))  # noqa: E731
        entry = {"library": f"{name}-shaped synthetic", "n_compounds": n, "rows": int(sum(sizes)),
                 "setup_s": time.perf_counter() - t0, "runs": []}
        buf = apex.ResultBuffers(10**6, dec.n_heads)
        eng.search(gen.probe_query(seed + 1, quant, 10**4, target=0), out=buf)
        for cons in ("none", "lipinski"):
            for k in (10**4, 10**5, 10**6):
                qs = [gen.probe_query(seed + 1, quant, k, target=t, lipinski=cons == "lipinski")
                      for t in range(targets)]
                eng.search(qs[0], out=buf)  # warm-up: the workspace grows to this k outside the timing
                eng.profile(True)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                res = [eng.search(q, out=buf) for q in qs]  # counts only: each result views buf
                dt = (time.perf_counter() - t1) / len(qs)
                found = [len(r.ids) for r in res]
                ms, launches, comps = eng.profile(False)
                kr = comps / (ms * 1e-3) if ms > 0 else 0.0
                t4, cpu = PAPER_T4[cons][name][k]
                entry["runs"].append({
                    "constraints": cons, "k": k, "seconds": dt, "compounds_per_s": n / dt,
                    "kernel_ms": ms / len(qs), "kernel_compounds_per_s": kr, "n_found_min": min(found),
                    "candidates_mean": float(np.mean([r.n_candidates for r in res])),
                    "reruns_max": max(r.n_reruns for r in res),
                    "roofline": {"bound": "alu", "achieved": 2 * kr / 1e12, "peak": VALU_PEAK / 1e12,
                                 "unit": "Tops/s", "frac": 2 * kr / VALU_PEAK,
                                 "ops_per_compound": "2 (objective add, threshold compare)",
                                 "kernel": "apex::k_scan"},
                    "paper_t4_seconds": t4, "paper_cpu_seconds": cpu, "speedup_vs_paper_t4": t4 / dt})
                log(f"probe {name} {cons} k={k}: {dt * 1e3:.1f} ms per search ({n / dt:.3g} compounds/s, "
                    f"paper T4 {t4} s)")
        out["libraries"].append(entry)
        del eng, lib, dec, tables, buf, res
        torch.cuda.empty_cache()
    return out


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline_full(lib_h, dec_h, q):
    """The FP64 oracle (as it is) on the host: the benchmark library and query on
    a bounded subset (all threads), the same on a small subset with one thread,
    the tiny case in full, and the probe configuration's 12M-shaped library in
    full (its runtime-table query, k = 1e4, with the Lipinski bounds)."""
    import oracle
    import workloads.gen as gen
    base = cpu_baseline(lib_h, dec_h, q)
    base.update(cpu_info())
    counts = lib_h.reaction_counts()
    small = [min(range(len(counts)), key=lambda t: counts[t])]
    qs = type(q)(w=q.w, constraints=q.constraints, k=q.k, reactions=small)
    t0 = time.perf_counter()
    oracle.topk(lib_h, dec_h, qs, nthreads=1)
    dt1 = time.perf_counter() - t0
    base["single_thread"] = {"value": counts[small[0]] / dt1, "unit": "compounds/s",
                             "sample": f"reaction {small[0]} ({counts[small[0]]} compounds), {dt1:.1f} s"}
    base["benchmark_library_full_extrapolated_s"] = sum(counts) / base["value"]
    c0_lib, c0_dec, c0_q = gen.config_c0()
    t0 = time.perf_counter()
    oracle.topk(c0_lib, c0_dec, c0_q)
    base["tiny_case_full"] = {"seconds": time.perf_counter() - t0, "compounds": c0_lib.n_compounds}
    n_slots, sizes = gen.library_shapes_probe(11, 12_450_000)
    p_lib, p_dec = gen.config_probe(11, n_slots, sizes)
    hs = oracle.heads(p_lib, p_dec, gen.sample_ids(11, "probe_sample", p_lib.n_compounds, 1 << 14))
    pq = gen.probe_query(12, lambda h, p: float(np.quantile(hs[:, h], p)), 10**4, target=0)
    t0 = time.perf_counter()
    oracle.topk(p_lib, p_dec, pq)
    dtp = time.perf_counter() - t0
    base["probe_12M_full"] = {"seconds": dtp, "compounds_per_s": p_lib.n_compounds / dtp,
                              "compounds": p_lib.n_compounds,
                              "query": "linear probe, Lipinski-style bounds, k=1e4 (paper CPU: 0.7 s)"}
    return base


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--quick", action="store_true", help="headline precision only (profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c1", choices=["c1", "c3", "c4", "probe"],
                    help="c1: 1.04e7-compound library (default); c3: 2.9e10-compound streamed library; "
                         "c4: serving a query stream over subsets of the c3 library; probe: the paper's runtime "
                         "table alone (linear probe)")
    ap.add_argument("--probe-libraries", default="12M,10B,70B", help="probe workload: libraries to run")
    ap.add_argument("--serve-queries", type=int, default=None,
                    help="serving stream length (0: skip; default 80, c4: 2000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (reference for hardware byte counters)")
    ap.add_argument("--serve-qps", type=float, default=None, help="arrival rate (default 100/s, c4: 5/s)")
    ap.add_argument("--seq-queries", type=int, default=None,
                    help="arrivals timed one at a time in FP32 for comparison (default all, c4: 20)")
    ap.add_argument("--legs", default="c3,c4,probe,cpu",
                    help="legs added to the default c1 run: c3, c4 (needs c3), probe, cpu; '' for none")
    args = ap.parse_args()
    legs = set(x for x in args.legs.split(",") if x) if not args.quick else set()
    if args.no_cpu_baseline:
        legs.discard("cpu")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the search runs on a single MI355X (a multi-GPU run would split "
              "the reaction list into contiguous compound ranges, one per GPU, and merge the per-GPU top-k)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_24380_amd as apex
    import workloads.gen as gen
    from workloads.gen import ACT_SILU

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "c3":
        return main_c3(args)
    if args.workload == "probe":
        res = probe_leg(libraries=args.probe_libraries.split(","))
        print(json.dumps({"metric": "seconds per search (the paper's runtime table)", "probe_runtime_table": res}),
              flush=True)
        return
    c4 = args.workload == "c4"
    if args.serve_queries is None:
        args.serve_queries = 2000 if c4 else 80
    if args.serve_qps is None:
        args.serve_qps = 5.0 if c4 else 100.0
    if args.seq_queries is None and c4:
        args.seq_queries = 20
    if c4:
        return main_c4(args)
    lib_h, dec_h = gen.config_c1()
    q = load_query()
    tables = torch.from_numpy(lib_h.tables).to(dev)
    lib = apex.Library(lib_h.n_slots, lib_h.slot_sizes, tables)
    dec = apex.Decoder(dec_h.dims, "silu" if dec_h.act == ACT_SILU else "relu",
                       [torch.from_numpy(w).to(dev) for w in dec_h.W], [torch.from_numpy(b).to(dev) for b in dec_h.b])
    eng = apex.Engine(lib, dec, precisions=("fp32", "bf16", "fp8"))
    n = lib.num_compounds
    gold = golden_ids()
    flops_c = algorithmic_flops_per_compound(dec_h.dims)

    def run(prec, steps, warmup):
        for _ in range(warmup):
            eng.search(q, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = eng.search(q, precision=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rec = len(set(r.ids.tolist()) & set(gold)) / len(gold)
        return {"compounds_per_s": n / dt, "ms_per_step": dt * 1e3, "recall_at_k": rec,
                "exact_id_set": set(r.ids.tolist()) == set(gold),
                "candidates": r.n_candidates, "reruns": r.n_reruns}

    def kernel_roofline(prec, steps=3):
        eng.profile(True)
        for _ in range(steps):
            eng.search(q, precision=prec)
        ms, launches, comps = eng.profile(False)
        avg_ms = ms / max(launches, 1)
        flops_launch = flops_c * comps / max(launches, 1)
        achieved = flops_launch / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
        return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[prec], "traffic": measured_traffic(prec), "traffic_unit": "bytes/launch",
                "kernel": f"apex::{fused_kernel(prec)[0]} (fused)",
                "avg_launch_ms": avg_ms, "launches_per_step": launches / steps,
                "compounds_per_launch": comps / max(launches, 1), "flops_per_compound": flops_c,
                "valu": valu_estimate(prec, flops_c, comps / max(launches, 1), avg_ms)}

    sample = json.load(open(os.path.join(GOLDEN, "c1_heads_sample.json")))
    s_ids = np.array(sample["ids"], np.uint64)
    s_h64 = np.array(sample["heads"], np.float64)

    def head_error(prec):
        """Per-head |heads in this precision - FP64 heads| over 1024 seeded compounds."""
        err = np.abs(eng.heads(s_ids, prec).astype(np.float64) - s_h64)
        return {"max": [float(x) for x in err.max(0)], "mean": [float(x) for x in err.mean(0)]}

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    log(f"engine ready ({n} compounds); timing {args.precision}")
    head = run(args.precision, args.steps, args.warmup)
    roof = kernel_roofline(args.precision)
    log(f"{args.precision}: {head['compounds_per_s']:.4g} compounds/s, {head['ms_per_step']:.3f} ms/step")
    others = {}
    if not args.quick:
        for p in ("fp32", "bf16", "fp8"):
            if p != args.precision:
                others[p] = run(p, max(2, args.steps // 4), 1)
                others[p]["roofline_frac"] = kernel_roofline(p)["frac"]
                log(f"{p}: {others[p]['compounds_per_s']:.4g} compounds/s")
    out = {
        "metric": METRIC,
        "value": head["compounds_per_s"],
        "unit": "compounds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded N(0,1) synthon embeddings, Xavier-uniform decoder)",
        "config": {"workload": "10,373,770-compound synthetic CSL (40 reactions: 28 two-slot, 12 three-slot, "
                               "lognormal slot sizes median 150 in [20, 3000]), d=256, decoder 256->512->512 (SiLU)->15, "
                               "objective -head1, 4 one-sided bounds, k=1000; BF16/FP8 enumerate a 4k pool rescored "
                               "in FP32",
                   "n_compounds": n, "k": q.k, "precision": args.precision},
        "recall_at_k": head["recall_at_k"],
        "exact_id_set_vs_oracle": head["exact_id_set"],
        "candidates_appended": head["candidates"],
        "reruns": head["reruns"],
        "roofline": roof,
        "other_precisions": others,
        "head_error_vs_fp64": {p: head_error(p) for p in (("fp32", "bf16", "fp8") if not args.quick
                                                          else (args.precision,))},
    }
    if "fp32" in others and args.precision != "fp32":
        out["speedup_vs_fp32"] = head["compounds_per_s"] / others["fp32"]["compounds_per_s"]
    if args.serve_queries and not args.quick:
        H = np.array(json.load(open(os.path.join(GOLDEN, "c1_heads_sample.json")))["heads"])
        out["serving"] = serve_bench(eng, lib_h.reaction_counts(), H, args.serve_queries, args.serve_qps, 1e5, 1e7,
                                     n_seq=args.seq_queries)
        out["serving"]["stream"] = (f"{args.serve_queries} queries, Poisson {args.serve_qps}/s, reaction subsets "
                                    "of the 1.04e7-compound library with 1e5-1e7 compounds each")
        log("serving stream done")
        out["p99_latency_ms_c1_stream"] = out["serving"]["served"]["p99_latency_ms"]
    del eng
    torch.cuda.empty_cache()
    if not args.quick:
        ref = reference_gemm(("bf16", "fp8", "fp32"))
        out["reference_gemm"] = {"shape": "8192 x 8192 x 8192", "library": "hipBLASLt (torch.matmul; FP8: "
                                 "torch._scaled_mm, E4M3 operands, BF16 output)", **ref}
        roof["reference_gemm_tflops"] = ref[args.precision]["tflops"]
        roof["frac_of_reference_gemm"] = roof["achieved"] / ref[args.precision]["tflops"]
        for p, o in others.items():
            o["frac_of_reference_gemm"] = o["roofline_frac"] * PEAK[p] / 1e12 / ref[p]["tflops"]
        log("reference GEMM: " + ", ".join(f"{p} {v['tflops']:.0f} TFLOP/s" for p, v in ref.items()))
    if "c3" in legs:
        c3, c4 = c3_leg(serve_queries=60 if "c4" in legs else 0)
        out["c3"] = c3
        if c4 is not None:
            out["serving_c4"] = c4
            out["p99_latency_ms"] = c4["served"]["p99_latency_ms"]
            out["p99_latency_stream"] = c4["stream"]
    if "probe" in legs:
        out["probe_runtime_table"] = probe_leg()
    if "cpu" in legs:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline_full(lib_h, dec_h, q)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
