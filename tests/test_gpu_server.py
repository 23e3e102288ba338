"""Serving loop (continuous batching) through the C ABI: results in a mix of
concurrently active queries equal each query's result alone; admission waits
for pool memory; cancellation; a query larger than the pool is rejected."""
import math
import time

import numpy as np
import pytest
import torch

import oracle
import workloads.gen as g
from parity import check_fp32_exact, lowp_recall
from workloads.gen import ACT_RELU, ACT_SILU, Constraint, Query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib3():
    from gpu_helpers import device_objects
    lib_h = g.make_library(53, [2, 3, 2, 3, 2, 2], [37, 53, 11, 9, 17, 70, 30, 5, 4, 29, 60, 12, 44, 47], 256)
    dec_h = g.make_decoder(53, [256, 512, 512, 15], ACT_SILU)
    objs = device_objects(lib_h, dec_h)
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 7, dtype=np.uint64))
    return lib_h, dec_h, objs, sample


def queries(sample, n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w = rng.standard_normal(15).astype(np.float32)
        heads = rng.choice(15, size=int(rng.integers(2, 5)), replace=False)
        cons = []
        for h in heads:
            qv = float(np.float32(np.quantile(sample[:, h], rng.uniform(0.6, 0.9))))
            cons.append(Constraint(int(h), -math.inf, qv) if rng.random() < 0.5 else
                        Constraint(int(h), float(np.float32(np.quantile(sample[:, h], rng.uniform(0.1, 0.4)))),
                                   math.inf))
        k = int(rng.choice([10, 100, 400]))
        subset = None if rng.random() < 0.5 else sorted(rng.choice(6, size=int(rng.integers(1, 6)), replace=False).tolist())
        out.append(Query(w=w, constraints=cons, k=k, reactions=subset))
    return out


def test_mixed_stream_equals_alone(lib3):
    import paper_2510_24380_amd as apex
    lib_h, dec_h, (lib, dec, eng), sample = lib3
    qs = queries(sample, 10)
    precs = ["fp32", "bf16", "fp32", "fp8", "bf16", "fp32", "bf16", "fp32", "fp8", "fp32"]
    alone = [eng.search(q, precision=p) for q, p in zip(qs, precs)]
    srv = apex.Server(eng, pool_bytes=256 << 20, max_active=4, chunk_compounds=1500)
    try:
        tickets = []
        for i, (q, p) in enumerate(zip(qs, precs)):
            tickets.append(srv.submit(q, precision=p))
            if i % 3 == 2:
                time.sleep(0.002)  # arrivals while others run
        results = [srv.poll(t, timeout_ms=60000) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    print(f"stats: {st}", flush=True)
    hits = want = 0
    for i, (a, r) in enumerate(zip(alone, results)):
        assert r is not None, f"query {i} did not finish"
        assert np.array_equal(a.ids, r.ids), f"query {i} ({precs[i]}): ids differ alone vs mixed"
        assert np.array_equal(a.objective, r.objective)
        assert np.array_equal(a.reaction, r.reaction) and np.array_equal(a.synthon, r.synthon)
        # and each served answer is the FP64 oracle's
        if precs[i] == "fp32":
            check_fp32_exact(lib_h, dec_h, qs[i], r, f"served fp32 query {i}")
        else:
            h, k = lowp_recall(lib_h, dec_h, qs[i], r, f"served {precs[i]} query {i}")
            hits, want = hits + h, want + k
    print(f"served low precision: recall {hits}/{want}", flush=True)
    assert hits >= 0.99 * want
    assert st["completed"] == 10 and st["failed"] == 0
    assert st["p99_latency_ms"] >= st["p50_latency_ms"] > 0


def test_admission_waits_for_memory(lib3):
    import paper_2510_24380_amd as apex
    lib_h, dec_h, (lib, dec, eng), sample = lib3
    qs = queries(sample, 6, seed=1)
    one = eng.query_workspace_size(qs[0], precision="fp32")
    # room for the server state and about one query at a time
    srv = apex.Server(eng, pool_bytes=one + (8 << 20), max_active=4, chunk_compounds=1500)
    try:
        ts = [srv.submit(q, precision="fp32") for q in qs]
        st0 = srv.stats()
        res = [srv.poll(t, timeout_ms=60000) for t in ts]
    finally:
        srv.close()
    assert st0["waiting"] + st0["active"] + st0["completed"] == 6
    for q, r in zip(qs, res):
        assert r is not None
        a = eng.search(q, precision="fp32")
        assert np.array_equal(a.ids, r.ids)


def test_cancel_and_reject(lib3):
    import paper_2510_24380_amd as apex
    from paper_2510_24380_amd import ApexError
    lib_h, dec_h, (lib, dec, eng), sample = lib3
    qs = queries(sample, 3, seed=2)
    srv = apex.Server(eng, pool_bytes=64 << 20, max_active=2, chunk_compounds=500)
    try:
        ts = [srv.submit(q, precision="bf16") for q in qs]
        srv.cancel(ts[2])
        outcomes = []
        for t in ts:
            try:
                outcomes.append(srv.poll(t, timeout_ms=60000) is not None)
            except ApexError as e:
                assert e.status == -6  # cancelled
                outcomes.append("cancelled")
        assert outcomes[0] is True and outcomes[1] is True
        big = Query(w=np.ones(15, np.float32), constraints=[], k=1 << 22)
        with pytest.raises(ApexError) as ei:
            srv.submit(big, precision="fp32")
        assert ei.value.status == -2
    finally:
        srv.close()


@pytest.fixture(scope="module")
def big_lib():
    """538,600 compounds (three reactions): more than eight times the server's
    2^16-compound warm-start sample, with a small decoder."""
    from gpu_helpers import device_objects
    lib_h = g.make_library(89, [2, 3, 2], [700, 610, 40, 37, 45, 300, 150], 64)
    dec_h = g.make_decoder(89, [64, 128, 128, 5], ACT_RELU)
    objs = device_objects(lib_h, dec_h)
    sample = oracle.heads(lib_h, dec_h, g.sample_ids(7, "srv_sample", lib_h.n_compounds, 4096))
    return lib_h, dec_h, objs, sample


def test_served_warm_start_and_reruns_match_oracle(big_lib):
    """A forced small candidate buffer (below the warm-start sample size) and
    small chunks: the served queries take the warm start, overflow their
    buffers, re-run those chunks, and still return the oracle's answer; each
    equals the query searched alone."""
    import os
    import paper_2510_24380_amd as apex
    lib_h, dec_h, (lib, dec, eng), sample = big_lib
    assert lib_h.n_compounds >= 8 * (1 << 16)
    qs = [Query(w=np.array([1, 0, -0.5, 0, 0], np.float32),
                constraints=[Constraint(3, -math.inf, float(np.float32(np.quantile(sample[:, 3], 0.85))))], k=400),
          Query(w=np.array([0, 1, 0, 0, 0.3], np.float32), constraints=[], k=1000),
          Query(w=np.array([-1, 0, 0, 1, 0], np.float32),
                constraints=[Constraint(2, float(np.float32(np.quantile(sample[:, 2], 0.2))), math.inf)], k=50,
                reactions=[0, 2])]
    precs = ["fp32", "fp32", "bf16"]
    os.environ["APEX_TEST_CAP"] = "3000"
    try:
        print("case: served with a forced 3000-entry buffer", flush=True)
        srv = apex.Server(eng, pool_bytes=512 << 20, max_active=4, chunk_compounds=40000)
        try:
            tickets = [srv.submit(q, precision=p) for q, p in zip(qs, precs)]
            results = [srv.poll(t, timeout_ms=120000) for t in tickets]
        finally:
            srv.close()
        print("case: alone with a forced 3000-entry buffer", flush=True)
        alone = [eng.search(q, precision=p) for q, p in zip(qs, precs)]
    finally:
        del os.environ["APEX_TEST_CAP"]
    for i, (q, p, r, a) in enumerate(zip(qs, precs, results, alone)):
        print(f"served query {i}: reruns={r.n_reruns} candidates={r.n_candidates} scored={r.n_scored}", flush=True)
        assert r is not None
        assert np.array_equal(r.ids, a.ids) and np.array_equal(r.objective, a.objective)
        assert len(set(r.ids.tolist())) == len(r.ids)
        if p == "fp32":
            check_fp32_exact(lib_h, dec_h, q, r, f"served big fp32 query {i}")
        else:
            h, k = lowp_recall(lib_h, dec_h, q, r, f"served big {p} query {i}")
            assert h >= 0.99 * k
    assert sum(r.n_reruns for r in results) > 0
