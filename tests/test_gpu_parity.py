"""Parity of the HIP search (through the C ABI) with the FP64 oracle on seeded
libraries that span many tiles and ragged edges, in FP32 (exact id sets,
ties by id), BF16 and FP8 (recall against the oracle, FP32-rescored scores)."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads.gen as g
from workloads.gen import ACT_NONE, ACT_RELU, ACT_SILU, Constraint, Query

pytestmark = pytest.mark.gpu

from parity import check_fp32_exact, check_lowp, lowp_recall, nonfinite_case

if torch.cuda.is_available():
    from gpu_helpers import device_objects


# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c0():
    lib_h, dec_h, q = g.config_c0()
    objs = device_objects(lib_h, dec_h)
    return lib_h, dec_h, q, objs


def test_c0_fp32_exact(c0):
    lib_h, dec_h, q, (lib, dec, eng) = c0
    print("case: c0 fp32", flush=True)
    r = eng.search(q, precision="fp32")
    check_fp32_exact(lib_h, dec_h, q, r, "c0 fp32")


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_c0_low_precision(c0, prec):
    lib_h, dec_h, q, (lib, dec, eng) = c0
    print(f"case: c0 {prec}", flush=True)
    r = eng.search(q, precision=prec)
    check_lowp(lib_h, dec_h, q, r, f"c0 {prec}")


# A library with two- and three-slot reactions and ragged slot sizes, and the
# benchmark decoder shape (256 -> 512 -> 512 (SiLU) -> 15).
@pytest.fixture(scope="module")
def mixed():
    lib_h = g.make_library(41, [2, 3, 2, 3], [37, 53, 11, 9, 17, 70, 3, 5, 4, 29], 256)
    dec_h = g.make_decoder(41, [256, 512, 512, 15], ACT_SILU)
    objs = device_objects(lib_h, dec_h)
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 5, dtype=np.uint64))
    return lib_h, dec_h, objs, sample


def mixed_query(sample, k, q_hi=0.8, reactions=None):
    w = np.zeros(15, np.float32)
    w[2] = -1.0
    w[7] = 0.25
    cons = [Constraint(6, -math.inf, float(np.float32(np.quantile(sample[:, 6], q_hi)))),
            Constraint(11, float(np.float32(np.quantile(sample[:, 11], 0.25))), math.inf),
            Constraint(9, float(np.float32(np.quantile(sample[:, 9], 0.05))),
                       float(np.float32(np.quantile(sample[:, 9], 0.97))))]
    return Query(w=w, constraints=cons, k=k, reactions=reactions)


@pytest.mark.parametrize("k", [1, 50, 777])
def test_mixed_fp32_exact(mixed, k):
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print(f"case: mixed fp32 k={k}", flush=True)
    q = mixed_query(sample, k)
    r = eng.search(q, precision="fp32")
    check_fp32_exact(lib_h, dec_h, q, r, f"mixed fp32 k={k}")


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_mixed_low_precision(mixed, prec):
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print(f"case: mixed {prec}", flush=True)
    q = mixed_query(sample, 200)
    r = eng.search(q, precision=prec)
    check_lowp(lib_h, dec_h, q, r, f"mixed {prec}")


def test_mixed_subset_and_k_beyond_feasible(mixed):
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print("case: mixed subset", flush=True)
    q = mixed_query(sample, 5000, reactions=[1, 3])
    r = eng.search(q, precision="fp32")
    ref = check_fp32_exact(lib_h, dec_h, q, r, "mixed subset")
    assert ref.n_feasible < 5000 and len(r.ids) == ref.n_feasible


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_k_beyond_feasible(mixed, prec):
    """k above the number of feasible compounds, in the precisions whose tile
    passes share their tiles out between workgroups at run time: the answer is
    the feasible set, each compound once (no tile skipped or scored twice), and
    many small launches give the same bits as the default ones."""
    from parity import _feasible64, library_scales
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print(f"case: mixed subset, k beyond feasible, {prec}", flush=True)
    q = mixed_query(sample, 5000, reactions=[1, 3])
    r32 = eng.search(q, precision="fp32")
    ref = check_fp32_exact(lib_h, dec_h, q, r32, "fp32 reference")
    assert ref.n_feasible < 5000
    hs, _ = library_scales(lib_h, dec_h, q)
    runs = []
    for chunk in (None, "2048"):
        if chunk:
            os.environ["APEX_TEST_CHUNK"] = chunk
        try:
            r = eng.search(q, precision=prec)
        finally:
            os.environ.pop("APEX_TEST_CHUNK", None)
        ids = r.ids.tolist()
        assert len(set(ids)) == len(ids), f"{prec}: a compound returned twice"
        got, want = set(ids), set(r32.ids.tolist())
        # the answer is rescored in FP32 against the exact bounds
        extra = np.array(sorted(got - want), np.uint64)
        if len(extra):
            h64 = oracle.heads(lib_h, dec_h, extra)
            assert np.all(_feasible64(h64, q, slack=2e-5 * float(np.max(hs)))), f"{prec}: infeasible compound"
        # a feasible compound may be missed only within the low-precision error of a bound
        missing = np.array(sorted(want - got), np.uint64)
        if len(missing):
            h64 = oracle.heads(lib_h, dec_h, missing)
            near = ~_feasible64(h64, q, slack=-0.05 * float(np.max(hs)))
            assert np.all(near), f"{prec}: {int(np.sum(~near))} feasible compounds missed away from the bounds"
        print(f"[{prec} chunk={chunk}] {len(ids)} returned of {ref.n_feasible} feasible; "
              f"{len(missing)} missed at a bound, {len(extra)} extra at a bound", flush=True)
        runs.append(r)
    assert np.array_equal(runs[0].ids, runs[1].ids)
    assert np.array_equal(runs[0].objective.view(np.uint32), runs[1].objective.view(np.uint32))


def test_all_infeasible_returns_nothing(mixed):
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print("case: all infeasible", flush=True)
    q = Query(w=np.ones(15, np.float32), constraints=[Constraint(0, 1e30, math.inf)], k=10)
    for prec in ("fp32", "bf16", "fp8"):
        r = eng.search(q, precision=prec)
        assert len(r.ids) == 0


def test_forced_chunks_and_overflow_reruns(mixed):
    """Many small chunks and a tiny candidate buffer (forced from the host) give
    the same answer; the overflow path re-runs chunks."""
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print("case: forced chunks + overflow", flush=True)
    q = mixed_query(sample, 300, q_hi=0.95)
    base = eng.search(q, precision="fp32")
    os.environ["APEX_TEST_CHUNK"] = "2048"
    os.environ["APEX_TEST_CAP"] = "700"
    try:
        r = eng.search(q, precision="fp32")
    finally:
        del os.environ["APEX_TEST_CHUNK"]
        del os.environ["APEX_TEST_CAP"]
    print(f"reruns={r.n_reruns} candidates={r.n_candidates}", flush=True)
    assert r.n_reruns > 0
    assert np.array_equal(r.ids, base.ids) and np.array_equal(r.objective, base.objective)
    check_fp32_exact(lib_h, dec_h, q, r, "forced")


def test_fused_batch_equals_single(mixed):
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print("case: fused batch", flush=True)
    qs = [mixed_query(sample, 100), mixed_query(sample, 10, q_hi=0.6, reactions=[0, 2]),
          Query(w=np.eye(15, dtype=np.float32)[4], constraints=[], k=333)]
    for prec in ("fp32", "bf16"):
        fused = eng.search_batch(qs, precision=prec)
        for q, f in zip(qs, fused):
            single = eng.search(q, precision=prec)
            assert np.array_equal(f.ids, single.ids) and np.array_equal(f.objective, single.objective)


def test_fused_batch_of_32_queries(mixed):
    """The most queries one pass fuses (32): objectives over all 15 heads,
    bounds, k and reaction subsets all differ. Every fused answer equals the
    query searched alone and the FP64 oracle's answer (FP32: exact id set;
    BF16/FP8: recall over the batch and every returned compound re-scored)."""
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    print("case: fused batch of 32", flush=True)
    rng = np.random.default_rng(61)
    subsets = [None, [0, 2], [1], [3], [0, 1, 2, 3], [2, 3]]
    qs = []
    for i in range(32):
        w = rng.standard_normal(15).astype(np.float32)
        base = mixed_query(sample, 1 + int(rng.integers(0, 300)), q_hi=float(rng.uniform(0.5, 0.95)),
                           reactions=subsets[i % len(subsets)])
        qs.append(Query(w=w, constraints=base.constraints if i % 3 else [], k=base.k, reactions=base.reactions))
    assert all(np.all(q.w != 0) for q in qs)
    for prec in ("fp32", "bf16", "fp8"):
        print(f"case: fused batch of 32 {prec}", flush=True)
        fused = eng.search_batch(qs, precision=prec)
        assert len(fused) == 32
        hits = want = 0
        for i, (q, f) in enumerate(zip(qs, fused)):
            single = eng.search(q, precision=prec)
            assert np.array_equal(f.ids, single.ids), f"{prec} query {i}"
            assert np.array_equal(f.objective, single.objective), f"{prec} query {i}"
            if prec == "fp32":
                check_fp32_exact(lib_h, dec_h, q, f, f"fused fp32 query {i}")
            else:
                h, k = lowp_recall(lib_h, dec_h, q, f, f"fused {prec} query {i}")
                hits, want = hits + h, want + k
        if prec != "fp32":
            print(f"fused {prec}: recall over the batch {hits}/{want}", flush=True)
            assert hits >= 0.99 * want


def test_objective_bits_equal_listed_heads(mixed):
    """With w = e_h the objective of every returned compound is its head h, and
    the listed-compound kernels (warm-start sample, rescoring, answer heads) give
    the same bits as the enumeration that found it."""
    lib_h, dec_h, (lib, dec, eng), sample = mixed
    for prec in ("fp32", "bf16", "fp8"):
        for h in (0, 6, 14):
            print(f"case: objective = head {h} {prec}", flush=True)
            q = Query(w=np.eye(15, dtype=np.float32)[h], constraints=[], k=400)
            r = eng.search(q, precision=prec)
            heads = eng.heads(r.ids, "fp32")
            assert np.array_equal(r.objective.view(np.uint32), (heads[:, h] + 0.0).astype(np.float32).view(np.uint32))
            assert np.array_equal(r.heads.view(np.uint32), heads.view(np.uint32))
            if prec == "fp32":
                check_fp32_exact(lib_h, dec_h, q, r, f"objective = head {h}")


@pytest.mark.parametrize("dims,act", [([8, 3], ACT_NONE), ([16, 128, 64, 3], ACT_SILU)], ids=["linear", "mlp"])
def test_nonfinite_compounds_never_returned(dims, act):
    """Table rows holding +Inf or NaN make their compounds' heads non-finite;
    such compounds are never returned (the oracle's rule), in every precision,
    and the low-precision calibration ignores them."""
    lib_h, dec_h, q = nonfinite_case(dims, act)
    precs = ("fp32",) if len(dims) == 2 else ("fp32", "bf16", "fp8")
    lib, dec, eng = device_objects(lib_h, dec_h, precisions=precs)
    ref = oracle.topk(lib_h, dec_h, q)
    for prec in precs:
        print(f"case: non-finite rows {dims} {prec}", flush=True)
        r = eng.search(q, precision=prec)
        assert np.all(np.isfinite(r.objective)) and np.all(np.isfinite(r.heads))
        if prec == "fp32":
            check_fp32_exact(lib_h, dec_h, q, r, f"non-finite {prec}")
        else:
            check_lowp(lib_h, dec_h, q, r, f"non-finite {prec}")
        assert len(r.ids) == min(q.k, ref.n_feasible)


def test_ties_lower_id_wins():
    """Duplicated synthon rows give identical scores; lower ids rank first."""
    print("case: ties", flush=True)
    lib_h = g.make_library(43, [2], [40, 33], 64)
    lib_h.tables[5] = lib_h.tables[1]
    lib_h.tables[9] = lib_h.tables[1]
    lib_h.tables[40 + 7] = lib_h.tables[40 + 2]
    dec_h = g.make_decoder(43, [64, 128, 5], ACT_RELU)
    lib, dec, eng = device_objects(lib_h, dec_h, precisions=("fp32",))
    q = Query(w=np.array([1, 0, 0, 0, 0], np.float32), constraints=[], k=600)
    r = eng.search(q, precision="fp32")
    check_fp32_exact(lib_h, dec_h, q, r, "ties")
    o = r.objective
    assert any(o[i] == o[i + 1] for i in range(len(o) - 1))


@pytest.fixture(scope="module")
def dup_lib():
    """90,000 compounds with only 200 distinct embeddings (10 distinct rows in
    slot 0, 20 in slot 1): every objective is shared by 450 compounds."""
    lib_h = g.make_library(53, [2], [300, 300], 64)
    for r in range(300):
        lib_h.tables[r] = lib_h.tables[r % 10]
        lib_h.tables[300 + r] = lib_h.tables[300 + r % 20]
    dec_h = g.make_decoder(53, [64, 128, 5], ACT_RELU)
    return lib_h, dec_h, device_objects(lib_h, dec_h, precisions=("fp32",))


def test_many_ties_large_buffers(dup_lib):
    """Selections over tens of thousands of candidates (the sampled-pivot path)
    split a K-th key shared by hundreds of compounds by id; the same with many
    small chunks and a forced small buffer (overflow re-runs)."""
    lib_h, dec_h, (lib, dec, eng) = dup_lib
    print("case: many ties, large buffers", flush=True)
    q = Query(w=np.array([1, 0, 0, 0, 0], np.float32), constraints=[], k=5000)
    r = eng.search(q, precision="fp32")
    check_fp32_exact(lib_h, dec_h, q, r, "many ties")
    assert r.objective[-1] == r.objective[-2]
    # the first 32,768-compound chunk overflows a 14,000-entry buffer
    os.environ["APEX_TEST_CHUNK"] = "32768"
    os.environ["APEX_TEST_CAP"] = "14000"
    try:
        r2 = eng.search(q, precision="fp32")
    finally:
        del os.environ["APEX_TEST_CHUNK"]
        del os.environ["APEX_TEST_CAP"]
    print(f"reruns={r2.n_reruns}", flush=True)
    assert r2.n_reruns > 0
    assert np.array_equal(r2.ids, r.ids) and np.array_equal(r2.objective, r.objective)


def test_all_equal_objectives(dup_lib):
    """A zero objective ties every compound: the answer is the k smallest ids."""
    lib_h, dec_h, (lib, dec, eng) = dup_lib
    print("case: all objectives equal", flush=True)
    q = Query(w=np.zeros(5, np.float32), constraints=[], k=5000)
    r = eng.search(q, precision="fp32")
    assert np.array_equal(r.ids, np.arange(5000, dtype=np.uint64))
    assert np.all(r.objective == 0.0)


@pytest.fixture(scope="module")
def wide():
    """39,600 compounds (two- and three-slot reactions) for answers longer than
    the one-workgroup sort holds."""
    lib_h = g.make_library(59, [2, 2, 3], [150, 120, 90, 200, 20, 15, 12], 64)
    dec_h = g.make_decoder(59, [64, 128, 128, 5], ACT_SILU)
    return lib_h, dec_h, device_objects(lib_h, dec_h, precisions=("fp32", "bf16", "fp8"))


def test_answers_longer_than_one_workgroup_sort(wide):
    """k = 9000 (> 8192): the FP32 answer is ordered by the multi-workgroup rank
    sort, and the BF16 / FP8 pools (36,000 entries) are selected before that sort."""
    lib_h, dec_h, (lib, dec, eng) = wide
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 7, dtype=np.uint64))
    lo = float(np.float32(np.quantile(sample[:, 1], 0.3)))
    q = Query(w=np.array([1, 0, -0.5, 0, 0], np.float32), constraints=[Constraint(1, lo, math.inf)], k=9000)
    print("case: k=9000 fp32", flush=True)
    r = eng.search(q, precision="fp32")
    ref = check_fp32_exact(lib_h, dec_h, q, r, "k=9000 fp32")
    assert ref.n_feasible > 9000
    for prec in ("bf16", "fp8"):
        print(f"case: k=9000 {prec}", flush=True)
        r = eng.search(q, precision=prec)
        check_lowp(lib_h, dec_h, q, r, f"k=9000 {prec}")


def test_ids_beyond_32_bits():
    """A first reaction of 4.9e9 compounds pushes the second reaction's ids past
    2^32; a subset query on the second reaction returns the exact ids."""
    print("case: 64-bit ids", flush=True)
    lib_h = g.make_library(47, [2, 2], [70000, 70000, 30, 45], 64)
    dec_h = g.make_decoder(47, [64, 128, 5], ACT_RELU)
    lib, dec, eng = device_objects(lib_h, dec_h, precisions=("fp32",))
    q = Query(w=np.array([0, 1, 0, 0, 0], np.float32), constraints=[], k=40, reactions=[1])
    r = eng.search(q, precision="fp32")
    assert r.ids.min() >= 70000 * 70000 > 2 ** 32
    check_fp32_exact(lib_h, dec_h, q, r, "64-bit ids")


@pytest.mark.parametrize("shape", [([2, 3, 2, 3], [37, 53, 11, 9, 17, 70, 3, 5, 4, 29], 256, 15),
                                   ([2], [300, 300], 64, 5)])
def test_linear_probe_decoder_exact(shape):
    """One-layer decoder, the paper's linear heads (eq. "apex"): FP32 exact."""
    from workloads.gen import ACT_NONE
    n_slots, sizes, d, H = shape
    print(f"case: linear probe d={d} H={H}", flush=True)
    lib_h = g.make_library(59, n_slots, sizes, d)
    dec_h = g.make_decoder(59, [d, H], ACT_NONE)
    lib, dec, eng = device_objects(lib_h, dec_h, precisions=("fp32",))
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 3, dtype=np.uint64))
    w = np.zeros(H, np.float32)
    w[0], w[H - 1] = 1.0, -0.5
    cons = [Constraint(1, -math.inf, float(np.float32(np.quantile(sample[:, 1], 0.7)))),
            Constraint(2, float(np.float32(np.quantile(sample[:, 2], 0.2))), math.inf)]
    for k in (1, 100, 2000):
        q = Query(w=w, constraints=cons, k=k)
        r = eng.search(q, precision="fp32")
        check_fp32_exact(lib_h, dec_h, q, r, f"linear k={k}")
