"""Linear-probe engines (one decoder layer, up to 32 heads): the paper's own
scalar-contribution search (Section 4.3, eq. "apex"; Appendix A.5) through the
C ABI against the FP64 oracle, whose one-layer case is pinned to the closed form
of eq. "apex". 28 heads as in the paper's LinearProbe (Appendix A.8), bounds on
heads past 16, ragged two- and three-slot reactions spanning several 64 x 64
tiles, the warm start, forced chunks with candidate-buffer overflows, fused
batches, the serving loop, non-finite rows and answers longer than one
workgroup's sort (radix-sorted)."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads.gen as g
from workloads.gen import ACT_NONE, Constraint, Query

pytestmark = pytest.mark.gpu

from parity import check_fp32_exact, nonfinite_case

if torch.cuda.is_available():
    import paper_2510_24380_amd as apex
    from gpu_helpers import device_objects

H = 28


def _objs(lib_h, dec_h):
    return device_objects(lib_h, dec_h, precisions=("fp32",))


# 43,245 compounds: reactions of 150 x 70, 9 x 13 x 200, 65 x 129 and 3 x 5 x 64
@pytest.fixture(scope="module")
def small():
    lib_h = g.make_library(51, [2, 3, 2, 3], [150, 70, 9, 13, 200, 65, 129, 3, 5, 64], 64)
    dec_h = g.make_decoder(51, [64, H], ACT_NONE)
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 7, dtype=np.uint64))
    return lib_h, dec_h, _objs(lib_h, dec_h), sample


# 984,700 compounds: large enough for the threshold warm start
@pytest.fixture(scope="module")
def large():
    lib_h = g.make_library(52, [2, 3, 2], [700, 900, 40, 30, 60, 257, 1100], 64)
    dec_h = g.make_decoder(52, [64, H], ACT_NONE)
    sample = oracle.heads(lib_h, dec_h, g.sample_ids(52, "probe_sample", lib_h.n_compounds, 1 << 14))
    return lib_h, dec_h, _objs(lib_h, dec_h), sample


def _quantile(sample):
    return lambda h, q: float(np.quantile(sample[:, h], q))


def _wide_query(sample, k, reactions=None):
    """Objective over all 28 heads (seeded normal weights), bounds on heads 5,
    17 (two-sided) and 27."""
    w = g.normal_f32(53, "probe_w", H)
    q = _quantile(sample)
    cons = [Constraint(5, -math.inf, float(np.float32(q(5, 0.8)))),
            Constraint(17, float(np.float32(q(17, 0.1))), float(np.float32(q(17, 0.95)))),
            Constraint(27, float(np.float32(q(27, 0.3))), math.inf)]
    return Query(w=w, constraints=cons, k=k, reactions=reactions)


@pytest.mark.parametrize("k", [1, 50, 777])
def test_linear_fp32_exact(small, k):
    lib_h, dec_h, (lib, dec, eng), sample = small
    print(f"case: linear small k={k}", flush=True)
    q = _wide_query(sample, k)
    r = eng.search(q)
    check_fp32_exact(lib_h, dec_h, q, r, f"linear small k={k}")


def test_linear_docking_lipinski(large):
    """The runtime table's query shape (docking head minimised under four upper
    bounds), with the warm start."""
    lib_h, dec_h, (lib, dec, eng), sample = large
    for target in range(5):
        q = g.probe_query(54, _quantile(sample), 1000, target=target)
        print(f"case: linear large lipinski target={target}", flush=True)
        r = eng.search(q)
        assert r.n_scored >= lib_h.n_compounds
        check_fp32_exact(lib_h, dec_h, q, r, f"linear large target={target}")


@pytest.mark.parametrize("k", [9000, 20000])
def test_linear_long_answer(large, k):
    """Answers above 8192 entries are radix-sorted."""
    lib_h, dec_h, (lib, dec, eng), sample = large
    print(f"case: linear large k={k}", flush=True)
    q = _wide_query(sample, k)
    r = eng.search(q)
    check_fp32_exact(lib_h, dec_h, q, r, f"linear large k={k}")


def test_linear_forced_chunks_and_overflow(large, monkeypatch):
    lib_h, dec_h, (lib, dec, eng), sample = large
    monkeypatch.setenv("APEX_TEST_CHUNK", "40000")
    monkeypatch.setenv("APEX_TEST_CAP", "1200")
    # the guaranteed warm-start bound (rank K), looser than the speculative one,
    # so that the small buffer overflows
    monkeypatch.setenv("APEX_TEST_SPEC_RANK", str(1 << 30))
    q = _wide_query(sample, 300)
    print("case: linear forced chunks / cap", flush=True)
    r = eng.search(q)
    print(f"[forced] reruns={r.n_reruns} candidates={r.n_candidates}", flush=True)
    assert r.n_reruns > 0
    check_fp32_exact(lib_h, dec_h, q, r, "linear forced chunks")


def test_linear_speculative_threshold_redo(large, monkeypatch):
    """A warm-start threshold above the final K-th key (forced: the best sampled
    key) leaves fewer than K survivors; the query is enumerated again without it
    and the answer is still exact."""
    lib_h, dec_h, (lib, dec, eng), sample = large
    q = _wide_query(sample, 2000)
    monkeypatch.setenv("APEX_TEST_SPEC_RANK", "1")
    print("case: linear forced speculative rank 1", flush=True)
    r = eng.search(q)
    print(f"[spec] reruns={r.n_reruns} scored={r.n_scored}", flush=True)
    assert r.n_reruns > 0 and r.n_scored >= 2 * lib_h.n_compounds
    check_fp32_exact(lib_h, dec_h, q, r, "linear speculative redo")
    monkeypatch.delenv("APEX_TEST_SPEC_RANK")
    assert np.array_equal(eng.search(q).ids, r.ids)


def _violation64(lib_h, dec_h, q, ids):
    h = oracle.heads(lib_h, dec_h, np.asarray(ids, np.uint64))
    c = np.zeros(len(ids))
    for k in q.constraints:
        c -= np.maximum(0.0, k.lo - h[:, k.head]) + np.maximum(0.0, h[:, k.head] - k.hi)
    return c


def _check_keep_violators(lib_h, dec_h, q, r, sample, label):
    """Feasible compounds first (the exact feasible top-k), then violators by
    violation, against the oracle's lexicographic queue kept without its final
    removal (Section 4.3)."""
    ids, o, c = oracle.topk_lex(lib_h, dec_h, q, keep_violators=True, with_violation=True)
    nf = int(np.sum(c == 0.0))
    print(f"[{label}] feasible={nf} answer={len(ids)} gpu={len(r.ids)}", flush=True)
    assert len(r.ids) == len(ids)
    assert np.all(r.violation[:nf] == 0.0) and np.all(r.violation[nf:] < 0.0)
    scale = float(np.max(np.sqrt(np.mean(sample ** 2, axis=0))))
    tol = 1e-5 * np.maximum(np.abs(c[nf:]), scale)
    # the feasible part is the ordinary answer
    assert set(r.ids[:nf].tolist()) == set(ids[:nf].tolist()), f"{label}: feasible part"
    # violators: same ids unless their violations sit within FP32 error of the cut
    got, want = set(r.ids[nf:].tolist()), set(ids[nf:].tolist())
    if got != want:
        diff = np.array(sorted(got ^ want), np.uint64)
        cd = _violation64(lib_h, dec_h, q, diff)
        assert np.all(np.abs(cd - c[-1]) <= 4 * 1e-5 * scale), f"{label}: violators differ away from the cut"
        print(f"[{label}] {len(diff)} violators differ, all within FP32 error of the cut", flush=True)
    c_gpu64 = _violation64(lib_h, dec_h, q, r.ids[nf:])
    assert np.all(np.abs(r.violation[nf:] - c_gpu64) <= 1e-5 * np.maximum(np.abs(c_gpu64), scale)), label
    assert np.all(np.diff(r.violation[nf:].astype(np.float64)) <= 0.0), f"{label}: violation order"
    h64 = oracle.heads(lib_h, dec_h, r.ids)
    o64 = h64 @ np.asarray(q.w, np.float64)
    oscale = float(np.sqrt(np.mean((sample @ np.asarray(q.w, np.float64)) ** 2)))
    assert np.all(np.abs(r.objective - o64) <= 1e-5 * np.maximum(np.abs(o64), oscale)), f"{label}: objectives"
    assert np.all(np.abs(r.heads - h64) <= 1e-5 * np.maximum(np.abs(h64), scale)), f"{label}: heads"


def _stringent(sample, k, keep=True):
    qf = _quantile(sample)
    w = g.normal_f32(59, "probe_w3", H)
    cons = [Constraint(3, -math.inf, float(np.float32(qf(3, 0.05)))),
            Constraint(11, float(np.float32(qf(11, 0.9))), math.inf),
            Constraint(11, -math.inf, float(np.float32(qf(11, 0.97)))),
            Constraint(22, float(np.float32(qf(22, 0.4))), float(np.float32(qf(22, 0.6))))]
    return Query(w=w, constraints=cons, k=k, keep_violators=keep)


@pytest.mark.parametrize("k", [40, 600])
def test_linear_keep_violators(small, k):
    lib_h, dec_h, (lib, dec, eng), sample = small
    q = _stringent(sample, k)
    print(f"case: linear keep violators k={k}", flush=True)
    r = eng.search(q)
    _check_keep_violators(lib_h, dec_h, q, r, sample, f"keep violators k={k}")
    plain = eng.search(_stringent(sample, k, keep=False))
    nf = len(plain.ids)
    assert np.array_equal(r.ids[:nf], plain.ids) and np.array_equal(r.objective[:nf], plain.objective)


def test_linear_keep_violators_warm_start(large):
    """The violation pass over a library large enough for its own warm start."""
    lib_h, dec_h, (lib, dec, eng), sample = large
    q = _stringent(sample, 1500)
    print("case: linear keep violators (warm start)", flush=True)
    r = eng.search(q)
    _check_keep_violators(lib_h, dec_h, q, r, sample, "keep violators large")


def test_head_quantiles_and_counter_screen(large):
    """Head quantiles over listed compounds equal numpy's linear-interpolation
    quantiles of the FP64 heads (within FP32 error); a counter-screening query
    (Appendix A.11: minimise one docking head with the four others above their
    median, the medians from the engine's own sample) is exact against the
    oracle."""
    lib_h, dec_h, (lib, dec, eng), sample = large
    ids = g.sample_ids(60, "quantile_ids", lib_h.n_compounds, 5000)
    levels = [0.0, 0.05, 0.5, 0.9, 1.0]
    print("case: head quantiles", flush=True)
    got = eng.head_quantiles(levels, ids=ids)
    h64 = oracle.heads(lib_h, dec_h, ids)
    want = np.quantile(h64, levels, axis=0)
    scale = np.sqrt(np.mean(h64 ** 2, axis=0))
    assert got.shape == (len(levels), H)
    assert np.all(np.abs(got - want) <= 1e-5 * np.maximum(np.abs(want), scale))
    med = eng.head_quantiles([0.5], n=8192)[0]
    assert np.all(np.abs(med - np.median(sample, axis=0)) <= 0.1 * np.std(sample, axis=0))
    w = np.zeros(H, np.float32)
    w[0] = -1.0
    q = Query(w=w, constraints=[Constraint(h, float(med[h]), math.inf) for h in (1, 2, 3, 4)], k=2000)
    print("case: counter-screen query", flush=True)
    check_fp32_exact(lib_h, dec_h, q, eng.search(q), "counter-screen")


def test_linear_batch_equals_single_and_oracle(small):
    lib_h, dec_h, (lib, dec, eng), sample = small
    qs = [_wide_query(sample, 40), _wide_query(sample, 500, reactions=[1, 3]),
          g.probe_query(55, _quantile(sample), 100, target=2),
          Query(w=g.normal_f32(56, "probe_w2", H), constraints=[], k=1000),
          _wide_query(sample, 7, reactions=[2])]
    print("case: linear fused batch of 5", flush=True)
    rs = eng.search_batch(qs)
    for i, (q, r) in enumerate(zip(qs, rs)):
        alone = eng.search(q)
        assert np.array_equal(r.ids, alone.ids) and np.array_equal(r.objective, alone.objective), i
        check_fp32_exact(lib_h, dec_h, q, r, f"linear batch {i}")


def test_linear_heads_and_decode(small):
    lib_h, dec_h, (lib, dec, eng), sample = small
    ids = np.concatenate([np.arange(0, lib_h.n_compounds, 97, dtype=np.uint64),
                          np.array([lib_h.n_compounds - 1, lib_h.n_compounds], np.uint64)])
    print("case: linear heads", flush=True)
    h = eng.heads(ids)
    h64 = oracle.heads(lib_h, dec_h, ids[:-1])
    scale = np.sqrt(np.mean(sample ** 2, axis=0))
    assert h.shape == (len(ids), H)
    assert np.all(np.abs(h[:-1] - h64) <= 1e-5 * np.maximum(np.abs(h64), scale))
    assert np.all(np.isnan(h[-1]))


def test_linear_nonfinite_rows():
    lib_h, dec_h, q = nonfinite_case([64, H], ACT_NONE)
    lib, dec, eng = _objs(lib_h, dec_h)
    print("case: linear non-finite rows", flush=True)
    r = eng.search(q)
    assert np.all(np.isfinite(r.objective)) and np.all(np.isfinite(r.heads))
    check_fp32_exact(lib_h, dec_h, q, r, "linear non-finite")


def test_linear_server(large):
    lib_h, dec_h, (lib, dec, eng), sample = large
    qs = [_wide_query(sample, 100), g.probe_query(57, _quantile(sample), 1000, target=1),
          _wide_query(sample, 50, reactions=[0])]
    print("case: linear server", flush=True)
    srv = apex.Server(eng, pool_bytes=512 << 20, max_active=4, chunk_compounds=1 << 18)
    try:
        tickets = [srv.submit(q) for q in qs]
        served = [srv.poll(t) for t in tickets]
    finally:
        srv.close()
    for i, (q, r) in enumerate(zip(qs, served)):
        alone = eng.search(q)
        assert np.array_equal(r.ids, alone.ids) and np.array_equal(r.objective, alone.objective), i
        check_fp32_exact(lib_h, dec_h, q, r, f"linear served {i}")


def test_linear_decoder_limits():
    """A one-layer decoder may have up to 32 heads; decoders with hidden layers
    keep 16."""
    dev = torch.device("cuda:0")
    lib_h = g.make_library(58, [2], [20, 30], 16)
    tables = torch.from_numpy(lib_h.tables).to(dev)
    lib = apex.Library(lib_h.n_slots, lib_h.slot_sizes, tables)
    for dims, ok in (([16, 32], True), ([16, 33], False), ([16, 128, 17], False)):
        d = g.make_decoder(58, dims, ACT_NONE if len(dims) == 2 else 1)
        args = (dims, "none" if len(dims) == 2 else "relu", [torch.from_numpy(w).to(dev) for w in d.W],
                [torch.from_numpy(b).to(dev) for b in d.b])
        if ok:
            apex.Decoder(*args)
        else:
            with pytest.raises(apex.ApexError):
                apex.Decoder(*args)
