"""Pins for the FP64 oracle against facts that do not depend on its own code:
the paper's worked example, brute force over subsets (the definition of the
retrieval problem), a library forward pass (torch, fp64), the linear closed form
of eq. "apex", a textbook sorted-sums property, permutation invariance, ties, the
paper's lexicographic priority-queue form and degenerate queries."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads.gen as g
from workloads.gen import ACT_NONE, ACT_RELU, ACT_SILU, Constraint, Query

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def small_library(seed, n_slots, sizes, d):
    return g.make_library(seed, n_slots, sizes, d)


def torch_heads(lib, dec, t, idx):
    """Forward pass of one compound with torch fp64 library layers."""
    rows = []
    p = int(np.sum(lib.n_slots[:t]))
    base = int(np.sum(lib.slot_sizes[:p]))
    for s in range(int(lib.n_slots[t])):
        rows.append(base + idx[s])
        base += int(lib.slot_sizes[p + s])
    x = torch.tensor(lib.tables[rows].astype(np.float64)).sum(0)
    acts = {ACT_RELU: torch.relu, ACT_SILU: torch.nn.functional.silu, ACT_NONE: lambda v: v}
    for l in range(dec.n_layers):
        x = torch.nn.functional.linear(x, torch.tensor(dec.W[l], dtype=torch.float64),
                                       torch.tensor(dec.b[l], dtype=torch.float64))
        if l + 1 < dec.n_layers:
            x = acts[dec.act](x)
    return x.numpy()


def all_compounds(lib):
    """(id, t, idx) in the id order the paper's multi-index is read in: reaction,
    then slot 0 most significant."""
    out, p, cid = [], 0, 0
    for t in range(lib.n_reactions):
        ns = int(lib.n_slots[t])
        sizes = [int(x) for x in lib.slot_sizes[p:p + ns]]
        for idx in itertools.product(*[range(n) for n in sizes]):
            out.append((cid, t, idx))
            cid += 1
        p += ns
    return out


def brute_force(lib, dec, q):
    """Eq. "apex_topk" by definition: among feasible compounds, the subset of size
    min(k, n_feasible) with the largest objective sum (checked over all subsets)."""
    feas = []
    for cid, t, idx in all_compounds(lib):
        if q.reactions is not None and t not in q.reactions:
            continue
        h = torch_heads(lib, dec, t, idx)
        if all(c.lo <= h[c.head] <= c.hi for c in q.constraints):
            feas.append((cid, float(np.dot(q.w.astype(np.float64), h))))
    m = min(q.k, len(feas))
    best, best_sum = None, -math.inf
    for sub in itertools.combinations(range(len(feas)), m):
        s = sum(feas[i][1] for i in sub)
        if s > best_sum:
            best, best_sum = sub, s
    return set(feas[i][0] for i in best) if best is not None else set(), feas


def test_worked_example_counts():
    ex = json.load(open(os.path.join(GOLDEN, "paper_worked_example.json")))
    n = ex["synthons_per_slot"]
    lib = g.Library(n_slots=np.array([3], np.uint32), slot_sizes=np.array([n, n, n], np.uint32), d=1,
                    tables=np.zeros((3 * n, 1), np.float32))
    assert lib.n_rows == ex["n_synthons_total"]
    assert oracle.num_compounds(lib) == ex["n_products"]
    # ids beyond 2^32 decode to the mixed-radix digits, slot 0 most significant
    ids = np.array([0, 1, n, n * n, 2**32 + 7, ex["n_products"] - 1], dtype=np.uint64)
    r, s = oracle.decode(lib, ids)
    assert (r == 0).all()
    for i, cid in enumerate(ids.tolist()):
        assert s[i].tolist() == [cid // (n * n), (cid // n) % n, cid % n]
    with pytest.raises(ValueError):
        oracle.decode(lib, np.array([ex["n_products"]], dtype=np.uint64))


def test_id_order_is_bijective_and_ordered():
    lib = small_library(3, [2, 3, 2], [3, 4, 2, 3, 2, 5, 1], 4)
    comps = all_compounds(lib)
    ids = np.array([c[0] for c in comps], dtype=np.uint64)
    assert oracle.num_compounds(lib) == len(comps)
    r, s = oracle.decode(lib, ids)
    for i, (cid, t, idx) in enumerate(comps):
        assert r[i] == t
        assert tuple(s[i][:len(idx)]) == idx
        assert all(v == 0 for v in s[i][len(idx):])


@pytest.mark.parametrize("act", [ACT_RELU, ACT_SILU, ACT_NONE])
def test_forward_matches_torch(act):
    lib = small_library(5, [2, 3], [7, 5, 4, 3, 6], 16)
    dec = g.make_decoder(5, [16, 24, 12, 6], act)
    comps = all_compounds(lib)
    pick = [comps[i] for i in range(0, len(comps), 7)]
    ids = np.array([c[0] for c in pick], dtype=np.uint64)
    h = oracle.heads(lib, dec, ids)
    for i, (_, t, idx) in enumerate(pick):
        ref = torch_heads(lib, dec, t, idx)
        np.testing.assert_allclose(h[i], ref, rtol=1e-12, atol=1e-12)


def test_linear_decoder_is_the_apex_factorisation():
    """One linear layer: heads = sum over slots of v_{i,r,s} + b_i (eq. "apex"),
    with v = W u precomputed per synthon row."""
    lib = small_library(7, [2, 3], [9, 6, 5, 4, 3], 32)
    dec = g.make_decoder(7, [32, 5], ACT_NONE)
    v = lib.tables.astype(np.float64) @ dec.W[0].astype(np.float64).T  # [rows, H]
    comps = all_compounds(lib)
    ids = np.array([c[0] for c in comps], dtype=np.uint64)
    h = oracle.heads(lib, dec, ids)
    slot_row0 = np.concatenate([[0], np.cumsum(lib.slot_sizes.astype(np.int64))[:-1]])
    p_of_t = np.concatenate([[0], np.cumsum(lib.n_slots.astype(np.int64))[:-1]])
    for i, (_, t, idx) in enumerate(comps):
        ref = dec.b[0].astype(np.float64).copy()
        for s, j in enumerate(idx):
            ref += v[int(slot_row0[int(p_of_t[t]) + s]) + j]
        np.testing.assert_allclose(h[i], ref, rtol=1e-12, atol=1e-12)


def test_hoisted_first_layer_equals_unhoisted():
    """Distributing the first layer over the slot sum (the hoist the GPU uses)
    agrees with the oracle's plain sum-then-project to fp64 rounding."""
    lib = small_library(8, [3], [4, 3, 5], 24)
    dec = g.make_decoder(8, [24, 40, 7], ACT_SILU)
    P = lib.tables.astype(np.float64) @ dec.W[0].astype(np.float64).T
    comps = all_compounds(lib)
    ids = np.array([c[0] for c in comps], dtype=np.uint64)
    h = oracle.heads(lib, dec, ids)
    for i, (_, t, idx) in enumerate(comps):
        z = dec.b[0].astype(np.float64) + P[idx[0]] + P[4 + idx[1]] + P[7 + idx[2]]
        a = z / (1 + np.exp(-z))
        ref = dec.W[1].astype(np.float64) @ a + dec.b[1]
        np.testing.assert_allclose(h[i], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_brute_force_subsets(k):
    lib = small_library(11, [2, 3], [2, 3, 3, 2, 2], 8)
    dec = g.make_decoder(11, [8, 16, 16, 4], ACT_SILU)
    # constraint levels from the data so that some compounds are infeasible
    comps = all_compounds(lib)
    H = np.array([torch_heads(lib, dec, t, idx) for _, t, idx in comps])
    q = Query(w=np.array([0.0, -1.0, 0.0, 0.5], np.float32),
              constraints=[Constraint(2, np.float32(np.quantile(H[:, 2], 0.2)), math.inf),
                           Constraint(3, -math.inf, np.float32(np.quantile(H[:, 3], 0.8)))], k=k)
    want, feas = brute_force(lib, dec, q)
    r = oracle.topk(lib, dec, q)
    assert r.n_feasible == len(feas)
    assert set(r.answer_ids.tolist()) == want
    # the objective values are those of the returned compounds
    obj = dict(feas)
    for cid, o in zip(r.answer_ids.tolist(), r.objective):
        assert abs(obj[cid] - o) <= 1e-12 * max(1.0, abs(o))


def test_sorted_sums_top1():
    """Unconstrained linear two-slot library: the best compound pairs the best
    synthon of each slot (objective separates into a_i + b_j)."""
    lib = small_library(13, [2], [40, 55], 8)
    dec = g.make_decoder(13, [8, 1], ACT_NONE)
    q = Query(w=np.array([1.0], np.float32), constraints=[], k=1)
    r = oracle.topk(lib, dec, q)
    a = lib.tables[:40].astype(np.float64) @ dec.W[0][0].astype(np.float64)
    b = lib.tables[40:].astype(np.float64) @ dec.W[0][0].astype(np.float64)
    assert r.ids[0] == int(np.argmax(a)) * 55 + int(np.argmax(b))
    assert abs(r.objective[0] - (a.max() + b.max() + dec.b[0][0])) < 1e-12


def test_k_at_least_n_returns_everything_sorted():
    lib = small_library(17, [2, 2], [3, 4, 2, 2], 8)
    dec = g.make_decoder(17, [8, 8, 3], ACT_RELU)
    q = Query(w=np.array([1.0, 0.0, 0.0], np.float32), constraints=[], k=1000)
    r = oracle.topk(lib, dec, q)
    n = oracle.num_compounds(lib)
    assert r.n_feasible == n and len(r.answer_ids) == n
    keys = list(zip((-r.objective).tolist(), r.ids.tolist()))
    assert keys == sorted(keys)
    assert sorted(r.ids.tolist()) == list(range(n))


def test_all_infeasible_returns_nothing():
    lib = small_library(19, [2], [10, 10], 8)
    dec = g.make_decoder(19, [8, 8, 3], ACT_RELU)
    q = Query(w=np.array([1.0, 0.0, 0.0], np.float32), constraints=[Constraint(1, 1e30, math.inf)], k=5)
    r = oracle.topk(lib, dec, q)
    assert r.n_feasible == 0 and len(r.ids) == 0
    ids, _ = oracle.topk_lex(lib, dec, q)
    assert len(ids) == 0


def test_ties_go_to_the_lower_id():
    """Duplicate synthon rows give exactly equal scores; the lower id ranks first."""
    lib = small_library(23, [2], [6, 5], 8)
    lib.tables[2] = lib.tables[0]  # synthons 0 and 2 of slot 0 are identical
    lib.tables[6 + 3] = lib.tables[6 + 1]  # synthons 1 and 3 of slot 1 are identical
    dec = g.make_decoder(23, [8, 16, 2], ACT_SILU)
    q = Query(w=np.array([1.0, 0.0], np.float32), constraints=[], k=30)
    r = oracle.topk(lib, dec, q, extra=0)
    o = r.objective
    for i in range(len(o) - 1):
        assert o[i] > o[i + 1] or (o[i] == o[i + 1] and r.ids[i] < r.ids[i + 1])
    # the four copies of compound (0, 1) have equal scores
    h = oracle.heads(lib, dec, np.array([0 * 5 + 1, 0 * 5 + 3, 2 * 5 + 1, 2 * 5 + 3], np.uint64))
    assert (h == h[0]).all()


def test_lexicographic_queue_equals_mask_and_sort():
    """Section 4.3's (violation, objective) queue, violators dropped at the end,
    gives the same answer as filtering then sorting."""
    lib = small_library(29, [2, 3], [12, 9, 5, 4, 6], 16)
    dec = g.make_decoder(29, [16, 32, 32, 5], ACT_SILU)
    sample = oracle.heads(lib, dec, np.arange(0, oracle.num_compounds(lib), 3, dtype=np.uint64))
    for k in (1, 10, 50, 400):
        for qi in range(3):
            cons = [Constraint(1, -math.inf, np.float32(np.quantile(sample[:, 1], 0.5 + 0.2 * qi))),
                    Constraint(3, np.float32(np.quantile(sample[:, 3], 0.1 * qi)), math.inf)]
            q = Query(w=np.array([0, 0, -1, 0, 0.25], np.float32), constraints=cons, k=k,
                      reactions=[1] if qi == 2 else None)
            r = oracle.topk(lib, dec, q)
            ids, o = oracle.topk_lex(lib, dec, q)
            assert ids.tolist() == r.answer_ids.tolist()


def test_permutation_invariance():
    """Reordering synthons inside a slot relabels compounds but keeps the multiset
    of (score, synthon identities); swapping the two slots of a reaction keeps
    every score (the combine is a sum)."""
    lib = small_library(31, [2], [20, 15], 8)
    dec = g.make_decoder(31, [8, 16, 3], ACT_SILU)
    q = Query(w=np.array([1.0, -0.5, 0.0], np.float32),
              constraints=[Constraint(2, -0.3, math.inf)], k=400)
    base = oracle.topk(lib, dec, q, extra=0)
    perm = np.array(g.uniform_f64(1, "perm", 15).argsort())
    lib2 = g.Library(lib.n_slots, lib.slot_sizes, lib.d, lib.tables.copy())
    lib2.tables[20:] = lib.tables[20:][perm]
    r2 = oracle.topk(lib2, dec, q, extra=0)
    def as_set(res, remap):
        out = []
        for cid, o in zip(res.ids.tolist(), res.objective.tolist()):
            i, j = divmod(cid, 15)
            out.append((round(o, 12), i, remap(j)))
        return sorted(out)
    assert as_set(base, lambda j: j) == as_set(r2, lambda j: int(perm[j]))
    # swap slots: reaction with slot sizes (15, 20) built from the swapped rows
    lib3 = g.Library(lib.n_slots, np.array([15, 20], np.uint32), lib.d,
                     np.concatenate([lib.tables[20:], lib.tables[:20]]))
    ids = np.arange(300, dtype=np.uint64)
    h1 = oracle.heads(lib, dec, ids)
    i, j = np.divmod(ids.astype(np.int64), 15)
    h3 = oracle.heads(lib3, dec, (j * 20 + i).astype(np.uint64))
    np.testing.assert_allclose(h1, h3, rtol=1e-13, atol=1e-13)


def test_reaction_subset_restricts_the_search():
    lib = small_library(37, [2, 2, 3], [5, 6, 7, 3, 2, 3, 4], 8)
    dec = g.make_decoder(37, [8, 8, 2], ACT_RELU)
    q = Query(w=np.array([1.0, 0.0], np.float32), constraints=[], k=1000, reactions=[0, 2])
    r = oracle.topk(lib, dec, q)
    n0, n1 = 30, 21
    assert r.n_feasible == n0 + 24
    assert all(cid < n0 or cid >= n0 + n1 for cid in r.ids.tolist())


def test_c0_boundary_margins():
    """The configured tiny case has score and threshold margins far above float32
    error, so an exact id-set comparison with a float32 engine is meaningful."""
    lib, dec, q = g.config_c0()
    r = oracle.topk(lib, dec, q, extra=1, near_tol=1e-3)
    assert r.n_feasible > q.k
    scale = float(np.abs(r.objective[:q.k]).max())
    assert r.gap_k > 1e-5 * scale
    assert r.min_slack_selected > 1e-5
    assert r.min_violation_near > 1e-5


def test_generator_native_matches_numpy():
    a = g.normal_f32(3, "tables", 50_000, 123, native=False)
    b = g.normal_f32(3, "tables", 50_000, 123, native=True)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    z = g.normal_f32(4, "check", 400_000)
    assert abs(float(z.mean())) < 0.01 and abs(float(z.std()) - 1) < 0.01


def _all_heads(lib, dec, q=None):
    """(id, t, idx, heads) of every compound (of q's reactions), forward pass in
    torch fp64, independent of the oracle's loops."""
    out = []
    for cid, t, idx in all_compounds(lib):
        if q is not None and q.reactions is not None and t not in q.reactions:
            continue
        out.append((cid, t, idx, torch_heads(lib, dec, t, idx)))
    return out


@pytest.mark.parametrize("k", [1, 7, 20, 60])
def test_margins_brute_force(k):
    """The margin report of orc_topk, recomputed by brute force: the smallest
    distance of a returned compound from its nearest bound, and the smallest
    worst-bound violation among infeasible compounds that are within near_tol of
    feasibility and score at least the (k+1)-th feasible objective."""
    lib = small_library(71, [2, 3], [6, 5, 3, 4, 2], 8)
    dec = g.make_decoder(71, [8, 16, 4], ACT_SILU)
    rows = _all_heads(lib, dec)
    H = np.array([r[3] for r in rows])
    q = Query(w=np.array([1.0, 0.0, -0.5, 0.0], np.float32),
              constraints=[Constraint(1, np.float32(np.quantile(H[:, 1], 0.3)), math.inf),
                           Constraint(3, np.float32(np.quantile(H[:, 3], 0.1)),
                                      np.float32(np.quantile(H[:, 3], 0.85)))], k=k)
    near_tol = 0.5
    feas, infeas = [], []
    for cid, _, _, h in rows:
        o = float(np.dot(q.w.astype(np.float64), h))
        viol = [max(float(c.lo) - h[c.head], h[c.head] - float(c.hi)) for c in q.constraints]
        (feas if max(viol) <= 0 else infeas).append((cid, o, h, max(viol)))
    feas.sort(key=lambda e: (-e[1], e[0]))
    top = feas[:k]
    slack = min(min(h[c.head] - float(c.lo), float(c.hi) - h[c.head]) for _, _, h, _ in top for c in q.constraints)
    cut = feas[k][1] if len(feas) > k else -math.inf
    near = [e for e in infeas if e[3] <= near_tol]
    near_cut = [e[3] for e in near if e[1] >= cut]
    r = oracle.topk(lib, dec, q, extra=1, near_tol=near_tol)
    assert r.n_feasible == len(feas)
    assert r.answer_ids.tolist() == [e[0] for e in top]
    assert r.n_near == len(near) > 0
    assert abs(r.min_slack_selected - slack) <= 1e-12 * max(1.0, abs(slack))
    want = min(near_cut) if near_cut else math.inf
    assert (r.min_violation_near == want) if math.isinf(want) else abs(r.min_violation_near - want) <= 1e-12
    if len(feas) > k:
        assert abs(r.gap_k - (feas[k - 1][1] - feas[k][1])) <= 1e-12
    else:  # every feasible compound is returned: no cut, every near compound counts
        assert math.isinf(r.gap_k) and abs(r.min_violation_near - min(e[3] for e in near)) <= 1e-12


def nonfinite_library():
    """Two-slot library with a linear decoder: slot-0 synthon 2 carries +Inf in a
    column every head reads with a positive weight (its compounds get +Inf heads
    and, with non-negative objective weights, a +Inf objective), slot-1 synthon 1
    carries a NaN (its compounds get NaN heads)."""
    lib = small_library(73, [2], [5, 4], 8)
    dec = g.make_decoder(73, [8, 3], ACT_NONE)
    dec.W[0][:, 3] = np.array([0.5, 0.3, 0.2], np.float32)
    lib.tables[2, 3] = np.inf
    lib.tables[5 + 1, 6] = np.nan
    return lib, dec


def test_nonfinite_compounds_are_never_returned():
    """A compound whose objective or any head is NaN or +-Inf is not a
    candidate: the answer is the finite compounds only, by (objective desc, id)."""
    lib, dec = nonfinite_library()
    q = Query(w=np.array([1.0, 0.5, 0.25], np.float32), constraints=[], k=100)
    rows = _all_heads(lib, dec)
    fin = [(cid, float(np.dot(q.w.astype(np.float64), h))) for cid, _, _, h in rows
           if np.all(np.isfinite(h)) and np.isfinite(np.dot(q.w.astype(np.float64), h))]
    fin.sort(key=lambda e: (-e[1], e[0]))
    assert len(fin) == 4 * 3
    # the +Inf compounds exist and would rank first if they were candidates
    o_all = {cid: float(np.dot(q.w.astype(np.float64), h)) for cid, _, _, h in rows}
    assert any(math.isinf(v) and v > 0 for v in o_all.values())
    r = oracle.topk(lib, dec, q)
    assert r.n_feasible == 12 and r.answer_ids.tolist() == [e[0] for e in fin]
    ids, _ = oracle.topk_lex(lib, dec, q)
    assert ids.tolist() == [e[0] for e in fin]
    # with a bound on the infinite head the same compounds stay out
    q2 = Query(w=q.w, constraints=[Constraint(0, -math.inf, math.inf)], k=100)
    assert oracle.topk(lib, dec, q2).answer_ids.tolist() == [e[0] for e in fin]


@pytest.mark.parametrize("k", [3, 25, 200])
def test_violation_ranked_fallback_brute_force(k):
    """The queue of Section 4.3 without the final removal: compounds ordered by
    (violation desc, objective desc, id asc), where the violation is minus the
    summed distances outside the bounds; with few feasible compounds the
    least-violating ones follow them."""
    lib = small_library(79, [2, 3], [5, 4, 3, 3, 2], 8)
    dec = g.make_decoder(79, [8, 12, 12, 4], ACT_SILU)
    rows = _all_heads(lib, dec)
    H = np.array([r[3] for r in rows])
    cons = [Constraint(0, np.float32(np.quantile(H[:, 0], 0.7)), math.inf),
            Constraint(2, -math.inf, np.float32(np.quantile(H[:, 2], 0.4)))]
    q = Query(w=np.array([0.0, 1.0, 0.0, -0.25], np.float32), constraints=cons, k=k)
    ent = []
    for cid, _, _, h in rows:
        c = -sum(max(0.0, float(x.lo) - h[x.head]) + max(0.0, h[x.head] - float(x.hi)) for x in cons)
        ent.append((c, float(np.dot(q.w.astype(np.float64), h)), cid))
    ent.sort(key=lambda e: (-e[0], -e[1], e[2]))
    want = ent[:k]
    ids, o, c = oracle.topk_lex(lib, dec, q, keep_violators=True, with_violation=True)
    assert ids.tolist() == [e[2] for e in want]
    np.testing.assert_allclose(c, [e[0] for e in want], rtol=0, atol=1e-12)
    n_feas = sum(1 for e in ent if e[0] == 0.0)
    assert 0 < n_feas < 200
    # its feasible head is the ordinary answer; violators only fill places the
    # feasible set cannot
    r = oracle.topk(lib, dec, q)
    m = min(k, n_feas)
    assert ids[:m].tolist() == r.answer_ids.tolist()
    assert np.all(c[:m] == 0.0) and np.all(c[m:] < 0.0)


# ----------------------------------------------------------------------------
# Associative embeddings (Section 4.2, eq. "assoc_embeds")
# ----------------------------------------------------------------------------
def test_assoc_worked_example():
    """A hand-worked case (tests/golden/assoc_worked_example.json): distinct,
    non-square key matrices per R-group, so a transposed key, a swapped slot or
    a dropped term changes the result."""
    ex = json.load(open(os.path.join(GOLDEN, "assoc_worked_example.json")))
    u = oracle.assoc_embeddings(ex["n_slots"], ex["slot_sizes"], np.array(ex["keys"], np.float32),
                                np.array(ex["values"], np.float32))
    assert np.array_equal(u, np.array(ex["expected"], np.float64))


def test_assoc_identity_scaling_and_permutation():
    """Identity keys return the values; doubling a key doubles its rows exactly;
    permuting the synthons of a slot permutes its rows; the map is linear in
    the values."""
    ns, ss = [2, 3], [4, 3, 2, 5, 3]
    rows, d = sum(ss), 6
    V = g.normal_f32(70, "assoc_v", rows * d).reshape(rows, d)
    eye = np.repeat(np.eye(d, dtype=np.float32)[None], len(ss), axis=0)
    assert np.array_equal(oracle.assoc_embeddings(ns, ss, eye, V), V.astype(np.float64))
    dU = 4
    K = g.normal_f32(71, "assoc_k", len(ss) * d * dU).reshape(len(ss), d, dU)
    V = g.normal_f32(72, "assoc_v2", rows * dU).reshape(rows, dU)
    u = oracle.assoc_embeddings(ns, ss, K, V)
    K2 = K.copy()
    K2[3] *= 2
    u2 = oracle.assoc_embeddings(ns, ss, K2, V)
    base = np.cumsum([0] + ss)
    r3 = slice(base[3], base[4])
    assert np.array_equal(u2[r3], 2 * u[r3])
    mask = np.ones(rows, bool)
    mask[r3] = False
    assert np.array_equal(u2[mask], u[mask])
    perm = np.array([2, 0, 4, 1, 3])
    Vp = V.copy()
    Vp[r3] = V[r3][perm]
    assert np.array_equal(oracle.assoc_embeddings(ns, ss, K, Vp)[r3], u[r3][perm])
    Va = g.normal_f32(73, "assoc_v3", rows * dU).reshape(rows, dU)
    lin = oracle.assoc_embeddings(ns, ss, K, (V.astype(np.float64) + Va).astype(np.float32))
    assert np.allclose(lin, u + oracle.assoc_embeddings(ns, ss, K, Va), rtol=1e-6, atol=1e-6)
