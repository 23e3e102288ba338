"""Decoder shapes beyond the benchmark one, in every precision: first hidden
widths 128/256/512, second hidden widths that are not multiples of 64 (the
BF16/FP8 kernel pads them with zero neurons), one hidden layer, 16 heads, and
the three activations. FP32 searches must return the oracle's exact id set;
BF16/FP8 heads are checked against the FP64 oracle directly (the search's
recall alone would not expose a wrong low-precision kernel: its error margin
is calibrated from that same kernel), and their searches for recall."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads.gen as g
from workloads.gen import ACT_NONE, ACT_RELU, ACT_SILU, Constraint, Query

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from gpu_helpers import device_objects, score_tol

CASES = [
    ("h128_h96_relu", [64, 128, 96, 7], ACT_RELU),
    ("h256_h160_silu", [128, 256, 160, 12], ACT_SILU),
    ("h512_h32_linear16", [256, 512, 32, 16], ACT_NONE),
    ("one_hidden_h256_silu", [64, 256, 9], ACT_SILU),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, dims, act = request.param
    seed = 100 + CASES.index(request.param)
    lib_h = g.make_library(seed, [2, 3, 2], [61, 45, 7, 6, 33, 29, 90], dims[0])
    dec_h = g.make_decoder(seed, dims, act)
    lib, dec, eng = device_objects(lib_h, dec_h)
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 7, dtype=np.uint64))
    H = dims[-1]
    w = np.zeros(H, np.float32)
    w[0], w[H - 1] = 1.0, -0.5
    cons = [Constraint(1, -math.inf, float(np.float32(np.quantile(sample[:, 1], 0.7)))),
            Constraint(H - 2, float(np.float32(np.quantile(sample[:, H - 2], 0.2))), math.inf)]
    q = Query(w=w, constraints=cons, k=100)
    return name, lib_h, dec_h, eng, q, sample


def test_fp32_exact(case):
    name, lib_h, dec_h, eng, q, sample = case
    print(f"case: {name} fp32", flush=True)
    r = eng.search(q, precision="fp32")
    ref = oracle.topk(lib_h, dec_h, q, extra=1, near_tol=1e-3)
    k = min(q.k, ref.n_feasible)
    print(f"[{name}] n_feasible={ref.n_feasible} gap_k={ref.gap_k:.3e}", flush=True)
    assert len(r.ids) == k
    assert set(r.ids.tolist()) == set(ref.answer_ids.tolist())
    h64 = oracle.heads(lib_h, dec_h, r.ids)
    o64 = h64 @ q.w.astype(np.float64)
    os_ = float(np.sqrt(np.mean((sample @ q.w.astype(np.float64)) ** 2)))
    assert np.all(np.abs(r.objective - o64) <= score_tol(o64, os_))


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_heads_and_recall(case, prec):
    name, lib_h, dec_h, eng, q, sample = case
    print(f"case: {name} {prec}", flush=True)
    ids = g.sample_ids(9, "shape_head_sample", lib_h.n_compounds, 2048)
    h64 = oracle.heads(lib_h, dec_h, ids)
    rms = np.sqrt(np.mean(h64 ** 2, axis=0))
    err = np.abs(eng.heads(ids, prec).astype(np.float64) - h64)
    err32 = np.abs(eng.heads(ids, "fp32").astype(np.float64) - h64)
    print(f"[{name} {prec}] mean |err| / rms: {np.array2string(err.mean(0) / rms, precision=4)}", flush=True)
    # BF16 keeps 8 significant bits of every activation, E4M3 4: the mean head
    # error stays well under 1 % (BF16) or 6 % (FP8) of the head's RMS
    assert np.all(err.mean(0) <= (0.01 if prec == "bf16" else 0.06) * rms)
    assert np.all(err32.max(0) <= 1e-5 * np.maximum(rms, 1.0))
    r = eng.search(q, precision=prec)
    ref = oracle.topk(lib_h, dec_h, q)
    k = min(q.k, ref.n_feasible)
    recall = len(set(r.ids.tolist()) & set(ref.answer_ids.tolist())) / max(k, 1)
    print(f"[{name} {prec}] recall={recall:.4f}", flush=True)
    assert recall >= 0.99
