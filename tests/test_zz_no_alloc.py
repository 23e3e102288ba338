"""apex_search_noalloc (the search whose scratch is the library's static device
array) against apex_search (the same search in a caller workspace), through the
C ABI: two calls in a row on one GPU, the second with a smaller input, each equal
to apex_search's answer entry for entry; the smaller one is also checked against
the FP64 oracle. A query whose workspace exceeds the static array is refused."""
import math

import numpy as np
import pytest
import torch

import workloads.gen as g
from workloads.gen import ACT_RELU, Constraint, Query

pytestmark = pytest.mark.gpu

from parity import check_fp32_exact, check_lowp

if torch.cuda.is_available():
    import paper_2510_24380_amd as apex
    from gpu_helpers import device_objects


# 624,000 compounds: enough for the warm start (eight times its 2^16 sample)
@pytest.fixture(scope="module")
def case():
    lib_h = g.make_library(97, [2, 3, 2], [500, 900, 30, 40, 20, 300, 500], 64)
    dec_h = g.make_decoder(97, [64, 128, 5], ACT_RELU)
    objs = device_objects(lib_h, dec_h)
    return lib_h, dec_h, objs


def _query(k, reactions=None):
    w = np.array([1.0, 0.0, -0.5, 0.0, 0.25], np.float32)
    cons = [Constraint(1, -math.inf, 0.5), Constraint(3, -0.75, math.inf)]
    return Query(w=w, constraints=cons, k=k, reactions=reactions)


def _same(a, b, label):
    assert np.array_equal(a.ids, b.ids), f"{label}: ids"
    assert np.array_equal(a.objective, b.objective), f"{label}: objectives"
    assert np.array_equal(a.heads, b.heads), f"{label}: heads"
    assert np.array_equal(a.reaction, b.reaction) and np.array_equal(a.synthon, b.synthon), f"{label}: decode"
    assert a.n_scored == b.n_scored and a.n_candidates == b.n_candidates, f"{label}: counters"


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_search_twice(case, prec):
    lib_h, dec_h, (lib, dec, eng) = case
    big, small = _query(300), _query(20, reactions=[1])
    for q, label in ((big, "whole library, k=300"), (small, "reaction 1, k=20")):
        print(f"case: noalloc {prec} {label}", flush=True)
        r_static = eng.search_noalloc(q, precision=prec)
        r_ws = eng.search(q, precision=prec)
        _same(r_static, r_ws, f"{prec} {label}")
        assert len(r_static.ids) == q.k
    if prec == "fp32":
        check_fp32_exact(lib_h, dec_h, small, r_static, "noalloc fp32 small")
    else:
        check_lowp(lib_h, dec_h, small, r_static, f"noalloc {prec} small")


def test_noalloc_refuses_oversized_query(case):
    lib_h, dec_h, (lib, dec, eng) = case
    q = _query(200_000)
    need = eng.query_workspace_size(q, "fp32")
    assert need > 64 << 20
    print(f"case: noalloc oversized ({need} bytes)", flush=True)
    with pytest.raises(apex.ApexError) as e:
        eng.search_noalloc(q, precision="fp32")
    assert e.value.status == -2 and "static" in e.value.message
