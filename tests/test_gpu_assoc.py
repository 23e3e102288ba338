"""Associative embeddings u_{r,s} = K_r v_s (Section 4.2, eq. "assoc_embeds")
computed by the library's grouped FP32 MFMA GEMM, through the C ABI, against
the FP64 oracle (pinned by a hand-worked case, identity keys, scaling,
permutation and linearity): ragged R-groups (1 to 200 synthons, row tiles of 16
with ragged tails), output widths below, at and above one 128-column pass, and
value widths that are not multiples of 4. The tables it writes then feed a
search that is exact against the oracle on the same tables."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads.gen as g
from workloads.gen import ACT_NONE, Constraint, Query

pytestmark = pytest.mark.gpu

from parity import check_fp32_exact

if torch.cuda.is_available():
    import paper_2510_24380_amd as apex

N_SLOTS = [2, 3, 2, 2]
SIZES = [37, 5, 1, 16, 17, 200, 33, 64, 90]


@pytest.mark.parametrize("d,dU", [(64, 64), (200, 30), (128, 7), (256, 256)])
def test_assoc_embeddings_exact(d, dU):
    keys, values = g.make_factorizer(80 + d + dU, SIZES, d, dU)
    rows = sum(SIZES)
    dev = torch.device("cuda:0")
    out = torch.full((rows, d), float("nan"), dtype=torch.float32, device=dev)
    lib = apex.Library(N_SLOTS, SIZES, out)
    print(f"case: assoc d={d} dU={dU}", flush=True)
    lib.assoc_embeddings(torch.from_numpy(keys).to(dev), torch.from_numpy(values).to(dev))
    torch.cuda.synchronize()
    u = out.cpu().numpy().astype(np.float64)
    u64 = oracle.assoc_embeddings(N_SLOTS, SIZES, keys, values)
    scale = float(np.sqrt(np.mean(u64 ** 2)))
    err = np.abs(u - u64)
    print(f"[assoc d={d} dU={dU}] max err {err.max():.3e} (scale {scale:.3e})", flush=True)
    assert np.all(np.isfinite(u))
    assert np.all(err <= 1e-5 * np.maximum(np.abs(u64), scale))


def test_assoc_tables_feed_the_search():
    """The GPU-computed tables as a linear-probe library: search exact against
    the oracle on the same tables."""
    d, dU, H = 64, 64, 28
    keys, values = g.make_factorizer(91, SIZES, d, dU)
    dev = torch.device("cuda:0")
    out = torch.empty((sum(SIZES), d), dtype=torch.float32, device=dev)
    lib = apex.Library(N_SLOTS, SIZES, out)
    lib.assoc_embeddings(torch.from_numpy(keys).to(dev), torch.from_numpy(values).to(dev))
    torch.cuda.synchronize()
    lib_h = g.Library(np.array(N_SLOTS, np.uint32), np.array(SIZES, np.uint32), d, out.cpu().numpy())
    dec_h = g.make_decoder(91, [d, H], ACT_NONE)
    dec = apex.Decoder(dec_h.dims, "none", [torch.from_numpy(w).to(dev) for w in dec_h.W],
                       [torch.from_numpy(b).to(dev) for b in dec_h.b])
    eng = apex.Engine(lib, dec, precisions=("fp32",))
    sample = oracle.heads(lib_h, dec_h, np.arange(0, lib_h.n_compounds, 3, dtype=np.uint64))
    w = np.zeros(H, np.float32)
    w[4] = -1.0
    q = Query(w=w, constraints=[Constraint(9, -math.inf, float(np.float32(np.quantile(sample[:, 9], 0.7))))], k=300)
    print("case: assoc tables -> search", flush=True)
    check_fp32_exact(lib_h, dec_h, q, eng.search(q), "assoc tables")


def test_assoc_validation():
    dev = torch.device("cuda:0")
    out = torch.empty((sum(SIZES), 64), dtype=torch.float32, device=dev)
    lib = apex.Library(N_SLOTS, SIZES, out)
    keys = torch.zeros((len(SIZES), 64, 300), dtype=torch.float32, device=dev)
    values = torch.zeros((sum(SIZES), 300), dtype=torch.float32, device=dev)
    with pytest.raises(apex.ApexError) as e:
        lib.assoc_embeddings(keys, values)
    assert e.value.status == -4  # dU above the supported 256
