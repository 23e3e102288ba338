"""Builds device objects of the HIP library from the seeded workload containers."""
import numpy as np
import torch

import paper_2510_24380_amd as apex
from workloads.gen import ACT_NONE, ACT_RELU, ACT_SILU

ACT_NAME = {ACT_NONE: "none", ACT_RELU: "relu", ACT_SILU: "silu"}


def device_objects(lib_h, dec_h, precisions=("fp32", "bf16", "fp8")):
    dev = torch.device("cuda:0")
    tables = torch.from_numpy(np.ascontiguousarray(lib_h.tables)).to(dev)
    lib = apex.Library(lib_h.n_slots, lib_h.slot_sizes, tables)
    dec = apex.Decoder(dec_h.dims, ACT_NAME[dec_h.act], [torch.from_numpy(w).to(dev) for w in dec_h.W],
                       [torch.from_numpy(b).to(dev) for b in dec_h.b])
    eng = apex.Engine(lib, dec, precisions=precisions)
    return lib, dec, eng


def score_tol(o64, scale):
    """|o_gpu - o_64| <= 1e-5 * max(|o_64|, scale)."""
    return 1e-5 * np.maximum(np.abs(o64), scale)
