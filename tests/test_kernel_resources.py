"""The fused enumeration kernels keep all state in registers: no scratch and no
spills in any instantiation (figures recorded by the build from the compiler's
resource-usage remarks), and every one fits two waves per SIMD."""
import os

import pytest

RES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2510_24380_amd", "_build", "kernel_resources.txt")


def _rows():
    if not os.path.exists(RES):
        pytest.skip("no build record (run the build first)")
    rows = []
    for line in open(RES):
        rows.append(dict(kv.split("=", 1) for kv in line.split()))
    return rows


def test_enum_kernels_use_no_scratch():
    rows = [r for r in _rows() if "k_enum" in r["kernel"]]
    assert len(rows) >= 100
    bad = [r["kernel"] for r in rows if int(r.get("scratch", 0)) or int(r.get("vgpr_spill", 0))]
    assert not bad, bad


def test_enum_kernels_two_waves_per_simd():
    rows = [r for r in _rows() if "k_enum" in r["kernel"]]
    assert all(int(r["occupancy"]) >= 2 for r in rows)
    assert all(int(r["vgpr"]) + int(r.get("agpr", 0)) <= 256 for r in rows)
