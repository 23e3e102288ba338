"""Prints the one-wave MFMA issue table (cycles per MFMA, its vector work included)
from the issue probe: dependent-chain latency and the overlap of a wave's own
vector work with its MFMAs. Run on the GPU: python -m paper_2510_24380_amd.probe.issue"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def table(iters=10000):
    import torch
    lib = ctypes.CDLL(os.path.join(HERE, "libissue_probe.so"))
    lib.probe_issue.argtypes = [ctypes.c_int] * 5 + [ctypes.c_void_p, ctypes.c_void_p]
    out = torch.empty(64, dtype=torch.float32, device="cuda")
    cyc = torch.zeros(1, dtype=torch.int64, device="cuda")
    rows = []
    for fp8 in (0, 1):
        for nch in (1, 2, 4):
            cells = []
            for k, trans in ((0, 0), (4, 0), (8, 0), (2, 1), (4, 1)):
                rc = lib.probe_issue(fp8, nch, k, trans, iters, out.data_ptr(), cyc.data_ptr())
                if rc != 0:
                    raise RuntimeError(f"probe_issue failed ({rc})")
                cells.append(int(cyc.item()) / iters / nch)
            rows.append((fp8, nch, cells))
    return rows


def main():
    rows = table()
    print("| MFMA | chains | K = 0 | 4 FMAs | 8 FMAs | 2 exp2 | 4 exp2 |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for fp8, nch, cells in rows:
        name = "FP8 32x32x64 (scaled)" if fp8 else "BF16 32x32x16"
        print(f"| {name} | {nch} | " + " | ".join(f"{c:.1f}" for c in cells) + " |")


if __name__ == "__main__":
    main()
