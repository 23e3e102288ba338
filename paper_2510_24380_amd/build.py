"""Builds libapex.so (all HIP sources for gfx950) next to this file."""
import concurrent.futures
import glob
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libapex.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off: some of their forms have returned wrong
         # results on gfx950 without any error
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


RESOURCES = os.path.join(HERE, "_build", "kernel_resources.txt")
_FIELDS = {"VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
           "Occupancy [waves/SIMD]": "occupancy", "VGPRs Spill": "vgpr_spill", "LDS Size [bytes/block]": "lds"}


def _resources(text: str) -> list:
    """Per-kernel register, scratch and occupancy figures from the compiler's
    resource-usage remarks."""
    rows, cur = [], None
    for line in text.splitlines():
        m = re.search(r"remark:\s+(.*?)\s*\[-Rpass-analysis=kernel-resource-usage\]", line)
        if not m:
            continue
        body = m.group(1)
        if body.startswith("Function Name:"):
            cur = {"kernel": body.split(":", 1)[1].strip()}
            rows.append(cur)
        elif cur is not None and ":" in body:
            k, v = body.rsplit(":", 1)
            if k.strip() in _FIELDS:
                cur[_FIELDS[k.strip()]] = int(v.strip())
    return rows


def _compile(src: str, obj: str) -> list:
    cmd = ["hipcc"] + FLAGS + ["-c", src, "-o", obj]
    if os.path.basename(src).startswith("enum_"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return _resources(r.stderr)


def build(verbose: bool = False) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objs = [os.path.join(out_dir, os.path.basename(s) + ".o") for s in srcs]
    workers = min(8, os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        usage = [row for rows in ex.map(lambda so: _compile(*so), zip(srcs, objs)) for row in rows]
    # The fused kernels must keep everything in registers: scratch traffic in
    # them costs more than any other inefficiency.
    with open(RESOURCES, "w") as f:
        for row in sorted(usage, key=lambda r: r["kernel"]):
            f.write(" ".join(f"{k}={row[k]}" for k in ["kernel"] + [c for c in _FIELDS.values() if c in row]) + "\n")
    bad = [row["kernel"] for row in usage if row.get("scratch", 0) > 32 or row.get("vgpr_spill", 0) > 8]
    if bad:
        sys.stderr.write(f"warning: {len(bad)} enumeration kernels spill beyond a few values: {bad[:4]}\n")
    tmp = SO + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, SO)
    probe_src = os.path.join(HERE, "probe", "mfma_probe.hip")
    probe_so = os.path.join(HERE, "probe", "libmfma_probe.so")
    subprocess.check_call(["hipcc"] + FLAGS + ["-shared", probe_src, "-o", probe_so])
    # issue-rate probe: accumulators in VGPRs, as the fused kernels keep them
    issue_src = os.path.join(HERE, "probe", "issue_probe.hip")
    issue_so = os.path.join(HERE, "probe", "libissue_probe.so")
    subprocess.check_call(["hipcc"] + FLAGS + ["-mllvm", "-amdgpu-mfma-vgpr-form=1", "-shared", issue_src, "-o", issue_so])
    if verbose:
        print("built", SO, "and", probe_so)
    return SO


if __name__ == "__main__":
    build(verbose=True)
