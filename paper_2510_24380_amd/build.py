"""Builds libapex.so (all HIP sources for gfx950) next to this file."""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libapex.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off (hardware notes)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(src: str, obj: str) -> None:
    cmd = ["hipcc"] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(verbose: bool = False) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objs = [os.path.join(out_dir, os.path.basename(s) + ".o") for s in srcs]
    workers = min(8, os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda so: _compile(*so), zip(srcs, objs)))
    tmp = SO + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, SO)
    probe_src = os.path.join(HERE, "probe", "mfma_probe.hip")
    probe_so = os.path.join(HERE, "probe", "libmfma_probe.so")
    subprocess.check_call(["hipcc"] + FLAGS + ["-shared", probe_src, "-o", probe_so])
    if verbose:
        print("built", SO, "and", probe_so)
    return SO


if __name__ == "__main__":
    build(verbose=True)
