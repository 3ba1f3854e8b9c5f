"""Build libcbfs.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcbfs.so")
SOURCES = ["cbfs_run.hip", "cbfs_kernels.hip", "cbfs_query.hip", "cbfs_pll.hip", "cbfs_graph.cpp"]
# measurement only (bench.py --gather-ceiling): not linked into libcbfs
PROBE_SOURCE = "probe_gather.hip"
PROBE_LIB = os.path.join(HERE, "libcbfs_probe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # never emit packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every source into ``paper_2410_17226_amd/libcbfs.so`` and the gather probe into
    ``libcbfs_probe.so`` (always rebuilds)."""
    tmp = LIB + ".tmp"
    objs = []
    procs = []
    probe_tmp = PROBE_LIB + ".tmp"
    probe_cmd = [HIPCC] + FLAGS + ["-x", "hip", os.path.join(CSRC, PROBE_SOURCE), "-o", probe_tmp]
    procs.append((PROBE_SOURCE, subprocess.Popen(probe_cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature and says so
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write("\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    os.replace(probe_tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
