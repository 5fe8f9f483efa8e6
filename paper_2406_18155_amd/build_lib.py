"""Build libscprop.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libscprop.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-ffp-contract=fast",
         "-mllvm", "-simplifycfg-sink-common=false"]


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    objs = []
    procs = []
    for src in srcs:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        log = obj + ".log"
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
        # compiler output goes to a file (a pipe could fill up and block the child)
        with open(log, "w") as fh:
            procs.append((src, log, subprocess.Popen(cmd, stdout=fh, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, _, p in procs) >= jobs:
            time.sleep(0.2)
    failed = False
    for src, log, p in procs:
        p.wait()
        out = open(log, errors="replace").read()
        if p.returncode != 0 or verbose:
            sys.stderr.write(out)
        if p.returncode != 0:
            sys.stderr.write(f"compile failed: {src}\n")
            failed = True
    if failed:
        raise RuntimeError("libscprop build failed")
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
