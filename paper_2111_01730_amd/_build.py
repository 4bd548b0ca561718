"""Compile the hodbf HIP library for gfx950 in-tree (``paper_2111_01730_amd/libhodbf.so``)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhodbf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result", f"-I{ROOT}/include"]
# no packed-FP32 instructions in generated device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST = ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-fopenmp"]


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    hip, cpp = sources()
    jobs = []
    objs = []
    for f in hip + cpp:
        obj = os.path.join(OUT_DIR, f + ".o")
        objs.append(obj)
        flags = COMMON + (DEVICE if f.endswith(".hip") else HOST)
        pre = ["-x", "c++"] if f.endswith(".cpp") else []
        cmd = [hipcc, "-c"] + pre + [os.path.join(CSRC, f), "-o", obj] + flags
        jobs.append((f, cmd))
    procs = []
    for f, cmd in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((f, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errors = []
    for f, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the device-only feature flag; that note is harmless
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            errors.append(f"{f}:\n{text}")
        elif verbose and text.strip():
            print(text)
    if errors:
        raise RuntimeError("hodbf build failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    link = [hipcc, "-shared", "-fPIC", "-fopenmp", "-o", tmp] + objs + [
        f"-L{ROCM}/lib",
        f"-Wl,-rpath,{ROCM}/lib", f"-Wl,-rpath,{ROCM}/llvm/lib",
    ]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("hodbf link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
