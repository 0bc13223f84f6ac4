"""Build of the HIP library (gfx950) in-tree: paper_2407_12399_amd/libtopsimp.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtopsimp.so")
SOURCES = ["sort.hip", "persistence.hip", "solver.hip", "unet.hip", "api.cpp"]
HEADERS = ["internal.h", "persistence.h", "solver.h", "unet.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("TS_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-ffp-contract=off", "-Wall",
          "-Wno-unused-result", f"-I{os.path.join(HERE, '..', 'include')}"]
# no packed FP32 instructions in device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _obj(src):
    return os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source (always) and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    for src in SOURCES:
        cmd = [HIPCC] + COMMON
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + DEVICE
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", _obj(src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[0][1].wait() if procs[0][1].poll() is None else None
            for _, p in procs:
                if p.poll() is None:
                    p.wait()
                    break
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(f"--- {src} ---\n{text}")
        elif verbose and text.strip():
            print(text)
    if failed:
        raise RuntimeError("HIP build failed:\n" + "\n".join(failed))
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + [_obj(s) for s in SOURCES]
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
