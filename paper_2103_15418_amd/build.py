"""Builds liblpf.so (the HIP library behind include/lpf.h) for gfx950.

    python -m paper_2103_15418_amd.build        (or: python paper_2103_15418_amd/build.py)

Compiles every translation unit under csrc/ with hipcc and links them into
paper_2103_15418_amd/liblpf.so.  Packed-FP32 instructions are disabled for
all device code.
"""

from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblpf.so")
SOURCES = ["api.cpp", "serve.cpp", "ingest.hip", "filter.hip", "disk.hip", "catalog.hip", "flux.hip", "cnn.hip"]
ARCH = os.environ.get("LPF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int = 6) -> str:
    objs = []
    procs = []
    tmp = tempfile.mkdtemp(prefix="lpf_build_")
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(tmp, src + ".o")
        cmd = [HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
               "-I", INCLUDE, "-I", CSRC, *DEVICE_FLAGS, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the device-only feature; that warning is expected
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append(src)
            print(f"--- {src} failed:\n" + "\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print(f"--- {src}:\n" + "\n".join(lines))
    if failed:
        raise RuntimeError("HIP build failed: " + ", ".join(failed))
    tmp_lib = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs, "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
