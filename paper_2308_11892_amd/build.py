"""Build the HIP library libcptr.so in-tree for gfx950.

Host setup code is plain C++ built with FP contraction off; the API layer and
the kernels are built with hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libcptr.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = "/opt/rocm/bin/hipcc"
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
NO_PK = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def _write_build_info():
    """Revision of the sources the library was built from (read by the
    benchmark on machines without the git metadata)."""
    import hashlib
    import json
    info = {"kernels_hip_sha256": hashlib.sha256(open(os.path.join(CSRC, "kernels.hip"), "rb").read()).hexdigest()}
    try:
        sha = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True, text=True)
        dirty = subprocess.run(["git", "status", "--porcelain", "--untracked-files=no"], cwd=ROOT,
                               capture_output=True, text=True)
        if sha.returncode == 0:
            info["git_sha"] = sha.stdout.strip()
            info["git_dirty"] = bool(dirty.stdout.strip())
    except OSError:
        pass
    with open(os.path.join(HERE, "build_info.json"), "w") as f:
        json.dump(info, f)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    host = os.path.join(BUILD, "host_setup.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra",
          "-Wno-unused-parameter", f"-I{INC}", "-c", os.path.join(CSRC, "host_setup.cpp"),
          "-o", host])
    objs.append(host)
    for src in ("cptr_api.cpp", "cptr_serve.cpp", "kernels.hip"):
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        _run([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              "-ffp-contract=fast", *NO_PK, f"-I{INC}", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, OUT)
    _write_build_info()
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
