"""Build the HIP library libparspin.so for gfx950 (in-tree).

Every source is compiled with hipcc for gfx950 only, with packed-FP32
instructions disabled (-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libparspin.so")
SOURCES = ["kernels.hip", "calib.hip", "compile.cpp", "api.cpp", "batch.cpp", "server.cpp",
           "plan.cpp", "kt.cpp", "kt_engine.cpp", "tune.cpp"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include")]


def source_hash() -> str:
    """Hash of the library's sources and header: it heads saved tiling tables,
    which are valid only for the build they were timed with."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(HERE, "..", "include", "parspin.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    common = COMMON + [f'-DPS_LIB_HASH="{source_hash()}"']
    with tempfile.TemporaryDirectory(prefix="parspin_build_") as tmp:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = [] if src.endswith(".hip") else ["-x", "hip"]
            cmd = [HIPCC, *common, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
            if len([p for _, p in procs if p.poll() is None]) >= jobs:
                procs[0][1].wait()
        for src, p in procs:
            out, _ = p.communicate()
            text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                             if "not a recognized feature" not in l)
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed for {src}:\n{text}")
            if verbose and text.strip():
                print(text, file=sys.stderr)
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
